// Learned preconditioner z = r / diag(K) + N(r) for K = I + dt A with
// N = B^T diag(g2) B, B = C2 diag(g1) C1 (symmetric positive semi-definite):
// features, gate net, the convolution stack on r, its backward pass, the
// energy loss and Adam -- everything the network needs to be trained and
// applied on the GPU.  These are FP32 kernels (one thread per grid point,
// uniform weight reads); the 2D inference path used inside flexible CG has
// a fused BF16 MFMA kernel in cnn_mfma.hip.
//
// N runs as a plain four-layer gated stack: the gate net writes expanded
// gates [g1, g2, g1, 1] and adlbr_net_gates expands the weights to
// [W1, W2, flip(W2)^T, flip(W1)^T] (the correlation adjoint is the
// correlation with channel-transposed, spatially flipped taps).  The
// backward pass runs on the expanded stack and folds the gradients of tied
// weights and repeated gates back onto the parameters.
//
// Layout: activations are [channels][N] FP32 planes; convolutions are 3^d
// taps with zero padding outside the grid; tap t = ((tz*3)+ty)*3+tx over
// offsets -1, 0, +1.
#include "common.h"

namespace adlbr {

int apply_K(const adlbr_operator *op, const void *u, void *out, double dt, hipStream_t s);
int net_apply_mfma(const adlbr_net *net, const adlbr_operator *op, const float *r, float *z,
                   const float *rp, double *part, const CgState *st, hipStream_t s);
int net_mfma_blocks(int nx, int ny);
int net_pack_mfma(const adlbr_net *net, hipStream_t s);
int net_pack_mfma3d(const adlbr_net *net, hipStream_t s);
int net_apply_mfma3d(const adlbr_net *net, const adlbr_operator *op, const float *r, float *z,
                     const float *rp, double *part, const CgState *st, hipStream_t s);
long long net3d_tiles(const GridInfo &g);

namespace {

constexpr int kBS = 256;

struct NetDims {
    int dim, W, H, nf, G, GX, T;
    // parameter offsets; expanded layer offsets (net->layers)
    size_t oWA, obA, oWB, obB, oW1, oW2, count;
    size_t l1, l2, l3, l4, lcount;
};

NetDims net_dims(int dim, int W, int H) {
    NetDims d;
    d.dim = dim;
    d.W = W;
    d.H = H;
    d.T = dim == 2 ? 9 : 27;
    d.nf = dim == 2 ? 7 : 13;
    d.G = 2 * W;       // gate-net outputs g1, g2
    d.GX = 3 * W + 1;  // expanded gates of the four-layer stack
    size_t o = 0;
    d.oWA = o; o += (size_t)H * d.nf * d.T;
    d.obA = o; o += H;
    d.oWB = o; o += (size_t)d.G * H;
    d.obB = o; o += d.G;
    d.oW1 = o; o += (size_t)W * d.T;
    d.oW2 = o; o += (size_t)W * W * d.T;
    d.count = o;
    o = 0;
    d.l1 = o; o += (size_t)W * d.T;
    d.l2 = o; o += (size_t)W * W * d.T;
    d.l3 = o; o += (size_t)W * W * d.T;
    d.l4 = o; o += (size_t)W * d.T;
    d.lcount = o;
    return d;
}

int check_net(const adlbr_operator *op, const adlbr_net *net, NetDims *d) {
    if (!op || !net || !net->params || !net->layers) {
        set_error("net: null argument (params and layers are required)");
        return ADLBR_E_INVALID;
    }
    const GridInfo &g = operator_grid(op);
    if (net->dim != g.dim || net->width != 16 || net->hidden != 16 ||
        net->nfeat != (g.dim == 2 ? 7 : 13)) {
        set_error("net: need dim = grid dim, width = hidden = 16, nfeat = %d", g.dim == 2 ? 7 : 13);
        return ADLBR_E_UNSUPPORTED;
    }
    *d = net_dims(g.dim, net->width, net->hidden);
    return ADLBR_OK;
}

struct Pt {
    int x, y, z;
};

__device__ __forceinline__ Pt coord_of(long long i, const GridInfo &g) {
    Pt p;
    p.x = (int)(i % g.nx);
    const long long r = i / g.nx;
    p.y = (int)(r % g.ny);
    p.z = (int)(r / g.ny);
    return p;
}

// neighbour of p at tap t (returns -1 outside the grid)
template <int DIM>
__device__ __forceinline__ long long tap_nb(const Pt &p, long long i, int t, const GridInfo &g) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
    const int x = p.x + dx, y = p.y + dy, z = p.z + dz;
    if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || z < 0 || z >= g.nz) return -1;
    return i + dx + (long long)g.nx * (dy + (long long)g.ny * dz);
}

// ------------------------------------------------------------- features --
template <int DIM, typename TD>
__global__ void k_features(GridInfo g, const TD *diag, const float *w, const void *sbv, int wide,
                           double dt, float *F) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    const long long N = g.N;
    if (i >= N) return;
    constexpr int S = DIM == 2 ? 3 : 6;
    const double kd = 1.0 + dt * (double)diag[i];
    F[i] = (float)(1.0 / kd);
    double wq[S];
    for (int q = 0; q < S; ++q) {
        wq[q] = (double)w[widx<S>(q, i, N)];
        F[(1 + q) * N + i] = (float)(dt * wq[q] / kd);
    }
    // slots from the compact superbase form
    int o[6][3];
    if (DIM == 2) {
        int e0, e1, f0, f1;
        if (wide) {
            const short4 v = ((const short4 *)sbv)[i];
            e0 = v.x; e1 = v.y; f0 = v.z; f1 = v.w;
        } else {
            const char4 v = ((const char4 *)sbv)[i];
            e0 = v.x; e1 = v.y; f0 = v.z; f1 = v.w;
        }
        o[0][0] = e0; o[0][1] = e1; o[1][0] = f0; o[1][1] = f1;
        o[2][0] = -e0 - f0; o[2][1] = -e1 - f1;
    } else {
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c)
                o[q][c] = wide ? ((const int16_t *)sbv)[12 * i + 3 * q + c]
                               : ((const int8_t *)sbv)[12 * i + 3 * q + c];
        for (int c = 0; c < 3; ++c) {
            o[3][c] = -(o[0][c] + o[1][c]);
            o[4][c] = o[0][c] - o[2][c];
            o[5][c] = o[1][c] + o[2][c];
        }
    }
    if (DIM == 2) {
        double xx = 0, xy = 0, yy = 0;
        for (int q = 0; q < 3; ++q) {
            xx += 2 * wq[q] * o[q][0] * o[q][0];
            xy += 2 * wq[q] * o[q][0] * o[q][1];
            yy += 2 * wq[q] * o[q][1] * o[q][1];
        }
        double tr = xx + yy;
        tr = tr > 0 ? tr : 1.0;
        F[(1 + S) * N + i] = (float)(xx / tr);
        F[(2 + S) * N + i] = (float)(xy / tr);
        F[(3 + S) * N + i] = (float)(yy / tr);
    } else {
        const int pr[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
        double Dc[6];
        for (int k = 0; k < 6; ++k) {
            Dc[k] = 0.0;
            for (int q = 0; q < 6; ++q) Dc[k] += 2 * wq[q] * o[q][pr[k][0]] * o[q][pr[k][1]];
        }
        double tr = Dc[0] + Dc[3] + Dc[5];
        tr = tr > 0 ? tr : 1.0;
        for (int k = 0; k < 6; ++k) F[(1 + S + k) * N + i] = (float)(Dc[k] / tr);
    }
}

// ------------------------------------------------------- convolutions --
// out[co] = epi(sum_{t, ci} W[co][ci][t] * in_ci(p + off_t) (+ bias[co]))
// with in_ci = in[ci] * (in_gate ? in_gate[ci] : 1); epilogue: keep the
// pre-activation in `pre` (if given), multiply by gate[co] (if given),
// ReLU (if relu).
template <int DIM, int CIN, int COUT>
__global__ __launch_bounds__(kBS) void k_conv(GridInfo g, const float *__restrict__ in,
                                              const float *__restrict__ in_gate,
                                              const float *__restrict__ W,
                                              const float *__restrict__ bias,
                                              float *__restrict__ out, float *__restrict__ pre,
                                              const float *__restrict__ gate, int relu) {
    constexpr int T = DIM == 2 ? 9 : 27;
    const float *sw = W;  // uniform addresses: read through the scalar cache
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    const long long N = g.N;
    if (i >= N) return;
    const Pt p = coord_of(i, g);
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = bias ? bias[co] : 0.f;
    for (int t = 0; t < T; ++t) {
        const long long q = tap_nb<DIM>(p, i, t, g);
        if (q < 0) continue;
#pragma unroll 4
        for (int ci = 0; ci < CIN; ++ci) {
            float x = in[ci * N + q];
            if (in_gate) x *= in_gate[ci * N + q];
#pragma unroll
            for (int co = 0; co < COUT; ++co) acc[co] += sw[(co * CIN + ci) * T + t] * x;
        }
    }
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
        float v = acc[co];
        if (pre) pre[co * N + i] = v;
        if (gate) v *= gate[co * N + i];
        if (relu) v = fmaxf(v, 0.f);
        out[co * N + i] = v;
    }
}

// Gate layer B (1x1) + sigmoid: g[k] = 1 / (1 + exp(-(WB[k] . relu(h) + bB[k]))),
// k < 2W, written expanded for the four-layer stack: Gout = [g1, g2, g1, 1]
// ([3W+1][N]); G8 holds g1, g2 per point as 8-bit fixed point round(255 g)
// ([N][2W]) for the inference kernel.
template <int H, int W>
__global__ __launch_bounds__(kBS) void k_gate_b(long long N, const float *__restrict__ h,
                                                const float *__restrict__ WB,
                                                const float *__restrict__ bB, float *__restrict__ Gout,
                                                uint8_t *__restrict__ G8) {
    constexpr int GX = 3 * W + 1;
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i >= N) return;
    float hr[H];
#pragma unroll
    for (int c = 0; c < H; ++c) hr[c] = fmaxf(h[c * N + i], 0.f);
    for (int k = 0; k < 2 * W; ++k) {
        float a = bB[k];
#pragma unroll
        for (int c = 0; c < H; ++c) a += WB[k * H + c] * hr[c];
        const float gv = 1.f / (1.f + expf(-a));
        Gout[k * N + i] = gv;
        if (G8) G8[i * 2 * W + k] = (uint8_t)__float2int_rn(gv * 255.f);
        if (k < W) Gout[(2 * W + k) * N + i] = gv;
    }
    Gout[(GX - 1) * N + i] = 1.f;
}

// Expanded layer weights: L1 = W1, L2 = W2, L3[o][i][t] = W2[i][o][T-1-t],
// L4[0][i][t] = W1[i][0][T-1-t].
__global__ void k_expand_weights(const float *__restrict__ W1, const float *__restrict__ W2,
                                 float *__restrict__ L, int W, int T, size_t l2, size_t l3,
                                 size_t l4) {
    const int n1 = W * T, n2 = W * W * T;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += gridDim.x * blockDim.x) {
        const int t = e % T, io = e / T, i = io % W, o = io / W;  // e = (o * W + i) * T + t
        L[l2 + e] = W2[e];
        L[l3 + e] = W2[(i * W + o) * T + (T - 1 - t)];
        if (e < n1) {
            const int tt = e % T, c = e / T;  // e = c * T + t
            L[e] = W1[e];
            L[l4 + e] = W1[c * T + (T - 1 - tt)];
        }
    }
}

// Fold the expanded-stack gradients onto the tied parameters:
// gW1 += gL1 + flip(gL4), gW2 += gL2 + flip(gL3)^T.
__global__ void k_fold_weight_grads(const float *__restrict__ gL, float *__restrict__ gW1,
                                    float *__restrict__ gW2, int W, int T, size_t l2, size_t l3,
                                    size_t l4) {
    const int n1 = W * T, n2 = W * W * T;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += gridDim.x * blockDim.x) {
        const int t = e % T, io = e / T, i = io % W, o = io / W;  // W2 index (o, i, t)
        gW2[e] += gL[l2 + e] + gL[l3 + (i * W + o) * T + (T - 1 - t)];
        if (e < n1) {
            const int tt = e % T, c = e / T;
            gW1[e] += gL[e] + gL[l4 + c * T + (T - 1 - tt)];
        }
    }
}

// Fold the expanded gate gradients [3W+1][N] onto g1, g2 ([2W][N]):
// dg1 = dG[0:W] + dG[2W:3W], dg2 = dG[W:2W]; the constant last gate has none.
__global__ void k_fold_gate_grads(long long N, int W, const float *__restrict__ gx,
                                  float *__restrict__ gg) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i >= N) return;
    for (int k = 0; k < W; ++k) {
        gg[k * N + i] = gx[k * N + i] + gx[(2 * W + k) * N + i];
        gg[(W + k) * N + i] = gx[(W + k) * N + i];
    }
}

__global__ void k_fill_f32(float *p, long long n, float v) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i < n) p[i] = v;
}

// z = r * F0 + out   (F0 = 1 / diag K)
__global__ void k_precond_out(long long N, const float *r, const float *F0, const float *o,
                              float *z) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i < N) z[i] = r[i] * F0[i] + o[i];
}

// ------------------------------------------------------------ backward --
// ga = g * gate; ggate += g * pre   (per channel plane)
__global__ void k_gate_grad(long long n, const float *g, const float *gate, const float *pre,
                            float *ga, float *ggate) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    const float gv = g[i];
    ga[i] = gv * gate[i];
    ggate[i] += gv * pre[i];
}

// gin[ci](p) = sum_{t, co} W[co][ci][t] ga[co](p - off_t)  (transposed conv)
template <int DIM, int CIN, int COUT>
__global__ __launch_bounds__(kBS) void k_conv_bwd_data(GridInfo g, const float *__restrict__ ga,
                                                       const float *__restrict__ W,
                                                       float *__restrict__ gin) {
    constexpr int T = DIM == 2 ? 9 : 27;
    const float *sw = W;
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    const long long N = g.N;
    if (i >= N) return;
    const Pt p = coord_of(i, g);
    float acc[CIN];
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.f;
    for (int t = 0; t < T; ++t) {
        const long long q = tap_nb<DIM>(p, i, T - 1 - t, g);  // p - off_t
        if (q < 0) continue;
        for (int co = 0; co < COUT; ++co) {
            const float y = ga[co * N + q];
#pragma unroll
            for (int ci = 0; ci < CIN; ++ci) acc[ci] += sw[(co * CIN + ci) * T + t] * y;
        }
    }
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) gin[ci * N + i] = acc[ci];
}

// Weight gradient dW[co][ci][t] = sum_p ga[co](p) x_ci(p + off_t), with
// x_ci = in[ci] (* in_gate[ci]) (ReLU'd if relu_in), and the bias gradient
// db[co] = sum_p ga[co](p).  Each block walks a set of 256-point chunks and
// writes partials[block][COUT*CIN*T + COUT]; k_reduce_partials finishes.
template <int DIM, int CIN, int COUT, int PPT>
__global__ __launch_bounds__(kBS) void k_conv_bwd_w(GridInfo g, const float *__restrict__ in,
                                                    const float *__restrict__ in_gate, int relu_in,
                                                    const float *__restrict__ ga,
                                                    float *__restrict__ partials, int taps) {
    constexpr int TM = DIM == 2 ? 9 : 27;
    constexpr int C = 128;  // points per chunk
    const int T = taps;     // 1 for a 1x1 layer
    __shared__ float sg[COUT * C];
    __shared__ float sx[C * CIN];
    const long long N = g.N;
    float acc[PPT][TM];
    float accb = 0.f;
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
        for (int t = 0; t < TM; ++t) acc[k][t] = 0.f;
    const long long nchunk = (N + C - 1) / C;
    for (long long c = blockIdx.x; c < nchunk; c += gridDim.x) {
        __syncthreads();
        for (int e = threadIdx.x; e < COUT * C; e += kBS) {
            const int co = e / C, j = e % C;
            const long long i = c * C + j;
            sg[e] = i < N ? ga[co * N + i] : 0.f;
        }
        for (int t = 0; t < T; ++t) {
            const int tt = T == 1 ? (DIM == 2 ? 4 : 13) : t;  // centre tap for 1x1
            __syncthreads();
            for (int e = threadIdx.x; e < C * CIN; e += kBS) {
                const int j = e / CIN, ci = e % CIN;
                const long long i = c * C + j;
                float x = 0.f;
                if (i < N) {
                    const long long q = tap_nb<DIM>(coord_of(i, g), i, tt, g);
                    if (q >= 0) {
                        x = in[ci * N + q];
                        if (in_gate) x *= in_gate[ci * N + q];
                        if (relu_in) x = fmaxf(x, 0.f);
                    }
                }
                sx[e] = x;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int pair = threadIdx.x + k * kBS;
                if (pair < COUT * CIN) {
                    const int co = pair / CIN, ci = pair % CIN;
                    float s = 0.f;
                    for (int j = 0; j < C; ++j) s += sg[co * C + j] * sx[j * CIN + ci];
#pragma unroll
                    for (int tq = 0; tq < TM; ++tq)
                        if (tq == t) acc[k][tq] += s;
                }
            }
        }
        if ((int)threadIdx.x < COUT) {  // bias: sum of ga over the chunk
            float s = 0.f;
            for (int j = 0; j < C; ++j) s += sg[threadIdx.x * C + j];
            accb += s;
        }
    }
    const int stride = COUT * CIN * T + COUT;
    float *outp = partials + (long long)blockIdx.x * stride;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pair = threadIdx.x + k * kBS;
        if (pair < COUT * CIN)
            for (int t = 0; t < T; ++t) outp[pair * T + t] = acc[k][t];
    }
    if ((int)threadIdx.x < COUT) outp[COUT * CIN * T + threadIdx.x] = accb;
}

// 2D weight gradient on the matrix cores: the same sums as k_conv_bwd_w for
// 3x3 layers, dW[co][ci][t] = sum_p ga[co](p) x_ci(p + off_t), as GEMMs
// D_t[co][ci] += A[co][4 points] B_t[4 points][ci] with
// v_mfma_f32_16x16x4f32 (FP32 operands and accumulation).  Each block
// walks 16x16 tiles of points: ga on the tile and x on the tile plus a
// one-point halo (0 outside the grid) are staged in LDS, then every wave
// takes a quarter of the tile's 64 four-point steps for all 9 taps.  The
// four waves' results are summed in LDS in a fixed order and written as
// this block's partials (same layout as k_conv_bwd_w).
typedef float f32x4v __attribute__((ext_vector_type(4)));
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w2d_mfma(GridInfo g, const float *__restrict__ in,
                                                           const float *__restrict__ in_gate,
                                                           int relu_in,
                                                           const float *__restrict__ ga,
                                                           float *__restrict__ partials) {
    constexpr int TW = 16, HW = TW + 2, T = 9;
    __shared__ float sx[CIN * HW * HW];
    __shared__ float sg[COUT * TW * TW];
    __shared__ float red[4][COUT * CIN * T + COUT];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = g.nx, ny = g.ny;
    const int ntx = (nx + TW - 1) / TW, nty = (ny + TW - 1) / TW;
    const int i = lane & 15, kk = lane >> 4;  // A row (co) / B column (ci), k
    f32x4v acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = f32x4v{0.f, 0.f, 0.f, 0.f};
    float accb = 0.f;  // bias: sum of ga[co = i] over this lane's points
    for (int tile = blockIdx.x; tile < ntx * nty; tile += gridDim.x) {
        const int x0 = (tile % ntx) * TW, y0 = (tile / ntx) * TW;
        __syncthreads();
        for (int e = tid; e < CIN * HW * HW; e += 256) {
            const int ci = e / (HW * HW), q = e % (HW * HW);
            const int gx = x0 - 1 + q % HW, gy = y0 - 1 + q / HW;
            float v = 0.f;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const long long k = (long long)gy * nx + gx;
                v = in[ci * g.N + k];
                if (in_gate) v *= in_gate[ci * g.N + k];
                if (relu_in) v = fmaxf(v, 0.f);
            }
            sx[e] = v;
        }
        for (int e = tid; e < COUT * TW * TW; e += 256) {
            const int co = e / (TW * TW), q = e % (TW * TW);
            const int gx = x0 + q % TW, gy = y0 + q / TW;
            sg[e] = (gx < nx && gy < ny) ? ga[co * g.N + (long long)gy * nx + gx] : 0.f;
        }
        __syncthreads();
        for (int ks = wave; ks < TW * TW / 4; ks += 4) {
            const int p = ks * 4 + kk, py = p / TW, px = p % TW;
            const float a = i < COUT ? sg[i * TW * TW + p] : 0.f;
            accb += a;
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const float b = i < CIN ? sx[i * HW * HW + (py + t / 3) * HW + (px + t % 3)] : 0.f;
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    // D: lane holds D[co = 4 (lane >> 4) + c][ci = lane & 15]
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int co = 4 * kk + c, ci = i;
            if (co < COUT && ci < CIN) red[wave][(co * CIN + ci) * T + t] = acc[t][c];
        }
    // bias: lanes with the same co (i) hold disjoint point sets
    for (int d = 16; d < 64; d <<= 1) accb += __shfl_xor(accb, d, 64);
    if (kk == 0 && i < COUT) red[wave][COUT * CIN * T + i] = accb;
    __syncthreads();
    constexpr int stride = COUT * CIN * T + COUT;
    for (int e = tid; e < stride; e += 256)
        partials[(long long)blockIdx.x * stride + e] =
            ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// 3D weight gradient on the matrix cores, for 3x3x3 layers: the sums of
// k_conv_bwd_w as GEMMs D_t[co][ci] += A[co][4 points] B_t[4 points][ci]
// with v_mfma_f32_16x16x4f32 (FP32 operands and accumulation), as in 2D.
// Each block walks 8 x 8 x 4 tiles of points: ga on the tile and x on the
// tile plus a one-point halo (10 x 10 x 6, 0 outside the grid) are staged
// in LDS (every load of a thread is issued before its stores), then every
// wave takes a quarter of the tile's 64 four-point steps for all 27 taps.
// The four waves' sums are added in LDS in wave order (the x buffer is
// reused for that once the tiles are done) and written as this block's
// partials (same layout as k_conv_bwd_w).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w3d_mfma(GridInfo g, const float *__restrict__ in,
                                                           const float *__restrict__ in_gate,
                                                           int relu_in,
                                                           const float *__restrict__ ga,
                                                           float *__restrict__ partials) {
    constexpr int TX = 8, TY = 8, TZ = 4, HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    constexpr int TP = TX * TY * TZ, HP = HX * HY * HZ, T = 27;
    constexpr int stride = COUT * CIN * T + COUT;
    constexpr int SX = CIN * HP > stride ? CIN * HP : stride;
    __shared__ float sx[SX];  // x on the halo region; at the end the wave sums
    __shared__ float sg[COUT * TP];
    static_assert(CIN <= 16 && COUT <= 16, "one 16 x 16 MFMA tile");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, ntz = (nz + TZ - 1) / TZ;
    const int i = lane & 15, kk = lane >> 4;  // A row (co) / B column (ci), k
    f32x4v acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = f32x4v{0.f, 0.f, 0.f, 0.f};
    float accb = 0.f;  // bias: sum of ga[co = i] over this lane's points
    const long long ntiles = (long long)ntx * nty * ntz;
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = (int)(tile % ntx) * TX, y0 = (int)((tile / ntx) % nty) * TY,
                  z0 = (int)(tile / ((long long)ntx * nty)) * TZ;
        __syncthreads();
        {
            constexpr int NB = (CIN * HP + 255) / 256;
            float v[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int e = b * 256 + tid;
                v[b] = 0.f;
                if (e < CIN * HP) {
                    const int ci = e / HP, q = e % HP;
                    const int gx = x0 - 1 + q % HX, gy = y0 - 1 + (q / HX) % HY,
                              gz = z0 - 1 + q / (HX * HY);
                    if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
                        const long long k = ((long long)gz * ny + gy) * nx + gx;
                        float x = in[ci * g.N + k];
                        if (in_gate) x *= in_gate[ci * g.N + k];
                        v[b] = relu_in ? fmaxf(x, 0.f) : x;
                    }
                }
            }
            constexpr int NG = (COUT * TP + 255) / 256;
            float w[NG];
#pragma unroll
            for (int b = 0; b < NG; ++b) {
                const int e = b * 256 + tid;
                w[b] = 0.f;
                if (e < COUT * TP) {
                    const int co = e / TP, q = e % TP;
                    const int gx = x0 + q % TX, gy = y0 + (q / TX) % TY, gz = z0 + q / (TX * TY);
                    if (gx < nx && gy < ny && gz < nz)
                        w[b] = ga[co * g.N + ((long long)gz * ny + gy) * nx + gx];
                }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (b * 256 + tid < CIN * HP) sx[b * 256 + tid] = v[b];
#pragma unroll
            for (int b = 0; b < NG; ++b)
                if (b * 256 + tid < COUT * TP) sg[b * 256 + tid] = w[b];
        }
        __syncthreads();
        for (int ks = wave; ks < TP / 4; ks += 4) {
            const int p = ks * 4 + kk;
            const int px = p % TX, py = (p / TX) % TY, pz = p / (TX * TY);
            const float a = i < COUT ? sg[i * TP + p] : 0.f;
            accb += a;
            const int hb = i * HP + (pz * HY + py) * HX + px;  // tap (-1, -1, -1)
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const int off = ((t / 9) * HY + (t / 3) % 3) * HX + t % 3;
                const float b = i < CIN ? sx[hb + off] : 0.f;
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    // D: lane holds D[co = 4 (lane >> 4) + c][ci = lane & 15].  Bias: lanes
    // with the same co (i) hold disjoint point sets.
    for (int d = 16; d < 64; d <<= 1) accb += __shfl_xor(accb, d, 64);
    __syncthreads();  // the tiles are done with sx
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int co = 4 * kk + c, ci = i;
                    if (co < COUT && ci < CIN) {
                        float &r = sx[(co * CIN + ci) * T + t];
                        r = w == 0 ? acc[t][c] : r + acc[t][c];
                    }
                }
            if (kk == 0 && i < COUT) {
                float &r = sx[COUT * CIN * T + i];
                r = w == 0 ? accb : r + accb;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < stride; e += 256) partials[(long long)blockIdx.x * stride + e] = sx[e];
}

// grad[k] += sum over blocks of partials[b][k] (block order: deterministic);
// weights go to gW[0 .. nw), biases (the last nb entries) to gb (if given).
__global__ void k_reduce_partials(const float *partials, int nblocks, int stride, int nw,
                                  float *gW, float *gb) {
    const int k = blockIdx.x * kBS + threadIdx.x;
    if (k >= stride) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += (double)partials[(long long)b * stride + k];
    if (k < nw) gW[k] += (float)s;
    else if (gb) gb[k - nw] += (float)s;
}

// Gate net backward, point-wise part: gg = dG G (1 - G) (into dG's place),
// gh = (WB^T gg) * [h > 0].
template <int H, int G>
__global__ __launch_bounds__(kBS) void k_gate_b_bwd(long long N, const float *__restrict__ Gv,
                                                    float *__restrict__ gg,
                                                    const float *__restrict__ h,
                                                    const float *__restrict__ WB,
                                                    float *__restrict__ gh) {
    const float *sw = WB;
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i >= N) return;
    float acc[H];
#pragma unroll
    for (int c = 0; c < H; ++c) acc[c] = 0.f;
    for (int k = 0; k < G; ++k) {
        const float gv = Gv[k * N + i];
        const float v = gg[k * N + i] * gv * (1.f - gv);
        gg[k * N + i] = v;
#pragma unroll
        for (int c = 0; c < H; ++c) acc[c] += sw[k * H + c] * v;
    }
#pragma unroll
    for (int c = 0; c < H; ++c) gh[c * N + i] = h[c * N + i] > 0.f ? acc[c] : 0.f;
}

// ------------------------------------------------------------ loss, Adam --
struct LossState {
    double rr;
};

__global__ __launch_bounds__(kBS) void k_dot_self(long long N, const float *r, double *part) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    const double v = i < N ? (double)r[i] * (double)r[i] : 0.0;
    block_partial_sum(v, part);
}

__global__ __launch_bounds__(kBS) void k_dot_self_fin(LossState *ls, const double *part,
                                                      long long nb) {
    const double t = reduce_partials(part, nb);
    if (threadIdx.x == 0) ls->rr = t;
}

// gz = (Kz - r) / rr  (Kz already in gz); partials of (z.Kz/2 - z.r) / rr
__global__ __launch_bounds__(kBS) void k_loss_grad(long long N, const float *z, const float *r,
                                                   float *gz, const LossState *ls, double *part) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    const double rr = ls->rr;
    double v = 0.0;
    if (i < N) {
        const double kz = (double)gz[i], zi = (double)z[i], ri = (double)r[i];
        v = (0.5 * zi * kz - zi * ri) / rr;
        gz[i] = (float)((kz - ri) / rr);
    }
    block_partial_sum(v, part);
}

// loss += sum of the partials
__global__ __launch_bounds__(kBS) void k_loss_fin(const double *part, long long nb, double *loss) {
    const double t = reduce_partials(part, nb);
    if (threadIdx.x == 0) *loss += t;
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, long long n, float gscale,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    const float gi = gscale * g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

template <typename T>
__global__ void k_residual_vec(long long N, const T *b, const T *kx, T *r) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i < N) r[i] = b[i] - kx[i];
}

// ------------------------------------------------------------- drivers --
unsigned nblk(long long N) { return (unsigned)((N + kBS - 1) / kBS); }

template <int DIM>
int conv_launch(const GridInfo &g, int cin, int cout, const float *in, const float *in_gate,
                const float *W, const float *bias, float *out, float *pre, const float *gate,
                int relu, hipStream_t s) {
    const unsigned nb = nblk(g.N);
#define ADLBR_CONV(CI, CO)                                                                     \
    if (cin == CI && cout == CO) {                                                             \
        hipLaunchKernelGGL((k_conv<DIM, CI, CO>), dim3(nb), dim3(kBS), 0, s, g, in, in_gate, W, \
                           bias, out, pre, gate, relu);                                        \
        return ADLBR_OK;                                                                       \
    }
    ADLBR_CONV(1, 16)
    ADLBR_CONV(16, 16)
    ADLBR_CONV(16, 1)
    ADLBR_CONV(7, 16)
    ADLBR_CONV(13, 16)
#undef ADLBR_CONV
    set_error("conv: unsupported channel counts %d -> %d", cin, cout);
    return ADLBR_E_UNSUPPORTED;
}

template <int DIM>
int bwd_data_launch(const GridInfo &g, int cin, int cout, const float *ga, const float *W,
                    float *gin, hipStream_t s) {
    const unsigned nb = nblk(g.N);
    if (cin == 16 && cout == 16) {
        hipLaunchKernelGGL((k_conv_bwd_data<DIM, 16, 16>), dim3(nb), dim3(kBS), 0, s, g, ga, W, gin);
        return ADLBR_OK;
    }
    if (cin == 16 && cout == 1) {
        hipLaunchKernelGGL((k_conv_bwd_data<DIM, 16, 1>), dim3(nb), dim3(kBS), 0, s, g, ga, W, gin);
        return ADLBR_OK;
    }
    set_error("conv backward: unsupported channel counts");
    return ADLBR_E_UNSUPPORTED;
}

constexpr int kWgBlocks = 240;

template <int DIM>
int bwd_w_launch(const GridInfo &g, int cin, int cout, int taps, const float *in,
                 const float *in_gate, int relu_in, const float *ga, float *partials, float *gW,
                 float *gb, hipStream_t s) {
#define ADLBR_BW(CI, CO, PPT)                                                                 \
    if (cin == CI && cout == CO) {                                                            \
        if (DIM == 2 && taps == 9 && CI <= 16 && CO <= 16)                                    \
            hipLaunchKernelGGL((k_conv_bwd_w2d_mfma<CI, (CO <= 16 ? CO : 16)>),               \
                               dim3(kWgBlocks), dim3(kBS), 0, s, g, in, in_gate, relu_in, ga, \
                               partials);                                                     \
        else if (DIM == 3 && taps == 27 && CI <= 16 && CO <= 16)                              \
            hipLaunchKernelGGL((k_conv_bwd_w3d_mfma<CI, (CO <= 16 ? CO : 16)>),               \
                               dim3(kWgBlocks), dim3(kBS), 0, s, g, in, in_gate, relu_in, ga, \
                               partials);                                                     \
        else                                                                                  \
            hipLaunchKernelGGL((k_conv_bwd_w<DIM, CI, CO, PPT>), dim3(kWgBlocks), dim3(kBS),  \
                               0, s, g, in, in_gate, relu_in, ga, partials, taps);            \
        const int stride = CO * CI * taps + CO;                                               \
        hipLaunchKernelGGL(k_reduce_partials, dim3((stride + kBS - 1) / kBS), dim3(kBS), 0, s,  \
                           partials, kWgBlocks, stride, CO * CI * taps, gW, gb);              \
        return ADLBR_OK;                                                                      \
    }
    ADLBR_BW(1, 16, 1)
    ADLBR_BW(16, 16, 1)
    ADLBR_BW(16, 1, 1)
    ADLBR_BW(7, 16, 1)
    ADLBR_BW(13, 16, 1)
    ADLBR_BW(16, 32, 2)
#undef ADLBR_BW
    set_error("conv weight gradient: unsupported channel counts");
    return ADLBR_E_UNSUPPORTED;
}

struct NetWs {
    float *g0, *g1, *ga, *gl, *partials;
    size_t total;
};

NetWs net_ws(long long N, const NetDims &d, char *base) {
    NetWs w;
    size_t o = 0;
    const size_t plane = align_up(4 * (size_t)N);
    w.g0 = (float *)(base + o);  o += 16 * plane;
    w.g1 = (float *)(base + o);  o += 16 * plane;
    w.ga = (float *)(base + o);  o += 49 * plane;
    w.gl = (float *)(base + o);  o += align_up(4 * d.lcount);
    w.partials = (float *)(base + o);
    o += align_up(4 * (size_t)kWgBlocks * (16 * 16 * 27 + 64 + 49 * 16 + 49));
    w.total = o;
    return w;
}

template <int DIM>
int forward_impl(const adlbr_operator *op, const adlbr_net *net, const NetDims &d, const float *r,
                 float *z, float *saved, float *bufA, float *bufB, hipStream_t s) {
    const GridInfo &g = operator_grid(op);
    const long long N = g.N;
    const float *L = net->layers;
    const float *G = net->gates;
    float *pre = saved;
    int rc;
    rc = conv_launch<DIM>(g, 1, 16, r, nullptr, L + d.l1, nullptr, bufA, pre, G, 0, s);
    if (rc) return rc;
    rc = conv_launch<DIM>(g, 16, 16, bufA, nullptr, L + d.l2, nullptr, bufB,
                          pre ? pre + 16 * N : nullptr, G + 16 * N, 0, s);
    if (rc) return rc;
    rc = conv_launch<DIM>(g, 16, 16, bufB, nullptr, L + d.l3, nullptr, bufA,
                          pre ? pre + 32 * N : nullptr, G + 32 * N, 0, s);
    if (rc) return rc;
    rc = conv_launch<DIM>(g, 16, 1, bufA, nullptr, L + d.l4, nullptr, bufB,
                          pre ? pre + 48 * N : nullptr, G + 48 * N, 0, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_precond_out, dim3(nblk(N)), dim3(kBS), 0, s, N, r, net->features, bufB, z);
    return ADLBR_OK;
}

}  // namespace

int net_apply(const adlbr_net *net, const adlbr_operator *op, double dt, const void *r, void *z,
              hipStream_t s) {
    (void)dt;
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    if (operator_storage(op) != ADLBR_F32) {
        set_error("net: the operator's storage must be ADLBR_F32");
        return ADLBR_E_UNSUPPORTED;
    }
    if (d.dim == 2 && net->gates8)
        return net_apply_mfma(net, op, (const float *)r, (float *)z, nullptr, nullptr, nullptr, s);
    if (d.dim == 3 && net->gates8 && net->scratch)
        return net_apply_mfma3d(net, op, (const float *)r, (float *)z, nullptr, nullptr, nullptr,
                                s);
    if (!net->scratch) {
        set_error("net: the FP32 inference path needs net->scratch ([2W][N] FP32)");
        return ADLBR_E_INVALID;
    }
    const long long N = operator_grid(op).N;
    float *A = net->scratch, *B = net->scratch + 16 * N;
    return d.dim == 2 ? forward_impl<2>(op, net, d, (const float *)r, (float *)z, nullptr, A, B, s)
                      : forward_impl<3>(op, net, d, (const float *)r, (float *)z, nullptr, A, B, s);
}

namespace {
// Partials of <z, r> and <z, rp> (rp may be null) over 256-point blocks.
__global__ __launch_bounds__(kBS) void k_dots2(long long N, const float *__restrict__ z,
                                               const float *__restrict__ r,
                                               const float *__restrict__ rp, double *part) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (i < N) {
        const double zi = (double)z[i];
        a = zi * (double)r[i];
        if (rp) b = zi * (double)rp[i];
    }
    block_partial_sum(a, part);
    block_partial_sum(b, part + gridDim.x);
}
}  // namespace

int net_apply_dots(const adlbr_net *net, const adlbr_operator *op, const float *r,
                   const float *rp, float *z, double *part, long long *nparts,
                   const CgState *st, hipStream_t s) {
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    const GridInfo &g = operator_grid(op);
    if (d.dim == 2 && net->gates8 && operator_storage(op) == ADLBR_F32) {
        *nparts = net_mfma_blocks(g.nx, g.ny);
        return net_apply_mfma(net, op, r, z, rp, part, st, s);
    }
    if (d.dim == 3 && net->gates8 && net->scratch && operator_storage(op) == ADLBR_F32) {
        *nparts = net3d_tiles(g);
        return net_apply_mfma3d(net, op, r, z, rp, part, st, s);
    }
    rc = net_apply(net, op, 0.0, r, z, s);
    if (rc) return rc;
    *nparts = nblk(g.N);
    hipLaunchKernelGGL(k_dots2, dim3((unsigned)*nparts), dim3(kBS), 0, s, g.N, (const float *)z, r,
                       rp, part);
    return ADLBR_OK;
}

}  // namespace adlbr

using namespace adlbr;

extern "C" int adlbr_net_param_count(int dim, int width, int hidden, size_t *count) {
    clear_error();
    if ((dim != 2 && dim != 3) || width != 16 || hidden != 16 || !count) {
        set_error("adlbr_net_param_count: dim 2/3, width = hidden = 16");
        return ADLBR_E_INVALID;
    }
    *count = net_dims(dim, width, hidden).count;
    return ADLBR_OK;
}

extern "C" int adlbr_net_workspace(adlbr_operator *op, const adlbr_net *net, size_t *bytes) {
    clear_error();
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    if (!bytes) return ADLBR_E_INVALID;
    *bytes = net_ws(operator_grid(op).N, d, nullptr).total;
    return ADLBR_OK;
}

extern "C" int adlbr_net_features(adlbr_operator *op, double dt, adlbr_net *net, void *stream) {
    clear_error();
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    if (!net->features || !(dt >= 0.0)) {
        set_error("adlbr_net_features: need net->features and dt >= 0");
        return ADLBR_E_INVALID;
    }
    if (operator_storage(op) != ADLBR_F32) {
        set_error("adlbr_net_features: the operator's storage must be ADLBR_F32");
        return ADLBR_E_UNSUPPORTED;
    }
    const GridInfo &g = operator_grid(op);
    hipStream_t s = as_stream(stream);
    const float *w = (const float *)operator_weights(op);
    if (g.dim == 2)
        hipLaunchKernelGGL((k_features<2, float>), dim3(nblk(g.N)), dim3(kBS), 0, s, g,
                           (const float *)operator_diag(op), w, operator_slots(op),
                           operator_wide(op), dt, net->features);
    else
        hipLaunchKernelGGL((k_features<3, float>), dim3(nblk(g.N)), dim3(kBS), 0, s, g,
                           (const float *)operator_diag(op), w, operator_slots(op),
                           operator_wide(op), dt, net->features);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_net_gates(adlbr_operator *op, adlbr_net *net, void *stream) {
    clear_error();
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    if (!net->features || !net->hidden_act || !net->gates) {
        set_error("adlbr_net_gates: need features, hidden_act and gates buffers");
        return ADLBR_E_INVALID;
    }
    const GridInfo &g = operator_grid(op);
    hipStream_t s = as_stream(stream);
    const float *P = net->params;
    rc = g.dim == 2 ? conv_launch<2>(g, d.nf, 16, net->features, nullptr, P + d.oWA, P + d.obA,
                                     net->hidden_act, nullptr, nullptr, 0, s)
                    : conv_launch<3>(g, d.nf, 16, net->features, nullptr, P + d.oWA, P + d.obA,
                                     net->hidden_act, nullptr, nullptr, 0, s);
    if (rc) return rc;
    hipLaunchKernelGGL((k_gate_b<16, 16>), dim3(nblk(g.N)), dim3(kBS), 0, s, g.N,
                       (const float *)net->hidden_act, P + d.oWB, P + d.obB, net->gates,
                       net->gates8);
    hipLaunchKernelGGL(k_expand_weights, dim3(16), dim3(kBS), 0, s, P + d.oW1, P + d.oW2,
                       net->layers, d.W, d.T, d.l2, d.l3, d.l4);
    rc = g.dim == 2 ? net_pack_mfma(net, s) : net_pack_mfma3d(net, s);
    if (rc) return rc;
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_net_forward(adlbr_operator *op, const adlbr_net *net, const float *r, float *z,
                                 float *saved, void *stream) {
    clear_error();
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    if (!r || !z || !net->gates || !net->features) {
        set_error("adlbr_net_forward: null argument");
        return ADLBR_E_INVALID;
    }
    const GridInfo &g = operator_grid(op);
    hipStream_t s = as_stream(stream);
    if (!net->scratch) {
        set_error("adlbr_net_forward: net->scratch ([2W][N] FP32) is required");
        return ADLBR_E_INVALID;
    }
    float *A = net->scratch, *B = net->scratch + 16 * g.N;
    rc = g.dim == 2 ? forward_impl<2>(op, net, d, r, z, saved, A, B, s)
                    : forward_impl<3>(op, net, d, r, z, saved, A, B, s);
    if (rc) return rc;
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_net_precondition(adlbr_operator *op, const adlbr_net *net, const float *r,
                                      float *z, void *stream) {
    clear_error();
    if (!r || !z || r == z) {
        set_error("adlbr_net_precondition: null or aliased argument");
        return ADLBR_E_INVALID;
    }
    return net_apply(net, op, 0.0, r, z, as_stream(stream));
}

extern "C" int adlbr_net_backward(adlbr_operator *op, const adlbr_net *net, const float *r,
                                  const float *gz, const float *saved, float *gparams,
                                  float *ggates, void *workspace, size_t ws_bytes, void *stream) {
    clear_error();
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    if (!r || !gz || !saved || !gparams || !ggates || !workspace) {
        set_error("adlbr_net_backward: null argument");
        return ADLBR_E_INVALID;
    }
    const GridInfo &g = operator_grid(op);
    const long long N = g.N;
    NetWs w = net_ws(N, d, (char *)workspace);
    if (ws_bytes < w.total) {
        set_error("adlbr_net_backward: workspace has %zu bytes, %zu needed", ws_bytes, w.total);
        return ADLBR_E_NOMEM;
    }
    hipStream_t s = as_stream(stream);
    const float *L = net->layers;
    const float *G = net->gates;
    const int taps = d.T;
    // gradients of the expanded layers go to w.gl, then fold onto W1, W2
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk((long long)d.lcount)), dim3(kBS), 0, s, w.gl,
                       (long long)d.lcount, 0.f);
    // layer 4: out = pre4 * G[48]; dL/dout = gz
    const float *gcur = gz;
    const size_t offs[4] = {0, 16, 32, 48};
    const int cins[4] = {1, 16, 16, 16}, couts[4] = {16, 16, 16, 1};
    const size_t oW[4] = {d.l1, d.l2, d.l3, d.l4};
    float *gbuf[2] = {w.g0, w.g1};
    for (int l = 3; l >= 0; --l) {
        const long long n = (long long)couts[l] * N;
        hipLaunchKernelGGL(k_gate_grad, dim3(nblk(n)), dim3(kBS), 0, s, n, gcur, G + offs[l] * N,
                           saved + offs[l] * N, w.ga, ggates + offs[l] * N);
        // input of layer l: r, or the previous layer's pre-gate output times its gates
        const float *in = l == 0 ? r : saved + offs[l - 1] * N;
        const float *in_gate = l == 0 ? nullptr : G + offs[l - 1] * N;
        rc = g.dim == 2 ? bwd_w_launch<2>(g, cins[l], couts[l], taps, in, in_gate, 0, w.ga,
                                          w.partials, w.gl + oW[l], nullptr, s)
                        : bwd_w_launch<3>(g, cins[l], couts[l], taps, in, in_gate, 0, w.ga,
                                          w.partials, w.gl + oW[l], nullptr, s);
        if (rc) return rc;
        if (l > 0) {
            float *gin = gbuf[l & 1];
            rc = g.dim == 2 ? bwd_data_launch<2>(g, cins[l], couts[l], w.ga, L + oW[l], gin, s)
                            : bwd_data_launch<3>(g, cins[l], couts[l], w.ga, L + oW[l], gin, s);
            if (rc) return rc;
            gcur = gin;
        }
    }
    hipLaunchKernelGGL(k_fold_weight_grads, dim3(16), dim3(kBS), 0, s, (const float *)w.gl,
                       gparams + d.oW1, gparams + d.oW2, d.W, d.T, d.l2, d.l3, d.l4);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_net_gates_backward(adlbr_operator *op, const adlbr_net *net,
                                        const float *ggates, float *gparams, void *workspace,
                                        size_t ws_bytes, void *stream) {
    clear_error();
    NetDims d;
    int rc = check_net(op, net, &d);
    if (rc) return rc;
    if (!ggates || !gparams || !workspace || !net->hidden_act) {
        set_error("adlbr_net_gates_backward: null argument");
        return ADLBR_E_INVALID;
    }
    const GridInfo &g = operator_grid(op);
    const long long N = g.N;
    NetWs w = net_ws(N, d, (char *)workspace);
    if (ws_bytes < w.total) {
        set_error("adlbr_net_gates_backward: workspace too small");
        return ADLBR_E_NOMEM;
    }
    hipStream_t s = as_stream(stream);
    const float *P = net->params;
    // fold the expanded gate gradients onto g1, g2 (into w.ga); then
    // gg = dg g (1 - g) in place (the first 2W expanded gates are g1, g2);
    // gh (in w.g0) = WB^T gg * [h > 0]
    hipLaunchKernelGGL(k_fold_gate_grads, dim3(nblk(N)), dim3(kBS), 0, s, N, d.W, ggates, w.ga);
    hipLaunchKernelGGL((k_gate_b_bwd<16, 32>), dim3(nblk(N)), dim3(kBS), 0, s, N, net->gates, w.ga,
                       net->hidden_act, P + d.oWB, w.g0);
    // WB, bB: 1x1 layer, input relu(h)
    rc = g.dim == 2 ? bwd_w_launch<2>(g, 16, 32, 1, net->hidden_act, nullptr, 1, w.ga, w.partials,
                                      gparams + d.oWB, gparams + d.obB, s)
                    : bwd_w_launch<3>(g, 16, 32, 1, net->hidden_act, nullptr, 1, w.ga, w.partials,
                                      gparams + d.oWB, gparams + d.obB, s);
    if (rc) return rc;
    // WA, bA: conv on the features
    rc = g.dim == 2 ? bwd_w_launch<2>(g, d.nf, 16, d.T, net->features, nullptr, 0, w.g0,
                                      w.partials, gparams + d.oWA, gparams + d.obA, s)
                    : bwd_w_launch<3>(g, d.nf, 16, d.T, net->features, nullptr, 0, w.g0,
                                      w.partials, gparams + d.oWA, gparams + d.obA, s);
    if (rc) return rc;
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_net_loss_grad(adlbr_operator *op, double dt, const float *r, const float *z,
                                   float *gz, double *loss, void *workspace, size_t ws_bytes,
                                   void *stream) {
    clear_error();
    if (!op || !r || !z || !gz || !loss || !workspace || operator_storage(op) != ADLBR_F32) {
        set_error("adlbr_net_loss_grad: bad argument (FP32 operator required)");
        return ADLBR_E_INVALID;
    }
    const long long N = operator_grid(op).N;
    const size_t need = align_up(sizeof(LossState)) + align_up(8 * (size_t)nblk(N) + 64);
    if (ws_bytes < need) {
        set_error("adlbr_net_loss_grad: workspace too small");
        return ADLBR_E_NOMEM;
    }
    hipStream_t s = as_stream(stream);
    LossState *ls = (LossState *)workspace;
    double *part = (double *)((char *)workspace + align_up(sizeof(LossState)));
    const long long nb = nblk(N);
    hipLaunchKernelGGL(k_dot_self, dim3(nb), dim3(kBS), 0, s, N, r, part);
    hipLaunchKernelGGL(k_dot_self_fin, dim3(1), dim3(kBS), 0, s, ls, (const double *)part, nb);
    int rc = apply_K(op, z, gz, dt, s);  // gz = K z
    if (rc) return rc;
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(kBS), 0, s, N, z, r, gz, (const LossState *)ls,
                       part);
    hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(kBS), 0, s, (const double *)part, nb, loss);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_net_adam(float *params, const float *grads, float *m, float *v, int64_t n,
                              int32_t step, double grad_scale, double lr, double beta1,
                              double beta2, double eps, void *stream) {
    clear_error();
    if (!params || !grads || !m || !v || n < 1 || step < 1 || !(grad_scale > 0.0)) {
        set_error("adlbr_net_adam: bad argument");
        return ADLBR_E_INVALID;
    }
    const float c1 = (float)(1.0 - pow(beta1, step)), c2 = (float)(1.0 - pow(beta2, step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(kBS), 0, as_stream(stream), params, grads, m, v,
                       (long long)n, (float)grad_scale, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_residual(adlbr_operator *op, double dt, const void *b, const void *x, void *r,
                              void *stream) {
    clear_error();
    if (!op || !b || !x || !r || r == x) {
        set_error("adlbr_residual: null or aliased argument");
        return ADLBR_E_INVALID;
    }
    hipStream_t s = as_stream(stream);
    const long long N = operator_grid(op).N;
    int rc = apply_K(op, x, r, dt, s);  // r = K x
    if (rc) return rc;
    const int sto = operator_storage(op);
    if (sto == ADLBR_F32)
        hipLaunchKernelGGL(k_residual_vec<float>, dim3(nblk(N)), dim3(kBS), 0, s, N,
                           (const float *)b, (const float *)r, (float *)r);
    else if (sto == ADLBR_F64)
        hipLaunchKernelGGL(k_residual_vec<double>, dim3(nblk(N)), dim3(kBS), 0, s, N,
                           (const double *)b, (const double *)r, (double *)r);
    else {
        set_error("adlbr_residual: storage must be F32 or F64");
        return ADLBR_E_UNSUPPORTED;
    }
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}
