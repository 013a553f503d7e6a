// Solution-dependent diffusion tensor from the structure tensor
// (Section 4: coherence-enhancing diffusion, 2D and 3D; edge-enhancing
// diffusion in 3D):
//   u_sigma = K_sigma * u,  J = K_rho * (grad u_sigma grad u_sigma^T),
//   D = sum_k lambda_k v_k v_k^T over the eigenpairs of J.
// Separable Gaussian passes (x, y[, z]) with half-sample mirror boundary,
// central differences, then a per-point eigen map.  All passes stream the
// planes through HBM with coalesced x-fastest accesses; the Gaussian taps
// (truncated at ceil(3 s), normalized) are computed on the host in FP64.
#include <mutex>

#include "common.h"

// Scratch of adlbr_structure_tensor_noalloc: the two working halves that
// adlbr_structure_tensor takes from its workspace, in device memory the
// library holds from load to process exit (one copy per GPU).  Host code
// uses only the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace adlbr {
namespace {

constexpr int kMaxR = 31;

struct Taps {
    float f[2 * kMaxR + 1];
    double d[2 * kMaxR + 1];
    int r;
};

Taps make_taps(double s) {
    Taps t;
    int r = (int)ceil(3.0 * s);
    if (r < 1) r = 1;
    t.r = r;
    double sum = 0.0, g[2 * kMaxR + 1];
    for (int k = -r; k <= r; ++k) {
        g[k + r] = exp(-(double)(k * k) / (2.0 * s * s));
        sum += g[k + r];
    }
    for (int k = 0; k < 2 * r + 1; ++k) {
        t.d[k] = g[k] / sum;
        t.f[k] = (float)t.d[k];
    }
    return t;
}

template <typename T> __device__ __forceinline__ T tap(const Taps &t, int k);
template <> __device__ __forceinline__ float tap<float>(const Taps &t, int k) { return t.f[k]; }
template <> __device__ __forceinline__ double tap<double>(const Taps &t, int k) { return t.d[k]; }

__device__ __forceinline__ int mirror(int i, int n) {
    // half-sample symmetric extension: -1 -> 0, n -> n-1, period 2n
    const int p = 2 * n;
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - 1 - i;
}

// Blur `planes` planes along axis `ax`; blockIdx.y selects the plane.
template <typename T>
__global__ void k_blur(GridInfo g, const T *__restrict__ in, T *__restrict__ out, int ax, Taps t) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long N = g.N;
    if (i >= N) return;
    const long long off = (long long)blockIdx.y * N;
    const int nx = g.nx, ny = g.ny;
    const int x = (int)(i % nx);
    const long long rest = i / nx;
    const int y = (int)(rest % ny);
    const int z = (int)(rest / ny);
    const int p = ax == 0 ? x : (ax == 1 ? y : z);
    const int len = ax == 0 ? nx : (ax == 1 ? ny : g.nz);
    const long long stride = ax == 0 ? 1 : (ax == 1 ? (long long)nx : (long long)nx * ny);
    const T *src = in + off + i - (long long)p * stride;
    T acc = (T)0;
    if (p - t.r >= 0 && p + t.r < len) {
        for (int k = -t.r; k <= t.r; ++k) acc += tap<T>(t, k + t.r) * src[(long long)(p + k) * stride];
    } else {
        for (int k = -t.r; k <= t.r; ++k)
            acc += tap<T>(t, k + t.r) * src[(long long)mirror(p + k, len) * stride];
    }
    out[off + i] = acc;
}

// grad u_sigma by central differences (mirror boundary), outer products.
// add != 0 adds the products to J (the next component of a vector-valued
// image) instead of overwriting it.
template <typename T>
__global__ void k_grad_outer(GridInfo g, const T *__restrict__ us, T *__restrict__ J, int add) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long N = g.N;
    if (i >= N) return;
    const int nx = g.nx, ny = g.ny;
    const int x = (int)(i % nx);
    const long long rest = i / nx;
    const int y = (int)(rest % ny);
    const int z = (int)(rest / ny);
    const T half = (T)0.5;
    const T gx = half * (us[i + (mirror(x + 1, nx) - x)] - us[i + (mirror(x - 1, nx) - x)]);
    const T gy = half * (us[i + (long long)(mirror(y + 1, ny) - y) * nx] -
                         us[i + (long long)(mirror(y - 1, ny) - y) * nx]);
    if (g.dim == 2) {
        const T p[3] = {gx * gx, gx * gy, gy * gy};
#pragma unroll
        for (int k = 0; k < 3; ++k) J[k * N + i] = add ? J[k * N + i] + p[k] : p[k];
    } else {
        const long long sz = (long long)nx * ny;
        const T gz = half * (us[i + (long long)(mirror(z + 1, g.nz) - z) * sz] -
                             us[i + (long long)(mirror(z - 1, g.nz) - z) * sz]);
        const T p[6] = {gx * gx, gx * gy, gx * gz, gy * gy, gy * gz, gz * gz};
#pragma unroll
        for (int k = 0; k < 6; ++k) J[k * N + i] = add ? J[k * N + i] + p[k] : p[k];
    }
}

template <typename T> __device__ __forceinline__ T coh(T C, T dmu) {
    return dmu == (T)0 ? (T)0 : exp(-C / (dmu * dmu));
}

template <typename T> __device__ __forceinline__ T eed(T C, T mu) {
    return mu == (T)0 ? (T)1 : (T)1 - exp(-C / (mu * mu));
}

// 2D eigen map in closed form: D = lambda_2 Id + (lambda_1 - lambda_2) v1 v1^T
// with v1 the unit eigenvector of the larger eigenvalue mu_1.
template <typename T>
__global__ void k_eigmap2(long long N, const T *__restrict__ J, T *__restrict__ D, T alpha, T C,
                          int map) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T a = J[i], b = J[N + i], c = J[2 * N + i];
    const T hd = (T)0.5 * (a - c);
    const T disc = sqrt(hd * hd + b * b);
    const T mid = (T)0.5 * (a + c);
    const T mu1 = mid + disc, mu2 = mid - disc;
    T vx, vy;
    if (disc == (T)0) {
        vx = (T)1;
        vy = (T)0;
    } else if (a >= c) {
        vx = hd + disc;
        vy = b;
    } else {
        vx = b;
        vy = disc - hd;
    }
    const T nrm = sqrt(vx * vx + vy * vy);
    vx /= nrm;
    vy /= nrm;
    T l1, l2;
    if (map == ADLBR_MAP_CED) {
        l1 = alpha;
        l2 = alpha + ((T)1 - alpha) * coh(C, mu1 - mu2);
    } else {
        l1 = eed(C, mu1);
        l2 = (T)1;
    }
    const T dl = l1 - l2;
    D[i] = l2 + dl * vx * vx;
    D[N + i] = dl * vx * vy;
    D[2 * N + i] = l2 + dl * vy * vy;
}

// 3D eigen map: cyclic Jacobi rotations on the symmetric 3x3 J.
template <typename T>
__global__ void k_eigmap3(long long N, const T *__restrict__ J, T *__restrict__ D, T alpha, T C,
                          int map) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    T A[3][3] = {{J[i], J[N + i], J[2 * N + i]},
                 {J[N + i], J[3 * N + i], J[4 * N + i]},
                 {J[2 * N + i], J[4 * N + i], J[5 * N + i]}};
    T V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    const T eps = sizeof(T) == 8 ? (T)1e-15 : (T)1e-7;
    for (int sweep = 0; sweep < 12; ++sweep) {
        const T offd = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        const T scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (offd == (T)0 || offd <= eps * scale) break;
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            if (A[p][q] == (T)0) continue;
            // rotation zeroing A[p][q]: tan 2th = 2 A_pq / (A_qq - A_pp)
            const T th = (T)0.5 * atan2((T)2 * A[p][q], A[q][q] - A[p][p]);
            const T cs = cos(th), sn = sin(th);
            for (int k = 0; k < 3; ++k) {
                const T akp = A[k][p], akq = A[k][q];
                A[k][p] = cs * akp - sn * akq;
                A[k][q] = sn * akp + cs * akq;
            }
            for (int k = 0; k < 3; ++k) {
                const T apk = A[p][k], aqk = A[q][k];
                A[p][k] = cs * apk - sn * aqk;
                A[q][k] = sn * apk + cs * aqk;
            }
            for (int k = 0; k < 3; ++k) {
                const T vkp = V[k][p], vkq = V[k][q];
                V[k][p] = cs * vkp - sn * vkq;
                V[k][q] = sn * vkp + cs * vkq;
            }
        }
    }
    int o[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (A[o[b]][o[b]] > A[o[a]][o[a]]) {
                const int t = o[a];
                o[a] = o[b];
                o[b] = t;
            }
    const T mu[3] = {A[o[0]][o[0]], A[o[1]][o[1]], A[o[2]][o[2]]};
    T lam[3];
    if (map == ADLBR_MAP_CED) {
        lam[0] = alpha;
        lam[1] = alpha + ((T)1 - alpha) * coh(C, mu[0] - mu[1]);
        lam[2] = alpha + ((T)1 - alpha) * coh(C, mu[0] - mu[2]);
    } else {
        lam[0] = eed(C, mu[0]);
        lam[1] = eed(C, mu[1]);
        lam[2] = (T)1;
    }
    const int pr[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int q = 0; q < 6; ++q) {
        T acc = (T)0;
        for (int k = 0; k < 3; ++k) acc += lam[k] * V[pr[q][0]][o[k]] * V[pr[q][1]][o[k]];
        D[q * N + i] = acc;
    }
}

// ---------------------------------------------------------- tiled 2D --
// Kernel 1: u -> u_sigma -> central differences -> J = grad grad^T on a
// 32x32 tile, all in LDS.  The tile is loaded with mirrored indices; since
// the half-sample symmetric extension of u is symmetric about -1/2 and n-1/2
// and the Gaussian is symmetric, blurring the extended tile equals blurring
// with a mirror boundary at every pass, and u_sigma at a mirrored halo point
// equals u_sigma at its mirror image.
constexpr int kTile = 32;

template <typename T, int RS>
__global__ __launch_bounds__(256) void k_st_grad_tiled(int nx, int ny, int ncomp,
                                                       const T *__restrict__ u,
                                                       T *__restrict__ J, Taps ts) {
    constexpr int E = kTile + 2 + 2 * RS;   // u region edge
    constexpr int EU = kTile + 2;           // u_sigma region edge
    constexpr int KO = kTile * kTile / 256;  // outputs per thread
    static_assert(kTile * kTile % 256 == 0, "whole outputs per thread");
    __shared__ T su[E * E];
    __shared__ T sx[E * EU];                // blurred along x
    __shared__ T ss[EU * EU];               // u_sigma
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    const long long N = (long long)nx * ny;
    T jxx[KO], jxy[KO], jyy[KO];
#pragma unroll
    for (int o = 0; o < KO; ++o) jxx[o] = jxy[o] = jyy[o] = (T)0;
    for (int c = 0; c < ncomp; ++c) {
        const T *uc = u + c * N;
        {  // all of a thread's loads, then its LDS stores
            constexpr int B = (E * E + 255) / 256;
            T v[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int k0 = b * 256 + (int)threadIdx.x, k = k0 < E * E ? k0 : 0;
                const int gx = mirror(x0 - 1 - RS + k % E, nx), gy = mirror(y0 - 1 - RS + k / E, ny);
                v[b] = uc[(long long)gy * nx + gx];
            }
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (b * 256 + (int)threadIdx.x < E * E) su[b * 256 + threadIdx.x] = v[b];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < E * EU; k += 256) {
            const int yy = k / EU, xx = k % EU;
            T a = (T)0;
#pragma unroll
            for (int j = 0; j <= 2 * RS; ++j) a += tap<T>(ts, j) * su[yy * E + xx + j];
            sx[k] = a;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < EU * EU; k += 256) {
            const int yy = k / EU, xx = k % EU;
            T a = (T)0;
#pragma unroll
            for (int j = 0; j <= 2 * RS; ++j) a += tap<T>(ts, j) * sx[(yy + j) * EU + xx];
            ss[k] = a;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < KO; ++o) {
            const int k = o * 256 + (int)threadIdx.x;
            const int ty = k / kTile, tx = k % kTile;
            const int cc = (ty + 1) * EU + (tx + 1);
            const T half = (T)0.5;
            const T gxv = half * (ss[cc + 1] - ss[cc - 1]);
            const T gyv = half * (ss[cc + EU] - ss[cc - EU]);
            jxx[o] += gxv * gxv;
            jxy[o] += gxv * gyv;
            jyy[o] += gyv * gyv;
        }
        // the next component overwrites su, sx and ss
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < KO; ++o) {
        const int k = o * 256 + (int)threadIdx.x;
        const int ty = k / kTile, tx = k % kTile;
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx >= nx || gy >= ny) continue;
        const long long i = (long long)gy * nx + gx;
        J[i] = jxx[o];
        J[N + i] = jxy[o];
        J[2 * N + i] = jyy[o];
    }
}

// Kernel 2: J -> K_rho * J (x then y, mirrored tile) -> eigen map -> D.
// Both passes slide a window along the filter direction in registers: a
// thread takes 8 consecutive outputs of a row (x pass) or 4 of a column (y
// pass), reading 8 + 2 RR (4 + 2 RR) values instead of 25 per output.
// Every output still sums its taps in the order j = 0 .. 2 RR.
template <typename T, int RR>
__global__ __launch_bounds__(256) void k_st_smooth_map_tiled(int nx, int ny,
                                                             const T *__restrict__ J,
                                                             T *__restrict__ D, Taps tr, T alpha,
                                                             T C, int map) {
    constexpr int E = kTile + 2 * RR;
    constexpr int XO = 8, YO = 4;  // outputs per thread in the x and y passes
    static_assert(kTile % XO == 0 && (kTile / YO) * kTile == 256, "pass shapes");
    __shared__ T sj[3][E * E];
    __shared__ T sx[3][E * kTile];
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    const long long N = (long long)nx * ny;
    // staged B items per thread at a time: all their loads, then their LDS
    // stores (a lane past the end reloads the tile's first point)
    constexpr int B = 7;
    for (int kb = 0; kb < E * E; kb += B * 256) {
        T v[B][3];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k0 = kb + b * 256 + (int)threadIdx.x, k = k0 < E * E ? k0 : 0;
            const int gx = mirror(x0 - RR + k % E, nx), gy = mirror(y0 - RR + k / E, ny);
            const long long i = (long long)gy * nx + gx;
            v[b][0] = J[i];
            v[b][1] = J[N + i];
            v[b][2] = J[2 * N + i];
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k = kb + b * 256 + (int)threadIdx.x;
            if (k < E * E) {
                sj[0][k] = v[b][0];
                sj[1][k] = v[b][1];
                sj[2][k] = v[b][2];
            }
        }
    }
    __syncthreads();
    for (int it = threadIdx.x; it < E * (kTile / XO); it += 256) {
        const int yy = it / (kTile / XO), xs = (it % (kTile / XO)) * XO;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T win[XO + 2 * RR];
#pragma unroll
            for (int j = 0; j < XO + 2 * RR; ++j) win[j] = sj[c][yy * E + xs + j];
#pragma unroll
            for (int o = 0; o < XO; ++o) {
                T a = (T)0;
#pragma unroll
                for (int j = 0; j <= 2 * RR; ++j) a += tap<T>(tr, j) * win[o + j];
                sx[c][yy * kTile + xs + o] = a;
            }
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % kTile, ys = (threadIdx.x / kTile) * YO;
    T acc[3][YO];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T win[YO + 2 * RR];
#pragma unroll
        for (int j = 0; j < YO + 2 * RR; ++j) win[j] = sx[c][(ys + j) * kTile + tx];
#pragma unroll
        for (int o = 0; o < YO; ++o) {
            T a = (T)0;
#pragma unroll
            for (int j = 0; j <= 2 * RR; ++j) a += tap<T>(tr, j) * win[o + j];
            acc[c][o] = a;
        }
    }
#pragma unroll
    for (int o = 0; o < YO; ++o) {
        const int ty = ys + o;
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx >= nx || gy >= ny) continue;
        const T a = acc[0][o], b = acc[1][o], c = acc[2][o];
        const T hd = (T)0.5 * (a - c);
        const T disc = sqrt(hd * hd + b * b);
        const T mid = (T)0.5 * (a + c);
        const T mu1 = mid + disc, mu2 = mid - disc;
        T vx, vy;
        if (disc == (T)0) {
            vx = (T)1;
            vy = (T)0;
        } else if (a >= c) {
            vx = hd + disc;
            vy = b;
        } else {
            vx = b;
            vy = disc - hd;
        }
        const T nrm = sqrt(vx * vx + vy * vy);
        vx /= nrm;
        vy /= nrm;
        T l1, l2;
        if (map == ADLBR_MAP_CED) {
            l1 = alpha;
            l2 = alpha + ((T)1 - alpha) * coh(C, mu1 - mu2);
        } else {
            l1 = eed(C, mu1);
            l2 = (T)1;
        }
        const T dl = l1 - l2;
        const long long i = (long long)gy * nx + gx;
        D[i] = l2 + dl * vx * vx;
        D[N + i] = dl * vx * vy;
        D[2 * N + i] = l2 + dl * vy * vy;
    }
}

// The tiled path covers the common radii (sigma <= 1: r_sigma <= 3;
// rho <= 4: r_rho <= 12) in FP32; other cases use the streaming passes.
template <typename T> bool run_tensor_tiled(const GridInfo &g, const T *u, int ncomp,
                                            const Taps &ts, const Taps &tr,
                                            const adlbr_tensor_params *p, T *D, T *wa,
                                            hipStream_t s) {
    if (g.dim != 2 || sizeof(T) != 4) return false;
    const dim3 grid((g.nx + kTile - 1) / kTile, (g.ny + kTile - 1) / kTile);
#define ADLBR_ST1(RS)                                                                       \
    if (ts.r == RS) hipLaunchKernelGGL((k_st_grad_tiled<T, RS>), grid, dim3(256), 0, s, g.nx, g.ny, ncomp, u, wa, ts);
    if (ts.r < 1 || ts.r > 3) return false;
    if (tr.r < 1 || tr.r > 12) return false;
    ADLBR_ST1(1) ADLBR_ST1(2) ADLBR_ST1(3)
#undef ADLBR_ST1
#define ADLBR_ST2(RR)                                                                        \
    if (tr.r == RR) hipLaunchKernelGGL((k_st_smooth_map_tiled<T, RR>), grid, dim3(256), 0, s, g.nx, \
                                       g.ny, (const T *)wa, D, tr, (T)p->alpha, (T)p->C, p->eig_map);
    ADLBR_ST2(1) ADLBR_ST2(2) ADLBR_ST2(3) ADLBR_ST2(4) ADLBR_ST2(5) ADLBR_ST2(6)
    ADLBR_ST2(7) ADLBR_ST2(8) ADLBR_ST2(9) ADLBR_ST2(10) ADLBR_ST2(11) ADLBR_ST2(12)
#undef ADLBR_ST2
    return true;
}

// u holds ncomp planes of N values; J sums the gradient outer products of
// every component (the common tensor of a vector-valued image).  The
// workspace halves wa, wb (nj N values each): in 2D J gathers in wa and the
// per-component blur passes use wb; in 3D the other way round.
template <typename T>
int run_tensor(const GridInfo &g, const T *u, int ncomp, const adlbr_tensor_params *p, T *D,
               T *wa, T *wb, hipStream_t s) {
    const long long N = g.N;
    const int nj = g.dim == 2 ? 3 : 6;
    const unsigned nb = (unsigned)((N + 255) / 256);
    const Taps ts = make_taps(p->sigma), tr = make_taps(p->rho);
    if (run_tensor_tiled<T>(g, u, ncomp, ts, tr, p, D, wa, s)) {
        ADLBR_LAUNCH_CHECK();
        return ADLBR_OK;
    }
    if (g.dim == 2) {
        for (int c = 0; c < ncomp; ++c) {  // u_sigma of component c, its products
            hipLaunchKernelGGL(k_blur<T>, dim3(nb, 1), dim3(256), 0, s, g, u + c * N, wb, 0, ts);
            hipLaunchKernelGGL(k_blur<T>, dim3(nb, 1), dim3(256), 0, s, g, (const T *)wb, wb + N, 1, ts);
            hipLaunchKernelGGL(k_grad_outer<T>, dim3(nb), dim3(256), 0, s, g, (const T *)(wb + N), wa,
                               c > 0 ? 1 : 0);
        }
        hipLaunchKernelGGL(k_blur<T>, dim3(nb, nj), dim3(256), 0, s, g, (const T *)wa, wb, 0, tr);
        hipLaunchKernelGGL(k_blur<T>, dim3(nb, nj), dim3(256), 0, s, g, (const T *)wb, wa, 1, tr);
        hipLaunchKernelGGL(k_eigmap2<T>, dim3(nb), dim3(256), 0, s, N, (const T *)wa, D,
                           (T)p->alpha, (T)p->C, p->eig_map);
    } else {
        for (int c = 0; c < ncomp; ++c) {
            hipLaunchKernelGGL(k_blur<T>, dim3(nb, 1), dim3(256), 0, s, g, u + c * N, wa, 0, ts);
            hipLaunchKernelGGL(k_blur<T>, dim3(nb, 1), dim3(256), 0, s, g, (const T *)wa, wa + N, 1, ts);
            hipLaunchKernelGGL(k_blur<T>, dim3(nb, 1), dim3(256), 0, s, g, (const T *)(wa + N), wa, 2, ts);
            hipLaunchKernelGGL(k_grad_outer<T>, dim3(nb), dim3(256), 0, s, g, (const T *)wa, wb,
                               c > 0 ? 1 : 0);
        }
        hipLaunchKernelGGL(k_blur<T>, dim3(nb, nj), dim3(256), 0, s, g, (const T *)wb, wa, 0, tr);
        hipLaunchKernelGGL(k_blur<T>, dim3(nb, nj), dim3(256), 0, s, g, (const T *)wa, wb, 1, tr);
        hipLaunchKernelGGL(k_blur<T>, dim3(nb, nj), dim3(256), 0, s, g, (const T *)wb, wa, 2, tr);
        hipLaunchKernelGGL(k_eigmap3<T>, dim3(nb), dim3(256), 0, s, N, (const T *)wa, D,
                           (T)p->alpha, (T)p->C, p->eig_map);
    }
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

}  // namespace
}  // namespace adlbr

using namespace adlbr;

extern "C" int adlbr_tensor_workspace(const adlbr_grid *g, int dtype, size_t *bytes) {
    clear_error();
    GridInfo gi;
    int rc = check_grid(g, &gi);
    if (rc) return rc;
    if (!bytes || (dtype != ADLBR_F32 && dtype != ADLBR_F64)) {
        set_error("adlbr_tensor_workspace: dtype must be ADLBR_F32 or ADLBR_F64");
        return ADLBR_E_INVALID;
    }
    const int nj = gi.dim == 2 ? 3 : 6;
    *bytes = 2 * align_up(dtype_size(dtype) * nj * (size_t)gi.N);
    return ADLBR_OK;
}

namespace {
// Arguments shared by both tensor entry points; on success gi is the grid
// and need the scratch bytes (two halves of `half` bytes).
int tensor_args(const char *who, const adlbr_grid *g, const void *u, int dtype,
                const adlbr_tensor_params *p, const void *D, GridInfo *gi, size_t *half) {
    int rc = check_grid(g, gi);
    if (rc) return rc;
    if (!u || !p || !D) {
        set_error("%s: null pointer argument", who);
        return ADLBR_E_INVALID;
    }
    if (dtype != ADLBR_F32 && dtype != ADLBR_F64) {
        set_error("%s: dtype must be ADLBR_F32 or ADLBR_F64", who);
        return ADLBR_E_INVALID;
    }
    if (!(p->sigma > 0.0) || !(p->rho > 0.0) || p->sigma > 10.0 || p->rho > 10.0 ||
        !(p->alpha > 0.0) || !(p->alpha <= 1.0) || !(p->C >= 0.0) ||
        (p->eig_map != ADLBR_MAP_CED && p->eig_map != ADLBR_MAP_EED)) {
        set_error("%s: need 0 < sigma, rho <= 10, 0 < alpha <= 1, C >= 0", who);
        return ADLBR_E_INVALID;
    }
    const int nj = gi->dim == 2 ? 3 : 6;
    *half = align_up(dtype_size(dtype) * nj * (size_t)gi->N);
    return ADLBR_OK;
}

int tensor_run(const GridInfo &gi, const void *u, int ncomp, int dtype,
               const adlbr_tensor_params *p, void *D, char *b, size_t half, hipStream_t s) {
    if (dtype == ADLBR_F32)
        return run_tensor<float>(gi, (const float *)u, ncomp, p, (float *)D, (float *)b,
                                 (float *)(b + half), s);
    return run_tensor<double>(gi, (const double *)u, ncomp, p, (double *)D, (double *)b,
                              (double *)(b + half), s);
}

// Device address of `scratch` on each GPU, looked up once per device with
// that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(char **out) {
    int dev = -1;
    ADLBR_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("adlbr_structure_tensor_noalloc: device %d beyond the supported %d", dev,
                  kMaxDevices);
        return ADLBR_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("adlbr_structure_tensor_noalloc: hipGetSymbolAddress failed: %s",
                      hipGetErrorString(e));
            return ADLBR_E_HIP;
        }
        g_scratch_ptr[dev] = (char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return ADLBR_OK;
}
}  // namespace

extern "C" int adlbr_structure_tensor_vec(const adlbr_grid *g, const void *u, int ncomp,
                                          int dtype, const adlbr_tensor_params *p, void *D,
                                          void *workspace, size_t ws_bytes, void *stream) {
    clear_error();
    GridInfo gi;
    size_t half = 0;
    int rc = tensor_args("adlbr_structure_tensor", g, u, dtype, p, D, &gi, &half);
    if (rc) return rc;
    if (ncomp < 1) {
        set_error("adlbr_structure_tensor: ncomp = %d, need at least one component", ncomp);
        return ADLBR_E_INVALID;
    }
    if (!workspace) {
        set_error("adlbr_structure_tensor: null workspace");
        return ADLBR_E_INVALID;
    }
    if (ws_bytes < 2 * half) {
        set_error("adlbr_structure_tensor: workspace has %zu bytes, %zu needed", ws_bytes,
                  2 * half);
        return ADLBR_E_NOMEM;
    }
    return tensor_run(gi, u, ncomp, dtype, p, D, (char *)workspace, half, as_stream(stream));
}

extern "C" int adlbr_structure_tensor(const adlbr_grid *g, const void *u, int dtype,
                                      const adlbr_tensor_params *p, void *D, void *workspace,
                                      size_t ws_bytes, void *stream) {
    return adlbr_structure_tensor_vec(g, u, 1, dtype, p, D, workspace, ws_bytes, stream);
}

extern "C" int adlbr_structure_tensor_noalloc(const adlbr_grid *g, const void *u, int dtype,
                                              const adlbr_tensor_params *p, void *D,
                                              void *stream) {
    clear_error();
    GridInfo gi;
    size_t half = 0;
    int rc = tensor_args("adlbr_structure_tensor_noalloc", g, u, dtype, p, D, &gi, &half);
    if (rc) return rc;
    if (2 * half > kNoAllocScratchBytes) {
        set_error("adlbr_structure_tensor_noalloc: needs %zu bytes of scratch, the static "
                  "scratch holds %zu", 2 * half, kNoAllocScratchBytes);
        return ADLBR_E_NOMEM;
    }
    char *b = nullptr;
    rc = scratch_address(&b);
    if (rc) return rc;
    return tensor_run(gi, u, 1, dtype, p, D, b, half, as_stream(stream));
}
