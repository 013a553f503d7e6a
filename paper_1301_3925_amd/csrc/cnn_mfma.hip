// Fused inference kernel of the learned preconditioner in 2D:
//   z = r / diag(K) + N(r),  N = C1^T g1 C2^T g2 C2 g1 C1 applied as four
//   gated 3x3 convolutions 1->16->16->16->1 (expanded weights).
//
// One block computes a 16x16 tile of z.  The four layers run back to back
// in LDS with shrinking halos (r on 24x24, layer outputs on 22x22, 20x20,
// 18x18, 16x16), so r and z cross HBM once per tile and the gates once per
// tile plus halo.  Every layer runs on the matrix cores as an implicit GEMM
// with v_mfma_f32_16x16x16_bf16 (BF16 operands, FP32 accumulation), one
// 16-pixel group per instruction:
//   layer 1 (1 -> 16):  D[co][16 px] = W1[co][16 k = taps 0..8, zero-padded] X[k][px]
//   layers 2, 3:        sum over the 9 taps of W_t[co][16 ci] X_t[ci][16 px]
//   layer 4 (16 -> 1):  the same with only row co = 0 of W_t non-zero.
// The weight operands come pre-packed per lane from adlbr_net_gates.  The gates
// g1, g2 are 8-bit fixed point (g = q / 255, so they stay >= 0 and N stays
// positive semi-definite), staged in LDS once per tile.  Activations are
// stored as BF16 with a 40-byte pixel stride, which makes the 8-byte
// A-operand reads of 16 consecutive pixels bank-conflict free; layer 3
// writes over layer 1's buffer.  Zero padding: every layer's input is 0
// outside the grid.
#include "common.h"

namespace adlbr {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;        // output tile edge
constexpr int kStride = 20;   // shorts per pixel in LDS (16 channels + pad)
constexpr int kR0 = kT + 8;   // r region edge (24)
constexpr int kR1 = kT + 6;   // layer-1 output edge (22), also the g1 region
constexpr int kR2 = kT + 4;   // layer-2 output edge (20), also the g2 region
constexpr int kR3 = kT + 2;   // layer-3 output edge (18)
constexpr int kG = 32;        // gate bytes per point (g1, g2)

// packed weight operands: [layer 1: 64 lanes][layer 2: 9 x 64][layer 3: 9 x 64][layer 4: 9 x 64]
constexpr int kPack1 = 0, kPack2 = 64, kPack3 = 64 + 9 * 64, kPack4 = 64 + 18 * 64;
constexpr int kPackEntries = 64 + 27 * 64;

// round to nearest even BF16 (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ short bfbits(float f) { return __builtin_bit_cast(short, (__bf16)f); }
__device__ __forceinline__ float q8(uint32_t v) { return (float)v * (1.f / 255.f); }

// Pixel (py, px) of region index p of an R x R region, and the next pixel.
template <int R> struct Px {
    int y, x;
    __device__ __forceinline__ explicit Px(int p) : y(p / R), x(p % R) {}
    __device__ __forceinline__ void next() {
        if (++x == R) {
            x = 0;
            ++y;
        }
    }
};

// Store four channels c0 .. c0 + 3 of one pixel, each times its 8-bit
// gate (g4 holds the four gate bytes), as BF16 (one 8-byte LDS write).
__device__ __forceinline__ void store4(short *dst, f32x4 d, uint32_t g4, bool zero) {
    float v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = zero ? 0.f : d[c] * q8((g4 >> (8 * c)) & 0xffu);
    const uint32_t lo = (uint16_t)bfbits(v[0]) | ((uint32_t)(uint16_t)bfbits(v[1]) << 16);
    const uint32_t hi = (uint16_t)bfbits(v[2]) | ((uint32_t)(uint16_t)bfbits(v[3]) << 16);
    *(uint2 *)dst = make_uint2(lo, hi);
}

// One MFMA layer 16 -> 16: input region edge RI (LDS in), output edge RO;
// output gates from sg (LDS, pixel-major [GR * GR][16]; the output region
// sits at offset GO inside the gate region).  The product is taken as
// D[co][px] = W[co][ci] X[ci][px] (weights as the A operand, activations as
// B), so each lane ends with four consecutive channels of one pixel: one
// 4-byte gate read and one 8-byte store.  EDGE: the tile touches the grid
// boundary, so outputs outside the grid are set to 0.
template <int RI, int RO, int GR, int GO, bool EDGE>
__device__ __forceinline__ void mfma_layer(const short *__restrict__ sin, short *__restrict__ sout,
                                           const bf16x4 *wb, int gx0, int gy0, int nx, int ny,
                                           const uint8_t *__restrict__ sg) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int npx = RO * RO;
    constexpr int ngroups = (npx + 15) / 16;
    const int n = lane & 15;            // B column / D column: the pixel in the group
    const int kq = (lane >> 4) * 4;     // channel quad of B (ci) and of D (co)
    for (int grp = wave; grp < ngroups; grp += 4) {
        const int pa = grp * 16 + n;    // this lane's pixel
        const bool va = pa < npx;
        const Px<RO> pxa(va ? pa : 0);
        const short *base = sin + (pxa.y * RI + pxa.x) * kStride + kq;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            bf16x4 b = *(const bf16x4 *)(base + ((t / 3) * RI + (t % 3)) * kStride);
            if (!va) b = bf16x4{0, 0, 0, 0};
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wb[t], b, d, 0, 0, 0);
        }
        if (!va) continue;
        const uint32_t g4 = *(const uint32_t *)(sg + ((pxa.y + GO) * GR + (pxa.x + GO)) * 16 + kq);
        bool zero = false;
        if (EDGE) {
            const int gx = gx0 + pxa.x, gy = gy0 + pxa.y;
            zero = gx < 0 || gx >= nx || gy < 0 || gy >= ny;
        }
        store4(sout + pa * kStride + kq, d, g4, zero);
    }
}

// Inputs of one tile, fetched into registers ahead of time: r on the 24x24
// region (0 outside the grid), g1 on 22x22 and g2 on 20x20 (16 bytes each).
constexpr int kRPer = (kR0 * kR0 + 255) / 256;                  // r values per thread
constexpr int kGPer = (kR1 * kR1 + kR2 * kR2 + 255) / 256;      // gate vectors per thread
struct TileIn {
    float r[kRPer];
    uint4 g[kGPer];
    float rp;  // r_prev at this thread's pixel of the 16x16 tile (fused dots)
};

__device__ __forceinline__ void fetch_tile(int x0, int y0, int nx, int ny,
                                           const float *__restrict__ r,
                                           const uint8_t *__restrict__ G8,
                                           const float *__restrict__ rp, TileIn &in) {
    const int tid = threadIdx.x;
    {
        const int gx = x0 + tid % kT, gy = y0 + tid / kT;
        in.rp = (rp && gx < nx && gy < ny) ? rp[gy * nx + gx] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kRPer; ++j) {
        const int k = tid + 256 * j;
        const int gx = x0 - 4 + k % kR0, gy = y0 - 4 + k / kR0;
        in.r[j] = (k < kR0 * kR0 && gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? r[gy * nx + gx]
                                                                              : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kGPer; ++j) {
        const int k = tid + 256 * j;
        const bool first = k < kR1 * kR1;
        const int kk = first ? k : k - kR1 * kR1;
        const int R = first ? kR1 : kR2, h = first ? 3 : 2;
        const int gx = x0 - h + kk % R, gy = y0 - h + kk / R;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (k < kR1 * kR1 + kR2 * kR2 && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
            v = ((const uint4 *)(G8 + (gy * nx + gx) * kG))[first ? 0 : 1];
        in.g[j] = v;
    }
}

__device__ __forceinline__ void stage_tile(const TileIn &in, float *sr, uint8_t *sg1, uint8_t *sg2,
                                           float *srp) {
    const int tid = threadIdx.x;
    srp[tid] = in.rp;
#pragma unroll
    for (int j = 0; j < kRPer; ++j) {
        const int k = tid + 256 * j;
        if (k < kR0 * kR0) sr[k] = in.r[j];
    }
#pragma unroll
    for (int j = 0; j < kGPer; ++j) {
        const int k = tid + 256 * j;
        if (k < kR1 * kR1) ((uint4 *)sg1)[k] = in.g[j];
        else if (k < kR1 * kR1 + kR2 * kR2) ((uint4 *)sg2)[k - kR1 * kR1] = in.g[j];
    }
}

// The four layers of one staged tile at (x0, y0).  EDGE: the tile's input
// region leaves the grid, so outputs outside the grid are zeroed.
template <bool EDGE>
__device__ __forceinline__ void net_tile(int x0, int y0, int nx, int ny,
                                         const float *__restrict__ F0, float *__restrict__ z,
                                         const float *__restrict__ rp, double &zr, double &zrp,
                                         const bf16x4 &wb1, const bf16x4 *wb2, const bf16x4 *wb3,
                                         const bf16x4 *wb4, const float *sr, const uint8_t *sg1,
                                         const uint8_t *sg2, short *s13, short *s2,
                                         const float *srp) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto inside = [&](int gx, int gy) {
        return !EDGE || (gx >= 0 && gx < nx && gy >= 0 && gy < ny);
    };
    // 1 / diag K at the output pixels of this lane in layer 4 (tile rows
    // wave, wave + 4, ...; lanes 0..15), loaded now so the load overlaps
    // layers 1-3
    float f0v[kT / 4];
#pragma unroll
    for (int j = 0; j < kT / 4; ++j) {
        const int gx = x0 + (lane & 15), gy = y0 + wave + 4 * j;
        f0v[j] = (lane < 16 && (!EDGE || (gx < nx && gy < ny))) ? F0[gy * nx + gx] : 0.f;
    }

    // layer 1 (1 -> 16) on 22x22: D[co][px] = W1[co][tap] X[tap][px], the
    // taps (4 per lane quad, 9..15 zero) as the K dimension
    {
        constexpr int npx = kR1 * kR1;
        const int n = lane & 15, kq = (lane >> 4) * 4;
        for (int grp = wave; grp < (npx + 15) / 16; grp += 4) {
            const int pa = grp * 16 + n;
            const bool va = pa < npx;
            const Px<kR1> pxa(va ? pa : 0);
            const float *rb = sr + pxa.y * kR0 + pxa.x;
            bf16x4 b;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int t = kq + c;
                b[c] = (va && t < 9) ? bfbits(rb[(t / 3) * kR0 + (t % 3)]) : (short)0;
            }
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wb1, b, d, 0, 0, 0);
            if (!va) continue;
            const uint32_t g4 = *(const uint32_t *)(sg1 + pa * 16 + kq);
            store4(s13 + pa * kStride + kq, d, g4, !inside(x0 - 3 + pxa.x, y0 - 3 + pxa.y));
        }
    }
    __syncthreads();
    mfma_layer<kR1, kR2, kR2, 0, EDGE>(s13, s2, wb2, x0 - 2, y0 - 2, nx, ny, sg2);
    __syncthreads();
    mfma_layer<kR2, kR3, kR1, 2, EDGE>(s2, s13, wb3, x0 - 1, y0 - 1, nx, ny, sg1);
    __syncthreads();

    // layer 4 (16 -> 1, no gate) on the 16x16 tile: D[co][px] with only row
    // co = 0 of the weights non-zero, so lanes 0..15 (c = 0) hold the 16
    // pixels of a tile row; then z = r / diag K + N(r)
    {
        const int n = lane & 15, kq = (lane >> 4) * 4;
#pragma unroll
        for (int j = 0; j < kT / 4; ++j) {
            const int grp = wave + 4 * j;  // group grp = one tile row: pixels (grp, 0..15)
            const short *base = s13 + (grp * kR3 + n) * kStride + kq;
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const bf16x4 b = *(const bf16x4 *)(base + ((t / 3) * kR3 + (t % 3)) * kStride);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wb4[t], b, d, 0, 0, 0);
            }
            if (lane < 16) {
                const int gx = x0 + n, gy = y0 + grp;
                if (!EDGE || (gx < nx && gy < ny)) {
                    const int gi = gy * nx + gx;
                    const float rv = sr[(grp + 4) * kR0 + (n + 4)];
                    const float zv = rv * f0v[j] + d[0];
                    z[gi] = zv;
                    zr += (double)zv * (double)rv;
                    if (rp) zrp += (double)zv * (double)srp[grp * kT + n];
                }
            }
        }
    }
}

// Persistent over tiles: every block loads the packed weights once, and
// while it computes one tile the next tile's inputs are already in flight
// into registers (fetch_tile), then staged into LDS (stage_tile).
// With part given, the kernel also leaves the flexible-CG dot products
// <z, r> and <z, rp> (rp may be null) as per-block FP64 partials:
// part[blockIdx.x] and part[gridDim.x + blockIdx.x].
__global__ __launch_bounds__(256) void k_net2d_fused(int nx, int ny, const float *__restrict__ r,
                                                     const float *__restrict__ F0,
                                                     const uint8_t *__restrict__ G8,
                                                     const bf16x4 *__restrict__ wpack,
                                                     float *__restrict__ z,
                                                     const float *__restrict__ rp,
                                                     double *__restrict__ part,
                                                     const CgState *__restrict__ st) {
    if (st && (st->done || st->bad)) return;  // the solve has stopped: nothing reads z
    __shared__ __attribute__((aligned(16))) float sr[kR0 * kR0];
    __shared__ __attribute__((aligned(16))) uint8_t sg1[kR1 * kR1 * 16];
    __shared__ __attribute__((aligned(16))) uint8_t sg2[kR2 * kR2 * 16];
    // layer 1 output, later layer 3 output (s1 is dead once layer 2 has run)
    __shared__ __attribute__((aligned(16))) short s13[kR1 * kR1 * kStride];
    __shared__ __attribute__((aligned(16))) short s2[kR2 * kR2 * kStride];
    __shared__ float srp[kT * kT];
    const int lane = threadIdx.x & 63;
    const int ntx = (nx + kT - 1) / kT, ntiles = ntx * ((ny + kT - 1) / kT);
    // weight operands, packed per lane
    const bf16x4 wb1 = wpack[kPack1 + lane];
    bf16x4 wb2[9], wb3[9], wb4[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        wb2[t] = wpack[kPack2 + t * 64 + lane];
        wb3[t] = wpack[kPack3 + t * 64 + lane];
        wb4[t] = wpack[kPack4 + t * 64 + lane];
    }
    TileIn in;
    double zr = 0.0, zrp = 0.0;
    int tile = blockIdx.x;
    if (tile < ntiles) fetch_tile((tile % ntx) * kT, (tile / ntx) * kT, nx, ny, r, G8, rp, in);
    for (; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % ntx) * kT, y0 = (tile / ntx) * kT;
        __syncthreads();  // the previous tile is done with the LDS buffers
        stage_tile(in, sr, sg1, sg2, srp);
        const int next = tile + gridDim.x;
        if (next < ntiles) fetch_tile((next % ntx) * kT, (next / ntx) * kT, nx, ny, r, G8, rp, in);
        __syncthreads();
        // interior tiles (the 24x24 input region inside the grid) skip every
        // bounds check; the branch is uniform over the block
        if (x0 >= 4 && y0 >= 4 && x0 + kT + 4 <= nx && y0 + kT + 4 <= ny)
            net_tile<false>(x0, y0, nx, ny, F0, z, rp, zr, zrp, wb1, wb2, wb3, wb4, sr, sg1, sg2,
                            s13, s2, srp);
        else
            net_tile<true>(x0, y0, nx, ny, F0, z, rp, zr, zrp, wb1, wb2, wb3, wb4, sr, sg1, sg2,
                           s13, s2, srp);
    }
    if (part) {  // block sums of the dots, in sr's storage (fixed order)
        double *red = (double *)sr;  // 256 doubles fit in the 24 x 24 floats
        for (int k = 0; k < 2; ++k) {
            __syncthreads();
            red[threadIdx.x] = k ? zrp : zr;
            __syncthreads();
            for (int st = 128; st > 0; st >>= 1) {
                if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
                __syncthreads();
            }
            if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = red[0];
        }
    }
}

// Pack the weight operands (expanded weights L1..L4, the A operands of
// D = W X) as BF16 in lane order: for layers 2 and 3 lane holds
// W[co = lane & 15][ci = 4 (lane >> 4) + c][t]; for layer 1
// W1[co = lane & 15][tap = 4 (lane >> 4) + c] (taps >= 9 are 0); for layer 4
// W4[ci = 4 (lane >> 4) + c][t] in row co = 0 only.
__global__ void k_pack_mfma(const float *__restrict__ L1, const float *__restrict__ L2,
                            const float *__restrict__ L3, const float *__restrict__ L4,
                            bf16x4 *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kPackEntries) return;
    const int lane = e % 64;
    const int co = lane & 15, k0 = (lane >> 4) * 4;
    bf16x4 v;
    if (e < kPack2) {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = k0 + c < 9 ? bfbits(L1[co * 9 + k0 + c]) : (short)0;
    } else if (e < kPack4) {
        const bool second = e >= kPack3;
        const int t = ((e - (second ? kPack3 : kPack2)) / 64);
        const float *W = second ? L3 : L2;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = bfbits(W[(co * 16 + k0 + c) * 9 + t]);
    } else {  // A[co = lane & 15][ci = 4 (lane >> 4) + c], only row co = 0 non-zero
        const int t = (e - kPack4) / 64;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = co == 0 ? bfbits(L4[(k0 + c) * 9 + t]) : (short)0;
    }
    out[e] = v;
}


// ------------------------------------------------------------------ 3D --
// The 3D inference runs layer by layer: the thin layers (1 -> 16, 16 -> 1)
// on the vector units, k3PPT points per thread; the two 16 -> 16 layers on the
// matrix cores as implicit GEMMs over 8 x 8 x 8 tiles (27 taps x one
// v_mfma_f32_16x16x16_bf16 per 16-pixel group, the tile plus a one-point
// halo staged in LDS).  Activations cross HBM between layers as BF16
// [N][16] (32 bytes a point), gates as the 8-bit g1, g2 of every point.
constexpr int k3X = 8, k3Y = 8, k3Z = 8;                 // output tile
constexpr int k3HX = k3X + 2, k3HY = k3Y + 2, k3HZ = k3Z + 2;
constexpr int k3Halo = k3HX * k3HY * k3HZ;               // 1000 staged points
constexpr int k3Pts = k3X * k3Y * k3Z;                   // 512 outputs per block
constexpr int k3PPT = k3Pts / 256;                       // points per thread (layers 1, 4)
constexpr int k3GPW = k3Pts / 64;                        // 16-point groups per wave (MFMA)
static_assert(k3Pts % 256 == 0, "whole points per thread");
constexpr int k3T = 27;

__device__ __forceinline__ bool in_grid3(int x, int y, int z, int nx, int ny, int nz) {
    return x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
}

// The tile of block b (8 x 8 x 8 points) and the origin of its halo.
struct Tile3 {
    int x0, y0, z0;  // halo origin = tile origin - 1
};
__device__ __forceinline__ Tile3 tile3(const GridInfo &g, long long b) {
    const int ntx = (g.nx + k3X - 1) / k3X, nty = (g.ny + k3Y - 1) / k3Y;
    Tile3 t;
    t.x0 = (int)(b % ntx) * k3X - 1;
    t.y0 = (int)((b / ntx) % nty) * k3Y - 1;
    t.z0 = (int)(b / ((long long)ntx * nty)) * k3Z - 1;
    return t;
}
// LDS index of tile point p's neighbour at tap t in the halo region.
__device__ __forceinline__ int halo_idx(int p, int t) {
    const int px = p % k3X, py = (p / k3X) % k3Y, pz = p / (k3X * k3Y);
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    return (pz + 1 + dz) * (k3HX * k3HY) + (py + 1 + dy) * k3HX + (px + 1 + dx);
}

// Stage a BF16 [N][16] field over the tile's halo into LDS (STRIDE shorts
// per point, 0 outside the grid), 8 bytes per item: a thread issues kB loads
// before their LDS stores, so the block waits for one round trip to memory
// per kB items instead of one per item (all of them at once by default; a
// kernel short of registers takes fewer).  Needs blockDim.x == 256.
constexpr int k3StageItems = k3Halo * 4, k3StageIters = (k3StageItems + 255) / 256;
template <int STRIDE = kStride, int kB = k3StageIters>
__device__ __forceinline__ void stage3d(const GridInfo &g, const Tile3 &T, const uint2 *__restrict__ in,
                                        short *sx) {
#pragma unroll
    for (int i0 = 0; i0 < k3StageIters; i0 += kB) {
        uint2 v[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const int k = (int)threadIdx.x + 256 * (i0 + j);
            const int h = k >> 2, q = k & 3;
            const int x = T.x0 + h % k3HX, y = T.y0 + (h / k3HX) % k3HY, z = T.z0 + h / (k3HX * k3HY);
            v[j] = make_uint2(0u, 0u);
            if (i0 + j < k3StageIters && k < k3StageItems && in_grid3(x, y, z, g.nx, g.ny, g.nz))
                v[j] = in[4 * (x + (long long)g.nx * (y + (long long)g.ny * z)) + q];
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const int k = (int)threadIdx.x + 256 * (i0 + j);
            if (i0 + j < k3StageIters && k < k3StageItems) *(uint2 *)(sx + (k >> 2) * STRIDE + 4 * (k & 3)) = v[j];
        }
    }
}

// Layer 1: a1[p][co] = g1[p][co] sum_t W1[co][t] r(p + off_t), r = 0 outside
// the grid (tap t = (dz + 1) 9 + (dy + 1) 3 + (dx + 1)); k3PPT points per
// thread of an 8 x 8 x 8 tile, r of the tile and its halo staged in LDS.
__global__ __launch_bounds__(256) void k_net3d_l1(GridInfo g, const float *__restrict__ r,
                                                  const float *__restrict__ W1,
                                                  const uint8_t *__restrict__ G8,
                                                  uint4 *__restrict__ a1,
                                                  const CgState *__restrict__ st) {
    if (st && (st->done || st->bad)) return;
    __shared__ float sr[k3Halo];
    const Tile3 T = tile3(g, blockIdx.x);
    {
        constexpr int kIters = (k3Halo + 255) / 256;
        float v[kIters];  // all loads first, then the LDS stores
#pragma unroll
        for (int it = 0; it < kIters; ++it) {
            const int h = (int)threadIdx.x + 256 * it;
            const int x = T.x0 + h % k3HX, y = T.y0 + (h / k3HX) % k3HY, z = T.z0 + h / (k3HX * k3HY);
            const bool ok = h < k3Halo && in_grid3(x, y, z, g.nx, g.ny, g.nz);
            const float rv = r[ok ? x + (long long)g.nx * (y + (long long)g.ny * z) : 0];
            v[it] = ok ? rv : 0.f;  // a load from point 0 and a select: no branch per item
        }
#pragma unroll
        for (int it = 0; it < kIters; ++it)
            if ((int)threadIdx.x + 256 * it < k3Halo) sr[threadIdx.x + 256 * it] = v[it];
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < k3PPT; ++k) {
    const int p = (int)threadIdx.x + 256 * k;
    const int x = T.x0 + 1 + p % k3X, y = T.y0 + 1 + (p / k3X) % k3Y, z = T.z0 + 1 + p / (k3X * k3Y);
    if (!in_grid3(x, y, z, g.nx, g.ny, g.nz)) continue;
    const long long i = x + (long long)g.nx * (y + (long long)g.ny * z);
    float rv[k3T];
#pragma unroll
    for (int t = 0; t < k3T; ++t) rv[t] = sr[halo_idx(p, t)];
    const uint4 gq = ((const uint4 *)G8)[2 * i];  // g1: bytes 0 .. 15
    const uint32_t gw[4] = {gq.x, gq.y, gq.z, gq.w};
    uint32_t outw[8];
#pragma unroll
    for (int co = 0; co < 16; co += 2) {
        float a0 = 0.f, b0 = 0.f;
#pragma unroll
        for (int t = 0; t < k3T; ++t) {  // uniform weights: scalar loads, SGPR operands
            a0 += W1[co * k3T + t] * rv[t];
            b0 += W1[(co + 1) * k3T + t] * rv[t];
        }
        a0 *= q8((gw[co >> 2] >> (8 * (co & 3))) & 0xffu);
        b0 *= q8((gw[(co + 1) >> 2] >> (8 * ((co + 1) & 3))) & 0xffu);
        outw[co >> 1] = (uint32_t)(uint16_t)bfbits(a0) | ((uint32_t)(uint16_t)bfbits(b0) << 16);
    }
    a1[2 * i] = make_uint4(outw[0], outw[1], outw[2], outw[3]);
    a1[2 * i + 1] = make_uint4(outw[4], outw[5], outw[6], outw[7]);
    }
}

// Layers 2 and 3 (16 -> 16): out[p][co] = g[p][co] sum_t sum_ci W_t[co][ci]
// in(p + off_t)[ci], as D = W_t X_t on the matrix cores.  wpack: the layer's
// 27 A operands, per lane (row co = lane & 15, ci = 4 (lane >> 4) + c);
// goff: byte offset of the gate in each point's 32 gate bytes (0: g1,
// 16: g2).
__global__ __launch_bounds__(256) void k_net3d_mfma(GridInfo g, const uint2 *__restrict__ in,
                                                    const bf16x4 *__restrict__ wpack,
                                                    const uint8_t *__restrict__ G8, int goff,
                                                    uint2 *__restrict__ out,
                                                    const CgState *__restrict__ st) {
    if (st && (st->done || st->bad)) return;
    __shared__ __attribute__((aligned(16))) short sx[k3Halo * kStride];
    const Tile3 T = tile3(g, blockIdx.x);
    const int x0 = T.x0, y0 = T.y0, z0 = T.z0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bf16x4 wb[k3T];
#pragma unroll
    for (int t = 0; t < k3T; ++t) wb[t] = wpack[t * 64 + lane];
    const int n = lane & 15, kq = (lane >> 4) * 4;
    uint32_t gv[k3GPW];  // the gates of this lane's output points, requested before the matrix work
#pragma unroll
    for (int j = 0; j < k3GPW; ++j) {
        const int p = (wave * k3GPW + j) * 16 + n;
        const int x = x0 + 1 + p % k3X, y = y0 + 1 + (p / k3X) % k3Y, z = z0 + 1 + p / (k3X * k3Y);
        const long long i = in_grid3(x, y, z, g.nx, g.ny, g.nz) ? x + (long long)g.nx * (y + (long long)g.ny * z) : 0;
        gv[j] = *(const uint32_t *)(G8 + 32 * i + goff + kq);
    }
    stage3d<kStride, 8>(g, T, in, sx);  // 8 loads in flight: the weights stay in registers
    __syncthreads();
#pragma unroll
    for (int j = 0; j < k3GPW; ++j) {
        const int p = (wave * k3GPW + j) * 16 + n;  // this lane's output point in the tile
        const int px = p % k3X, py = (p / k3X) % k3Y, pz = p / (k3X * k3Y);
        const short *base = sx + ((pz + 1) * (k3HX * k3HY) + (py + 1) * k3HX + (px + 1)) * kStride + kq;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < k3T; ++t) {
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
            const bf16x4 b = *(const bf16x4 *)(base + (dz * (k3HX * k3HY) + dy * k3HX + dx) * kStride);
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wb[t], b, d, 0, 0, 0);
        }
        const int x = x0 + 1 + px, y = y0 + 1 + py, z = z0 + 1 + pz;
        if (!in_grid3(x, y, z, g.nx, g.ny, g.nz)) continue;
        const long long i = x + (long long)g.nx * (y + (long long)g.ny * z);
        const uint32_t g4 = gv[j];
        float v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = d[c] * q8((g4 >> (8 * c)) & 0xffu);
        out[4 * i + (kq >> 2)] =
            make_uint2((uint16_t)bfbits(v[0]) | ((uint32_t)(uint16_t)bfbits(v[1]) << 16),
                       (uint16_t)bfbits(v[2]) | ((uint32_t)(uint16_t)bfbits(v[3]) << 16));
    }
}

// Layer 4 (16 -> 1) and the output: z = F0 r + sum_t sum_ci W4[ci][t]
// a3(p + off_t)[ci], k3PPT points per thread of an 8 x 8 x 8 tile: a3 of the
// tile and its halo staged in LDS (16 channels, 32 bytes a point), the 16
// channels of every tap taken as 8 BF16 pairs by v_dot2c_f32_bf16 (FP32
// accumulation) against the tap's weight pairs, which are uniform (scalar
// loads).  On the matrix cores this layer would use one row of 16.  With
// part, the block's FP64 partials of <z, r> in part[blockIdx] and of
// <z, rp> in part[gridDim + blockIdx].
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_net3d_l4(GridInfo g, const uint2 *__restrict__ a3,
                                                  const uint32_t *__restrict__ w4,
                                                  const float *__restrict__ r,
                                                  const float *__restrict__ F0,
                                                  float *__restrict__ zout,
                                                  const float *__restrict__ rp,
                                                  double *__restrict__ part,
                                                  const CgState *__restrict__ st) {
    if (st && (st->done || st->bad)) return;
    __shared__ __attribute__((aligned(16))) short sx[k3Halo * 16];
    const Tile3 T = tile3(g, blockIdx.x);
    // the outputs' inputs, requested before the staging: loads from point 0
    // for a point outside the grid, dropped below
    int ip[k3PPT];
    bool live[k3PPT];
    float r0[k3PPT], f0[k3PPT], p0[k3PPT];
#pragma unroll
    for (int k = 0; k < k3PPT; ++k) {
        const int p = (int)threadIdx.x + 256 * k;
        const int x = T.x0 + 1 + p % k3X, y = T.y0 + 1 + (p / k3X) % k3Y, z = T.z0 + 1 + p / (k3X * k3Y);
        live[k] = in_grid3(x, y, z, g.nx, g.ny, g.nz);
        ip[k] = live[k] ? (int)(x + (long long)g.nx * (y + (long long)g.ny * z)) : 0;  // N < 2^28
        r0[k] = r[ip[k]];
        f0[k] = F0[ip[k]];
        p0[k] = (rp ? rp : r)[ip[k]];
    }
    stage3d<16>(g, T, a3, sx);
    __syncthreads();
    double zr = 0.0, zrp = 0.0;
#pragma unroll
    for (int k = 0; k < k3PPT; ++k) {
        const int p = (int)threadIdx.x + 256 * k;
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < k3T; ++t) {
            const uint4 *src = (const uint4 *)(sx + halo_idx(p, t) * 16);
            const uint4 lo = src[0], hi = src[1];
            const uint32_t v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
            for (int c = 0; c < 8; ++c)
                acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, v[c]),
                                                      __builtin_bit_cast(bf16x2v, w4[t * 8 + c]), acc,
                                                      false);
        }
        if (live[k]) {
            const float zi = f0[k] * r0[k] + acc;
            zout[ip[k]] = zi;
            zr += (double)zi * (double)r0[k];
            zrp += rp ? (double)zi * (double)p0[k] : 0.0;
        }
    }
    if (part) block_partial_sum2(zr, zrp, part, part + gridDim.x);
}

// The A operands of layers 2 and 3 (3D), per lane: [layer][tap][lane];
// then row 0 of layer 4's, [tap][ci / 4] (the only non-zero row).
constexpr int k3Pack4 = 2 * k3T * 64, k3PackEntries = k3Pack4 + k3T * 4;
__global__ void k_pack_mfma3d(const float *__restrict__ L2, const float *__restrict__ L3,
                              const float *__restrict__ L4, bf16x4 *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k3PackEntries) return;
    if (e >= k3Pack4) {
        const int t = (e - k3Pack4) / 4, q = (e - k3Pack4) % 4;
        bf16x4 v;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = bfbits(L4[(4 * q + c) * k3T + t]);
        out[e] = v;
        return;
    }
    const int lane = e % 64, t = (e / 64) % k3T;
    const float *W = e >= k3T * 64 ? L3 : L2;
    const int co = lane & 15, k0 = (lane >> 4) * 4;
    bf16x4 v;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = bfbits(W[(co * 16 + k0 + c) * k3T + t]);
    out[e] = v;
}

}  // namespace

// Offset (in floats) of the packed MFMA operands inside net->layers (2D).
constexpr size_t kPackOffset = 2 * 16 * 17 * 9;

int net_pack_mfma(const adlbr_net *net, hipStream_t s) {
    const float *L = net->layers;
    const size_t l2 = 16 * 9, l3 = l2 + 16 * 16 * 9, l4 = l3 + 16 * 16 * 9;
    hipLaunchKernelGGL(k_pack_mfma, dim3((kPackEntries + 255) / 256), dim3(256), 0, s, L, L + l2,
                       L + l3, L + l4, (bf16x4 *)(net->layers + kPackOffset));
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

long long net3d_tiles(const GridInfo &g) {
    return (long long)((g.nx + k3X - 1) / k3X) * ((g.ny + k3Y - 1) / k3Y) * ((g.nz + k3Z - 1) / k3Z);
}

// Packed 3D operands sit after the expanded 3D weights (T = 27).
constexpr size_t kPackOffset3 = 2 * 16 * 17 * 27;

int net_pack_mfma3d(const adlbr_net *net, hipStream_t s) {
    const float *L = net->layers;
    const size_t l2 = 16 * 27, l3 = l2 + 16 * 16 * 27, l4 = l3 + 16 * 16 * 27;
    static_assert(k3PackEntries * 2 <= 7168, "the packed operands fit the layers' reserve");
    hipLaunchKernelGGL(k_pack_mfma3d, dim3((k3PackEntries + 255) / 256), dim3(256), 0, s, L + l2,
                       L + l3, L + l4, (bf16x4 *)(net->layers + kPackOffset3));
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

int net_apply_mfma3d(const adlbr_net *net, const adlbr_operator *op, const float *r, float *z,
                     const float *rp, double *part, const CgState *st, hipStream_t s) {
    const GridInfo &g = operator_grid(op);
    const long long N = g.N;
    const float *L = net->layers;  // layer 1's weights come first
    const bf16x4 *pk = (const bf16x4 *)(net->layers + kPackOffset3);
    // activations as BF16 [N][16] in the two halves of the FP32 scratch
    uint4 *A = (uint4 *)net->scratch, *B = (uint4 *)(net->scratch + 8 * N);
    const unsigned nt = (unsigned)net3d_tiles(g);
    hipLaunchKernelGGL(k_net3d_l1, dim3(nt), dim3(256), 0, s, g, r, L, net->gates8, A, st);
    hipLaunchKernelGGL(k_net3d_mfma, dim3(nt), dim3(256), 0, s, g, (const uint2 *)A, pk,
                       net->gates8, 16, (uint2 *)B, st);
    hipLaunchKernelGGL(k_net3d_mfma, dim3(nt), dim3(256), 0, s, g, (const uint2 *)B, pk + k3T * 64,
                       net->gates8, 0, (uint2 *)A, st);
    hipLaunchKernelGGL(k_net3d_l4, dim3(nt), dim3(256), 0, s, g, (const uint2 *)A,
                       (const uint32_t *)(pk + k3Pack4), r, net->features, z, rp, part, st);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

// Blocks of the persistent inference grid for a grid of nx x ny points.
int net_mfma_blocks(int nx, int ny) {
    const int ntiles = ((nx + kT - 1) / kT) * ((ny + kT - 1) / kT);
    // three 51 KB blocks fit one CU's LDS: a persistent grid of 3 per CU
    return ntiles < 3 * 256 ? ntiles : 3 * 256;
}

int net_apply_mfma(const adlbr_net *net, const adlbr_operator *op, const float *r, float *z,
                   const float *rp, double *part, const CgState *st, hipStream_t s) {
    const GridInfo &g = operator_grid(op);
    hipLaunchKernelGGL(k_net2d_fused, dim3(net_mfma_blocks(g.nx, g.ny)), dim3(256), 0, s, g.nx,
                       g.ny, r, net->features, (const uint8_t *)net->gates8,
                       (const bf16x4 *)(net->layers + kPackOffset), z, rp, part, st);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

}  // namespace adlbr
