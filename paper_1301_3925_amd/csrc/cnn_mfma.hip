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
//   layer 1 (1 -> 16):  A[16 px][16 k = taps 0..8, zero-padded] x B[k][co]
//   layers 2, 3:        sum over the 9 taps of A_t[16 px][16 ci] x B_t[ci][co]
//   layer 4 (16 -> 1):  the same with only column co = 0 of B_t non-zero.
// The B operands come pre-packed per lane from adlbr_net_gates.  The gates
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

// packed B operands: [layer 1: 64 lanes][layer 2: 9 x 64][layer 3: 9 x 64][layer 4: 9 x 64]
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

// One MFMA layer 16 -> 16: input region edge RI (LDS in), output edge RO;
// output gates from sg (LDS, pixel-major [GR * GR][16]; the output region
// sits at offset GO inside the gate region).  EDGE: the tile touches the
// grid boundary, so outputs outside the grid are set to 0.
template <int RI, int RO, int GR, int GO, bool EDGE>
__device__ __forceinline__ void mfma_layer(const short *__restrict__ sin, short *__restrict__ sout,
                                           const bf16x4 *wb, int gx0, int gy0, int nx, int ny,
                                           const uint8_t *__restrict__ sg) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int npx = RO * RO;
    constexpr int ngroups = (npx + 15) / 16;
    const int i_row = lane & 15;        // A row / D column index
    const int kq = (lane >> 4) * 4;     // channel quad of A, pixel quad of D
    const int co = lane & 15;
    for (int grp = wave; grp < ngroups; grp += 4) {
        const int pa = grp * 16 + i_row;            // this lane's A pixel
        const bool va = pa < npx;
        const Px<RO> pxa(va ? pa : 0);
        const short *base = sin + (pxa.y * RI + pxa.x) * kStride + kq;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            bf16x4 a = *(const bf16x4 *)(base + ((t / 3) * RI + (t % 3)) * kStride);
            if (!va) a = bf16x4{0, 0, 0, 0};
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wb[t], d, 0, 0, 0);
        }
        // D: column co, rows (pixels) p0 .. p0 + 3
        const int p0 = grp * 16 + kq;
        Px<RO> q(p0 < npx ? p0 : 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (p0 + c < npx) {
                float v = d[c] * q8(sg[((q.y + GO) * GR + (q.x + GO)) * 16 + co]);
                if (EDGE) {
                    const int gx = gx0 + q.x, gy = gy0 + q.y;
                    if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) v = 0.f;
                }
                sout[(p0 + c) * kStride + co] = bfbits(v);
            }
            q.next();
        }
    }
}

template <bool EDGE>
__device__ __forceinline__ void net_tile(int nx, int ny, const float *__restrict__ r,
                                         const float *__restrict__ F0,
                                         const uint8_t *__restrict__ G8,
                                         const bf16x4 *__restrict__ wpack, float *__restrict__ z,
                                         float *sr, uint8_t *sg1, uint8_t *sg2, short *s13,
                                         short *s2) {
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto inside = [&](int gx, int gy) {
        return !EDGE || (gx >= 0 && gx < nx && gy >= 0 && gy < ny);
    };
    // r on the 24x24 region, 0 outside the grid; g1 on 22x22, g2 on 20x20
    for (int k = tid; k < kR0 * kR0; k += 256) {
        const int gx = x0 - 4 + k % kR0, gy = y0 - 4 + k / kR0;
        sr[k] = inside(gx, gy) ? r[gy * nx + gx] : 0.f;
    }
    for (int k = tid; k < kR1 * kR1 + kR2 * kR2; k += 256) {
        const bool first = k < kR1 * kR1;
        const int kk = first ? k : k - kR1 * kR1;
        const int R = first ? kR1 : kR2, h = first ? 3 : 2;
        const int gx = x0 - h + kk % R, gy = y0 - h + kk / R;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (inside(gx, gy)) v = ((const uint4 *)(G8 + (gy * nx + gx) * kG))[first ? 0 : 1];
        ((uint4 *)(first ? sg1 : sg2))[kk] = v;
    }
    // B operands, packed per lane
    const bf16x4 wb1 = wpack[kPack1 + lane];
    bf16x4 wb2[9], wb3[9], wb4[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        wb2[t] = wpack[kPack2 + t * 64 + lane];
        wb3[t] = wpack[kPack3 + t * 64 + lane];
        wb4[t] = wpack[kPack4 + t * 64 + lane];
    }
    __syncthreads();

    // layer 1 (1 -> 16) on 22x22: A row = pixel, k = tap (4 per lane quad)
    {
        constexpr int npx = kR1 * kR1;
        const int i_row = lane & 15, kq = (lane >> 4) * 4, co = lane & 15;
        for (int grp = wave; grp < (npx + 15) / 16; grp += 4) {
            const int pa = grp * 16 + i_row;
            const bool va = pa < npx;
            const Px<kR1> pxa(va ? pa : 0);
            const float *rb = sr + pxa.y * kR0 + pxa.x;
            bf16x4 a;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int t = kq + c;  // taps 9..15 and pixels past the end are 0
                a[c] = (va && t < 9) ? bfbits(rb[(t / 3) * kR0 + (t % 3)]) : (short)0;
            }
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wb1, d, 0, 0, 0);
            const int p0 = grp * 16 + kq;
            Px<kR1> q(p0 < npx ? p0 : 0);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (p0 + c < npx) {
                    float v = d[c] * q8(sg1[(p0 + c) * 16 + co]);
                    if (!inside(x0 - 3 + q.x, y0 - 3 + q.y)) v = 0.f;
                    s13[(p0 + c) * kStride + co] = bfbits(v);
                }
                q.next();
            }
        }
    }
    __syncthreads();
    mfma_layer<kR1, kR2, kR2, 0, EDGE>(s13, s2, wb2, x0 - 2, y0 - 2, nx, ny, sg2);
    __syncthreads();
    mfma_layer<kR2, kR3, kR1, 2, EDGE>(s2, s13, wb3, x0 - 1, y0 - 1, nx, ny, sg1);
    __syncthreads();

    // layer 4 (16 -> 1, no gate) on the 16x16 tile; column 0 of D is the
    // output, then z = r / diag K + N(r)
    {
        const int i_row = lane & 15, kq = (lane >> 4) * 4;
        for (int grp = wave; grp < (kT * kT) / 16; grp += 4) {
            // group grp = one tile row: pixels (grp, 0..15)
            const short *base = s13 + (grp * kR3 + i_row) * kStride + kq;
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const bf16x4 a = *(const bf16x4 *)(base + ((t / 3) * kR3 + (t % 3)) * kStride);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wb4[t], d, 0, 0, 0);
            }
            if ((lane & 15) == 0) {
                const int gy = y0 + grp;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int gx = x0 + kq + c;
                    if (!EDGE || (gx < nx && gy < ny)) {
                        const int gi = gy * nx + gx;
                        z[gi] = sr[(grp + 4) * kR0 + (kq + c + 4)] * F0[gi] + d[c];
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_net2d_fused(int nx, int ny, const float *__restrict__ r,
                                                     const float *__restrict__ F0,
                                                     const uint8_t *__restrict__ G8,
                                                     const bf16x4 *__restrict__ wpack,
                                                     float *__restrict__ z) {
    __shared__ float sr[kR0 * kR0];
    __shared__ __attribute__((aligned(16))) uint8_t sg1[kR1 * kR1 * 16];
    __shared__ __attribute__((aligned(16))) uint8_t sg2[kR2 * kR2 * 16];
    // layer 1 output, later layer 3 output (s1 is dead once layer 2 has run)
    __shared__ __attribute__((aligned(16))) short s13[kR1 * kR1 * kStride];
    __shared__ __attribute__((aligned(16))) short s2[kR2 * kR2 * kStride];
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
    // interior tiles (the 24x24 input region inside the grid) skip every
    // bounds check; the branch is uniform over the block
    if (x0 >= 4 && y0 >= 4 && x0 + kT + 4 <= nx && y0 + kT + 4 <= ny)
        net_tile<false>(nx, ny, r, F0, G8, wpack, z, sr, sg1, sg2, s13, s2);
    else
        net_tile<true>(nx, ny, r, F0, G8, wpack, z, sr, sg1, sg2, s13, s2);
}

// Pack the B operands (expanded weights L1..L4) as BF16 in lane order: for
// layers 2 and 3 lane holds W[co = lane & 15][ci = 4 (lane >> 4) + c][t];
// for layer 1 W1[co = lane & 15][tap = 4 (lane >> 4) + c] (taps >= 9 are 0);
// for layer 4 W4[ci = 4 (lane >> 4) + c][t] in column co = 0 only.
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
    } else {
        const int t = (e - kPack4) / 64;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = co == 0 ? bfbits(L4[(k0 + c) * 9 + t]) : (short)0;
    }
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

int net_apply_mfma(const adlbr_net *net, const adlbr_operator *op, const float *r, float *z,
                   hipStream_t s) {
    const GridInfo &g = operator_grid(op);
    dim3 grid((g.nx + kT - 1) / kT, (g.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_net2d_fused, grid, dim3(256), 0, s, g.nx, g.ny, r, net->features,
                       (const uint8_t *)net->gates8,
                       (const bf16x4 *)(net->layers + kPackOffset), z);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

}  // namespace adlbr
