// Fused inference kernel of the learned preconditioner in 2D:
//   z = r / diag(K) + N(r),  N = four gated 3x3 convolutions 1->16->16->16->1.
//
// One block computes a 16x16 tile of z.  The four layers run back to back
// in LDS with shrinking halos (r on 24x24, layer outputs on 22x22, 20x20,
// 18x18, 16x16), so r, the gates and z each cross HBM once per tile.  The
// two 16->16 layers are implicit GEMMs on the matrix cores:
//   out[16 pixels][16 co] += A_t[16 pixels][16 ci] * B_t[16 ci][16 co]
// over the 9 taps t with v_mfma_f32_16x16x16_bf16 (BF16 operands, FP32
// accumulation); the thin 1->16 and 16->1 layers use FP32 FMAs.
// Activations are stored as BF16 with a 40-byte pixel stride, which makes
// the 8-byte A-operand reads of 16 consecutive pixels bank-conflict free.
// Zero padding: every layer's input is 0 outside the grid.
#include "common.h"

namespace adlbr {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;        // output tile edge
constexpr int kStride = 20;   // shorts per pixel in LDS (16 channels + pad)
constexpr int kR0 = kT + 8;   // r region edge (24)
constexpr int kR1 = kT + 6;   // layer-1 output edge (22)
constexpr int kR2 = kT + 4;   // layer-2 output edge (20)
constexpr int kR3 = kT + 2;   // layer-3 output edge (18)
constexpr int kG = 49;        // gate channels per point

__device__ __forceinline__ short bfbits(float f) { return (short)f32_to_bf16(f).b; }
__device__ __forceinline__ float bfval(short b) { return bf16_to_f32(bf16{(uint16_t)b}); }

// One MFMA layer 16 -> 16: input region edge RI (LDS in), output edge RO.
template <int RI, int RO>
__device__ __forceinline__ void mfma_layer(const short *__restrict__ sin, short *__restrict__ sout,
                                           const bf16x4 *wb, int gx0, int gy0, int nx, int ny,
                                           const uint16_t *__restrict__ G16, int gate_off) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int npx = RO * RO;
    constexpr int ngroups = (npx + 15) / 16;
    const int i_row = lane & 15;        // A row / D column index
    const int kq = (lane >> 4) * 4;     // channel quad of A, pixel quad of D
    for (int grp = wave; grp < ngroups; grp += 4) {
        const int pa = grp * 16 + i_row;            // this lane's A pixel
        const bool va = pa < npx;
        const int oy = va ? pa / RO : 0, ox = va ? pa % RO : 0;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ty = t / 3, tx = t % 3;
            const short *src = sin + ((oy + ty) * RI + (ox + tx)) * kStride + kq;
            bf16x4 a = *(const bf16x4 *)src;
            if (!va) a = bf16x4{0, 0, 0, 0};
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wb[t], d, 0, 0, 0);
        }
        // D: column j = co = lane & 15, rows (pixels) kq..kq+3
        const int co = lane & 15;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int p = grp * 16 + kq + c;
            if (p >= npx) continue;
            const int py = p / RO, px = p % RO;
            const int gx = gx0 + px, gy = gy0 + py;
            float v = 0.f;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const long long gi = (long long)gy * nx + gx;
                v = d[c] * bf16_to_f32(bf16{G16[gi * kG + gate_off + co]});
            }
            sout[p * kStride + co] = bfbits(v);
        }
    }
}

__global__ __launch_bounds__(256) void k_net2d_fused(int nx, int ny, const float *__restrict__ r,
                                                     const float *__restrict__ F0,
                                                     const uint16_t *__restrict__ G16,
                                                     const float *__restrict__ W1,
                                                     const float *__restrict__ W2,
                                                     const float *__restrict__ W3,
                                                     const float *__restrict__ W4,
                                                     float *__restrict__ z) {
    __shared__ float sr[kR0 * kR0];
    __shared__ __attribute__((aligned(16))) short s1[kR1 * kR1 * kStride];
    __shared__ __attribute__((aligned(16))) short s2[kR2 * kR2 * kStride];
    __shared__ __attribute__((aligned(16))) short s3[kR3 * kR3 * kStride];
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
    const int tid = threadIdx.x, lane = tid & 63;

    // r on the 24x24 region, 0 outside the grid
    for (int k = tid; k < kR0 * kR0; k += 256) {
        const int gx = x0 - 4 + k % kR0, gy = y0 - 4 + k / kR0;
        sr[k] = (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? r[(long long)gy * nx + gx] : 0.f;
    }
    // B operands of the two MFMA layers: lane holds W[co = lane&15][ci = 4(lane>>4)+c][t]
    bf16x4 wb2[9], wb3[9];
    {
        const int co = lane & 15, ci0 = (lane >> 4) * 4;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                wb2[t][c] = bfbits(W2[(co * 16 + ci0 + c) * 9 + t]);
                wb3[t][c] = bfbits(W3[(co * 16 + ci0 + c) * 9 + t]);
            }
        }
    }
    __syncthreads();

    // layer 1 (1 -> 16, FP32 FMAs) on 22x22, times gates 0..15
    for (int k = tid; k < kR1 * kR1; k += 256) {
        const int py = k / kR1, px = k % kR1;
        const int gx = x0 - 3 + px, gy = y0 - 3 + py;
        short *dst = s1 + k * kStride;
        if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) {
#pragma unroll
            for (int co = 0; co < 16; ++co) dst[co] = 0;
            continue;
        }
        float in[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) in[t] = sr[(py + t / 3) * kR0 + (px + t % 3)];
        const long long gi = (long long)gy * nx + gx;
#pragma unroll
        for (int co = 0; co < 16; ++co) {
            float a = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) a += W1[co * 9 + t] * in[t];
            dst[co] = bfbits(a * bf16_to_f32(bf16{G16[gi * kG + co]}));
        }
    }
    __syncthreads();
    mfma_layer<kR1, kR2>(s1, s2, wb2, x0 - 2, y0 - 2, nx, ny, G16, 16);
    __syncthreads();
    mfma_layer<kR2, kR3>(s2, s3, wb3, x0 - 1, y0 - 1, nx, ny, G16, 32);
    __syncthreads();

    // layer 4 (16 -> 1, FP32 FMAs) on the 16x16 tile, gate 48, then z
    {
        const int py = tid / kT, px = tid % kT;
        const int gx = x0 + px, gy = y0 + py;
        if (gx < nx && gy < ny) {
            float a = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const short *src = s3 + ((py + t / 3) * kR3 + (px + t % 3)) * kStride;
#pragma unroll
                for (int ci = 0; ci < 16; ++ci) a += W4[ci * 9 + t] * bfval(src[ci]);
            }
            const long long gi = (long long)gy * nx + gx;
            const float o = a * bf16_to_f32(bf16{G16[gi * kG + 48]});
            z[gi] = sr[(py + 4) * kR0 + (px + 4)] * F0[gi] + o;
        }
    }
}

}  // namespace

int net_apply_mfma(const adlbr_net *net, const adlbr_operator *op, const float *r, float *z,
                   hipStream_t s) {
    const GridInfo &g = operator_grid(op);
    const float *L = net->layers;
    // expanded layer offsets for dim 2, width 16: [W1, W2, W3, W4]
    const size_t l2 = 16 * 9, l3 = l2 + 16 * 16 * 9, l4 = l3 + 16 * 16 * 9;
    dim3 grid((g.nx + kT - 1) / kT, (g.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_net2d_fused, grid, dim3(256), 0, s, g.nx, g.ny, r, net->features,
                       net->gates16, L, L + l2, L + l3, L + l4, z);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

}  // namespace adlbr
