// Fused inference kernel of the learned preconditioner in 2D:
//   z = r / diag(K) + N(r),  N = C1^T g1 C2^T g2 C2 g1 C1 applied as four
//   gated 3x3 convolutions 1->16->16->16->1 (expanded weights).
//
// One block computes a 16x16 tile of z.  The four layers run back to back
// in LDS with shrinking halos (r on 24x24, layer outputs on 22x22, 20x20,
// 18x18, 16x16), so r, the gates and z each cross HBM once per tile (plus
// halos).  The two 16->16 layers are implicit GEMMs on the matrix cores:
//   out[16 pixels][16 co] += A_t[16 pixels][16 ci] * B_t[16 ci][16 co]
// over the 9 taps t with v_mfma_f32_16x16x16_bf16 (BF16 operands, FP32
// accumulation); the B operands come pre-packed per lane from
// adlbr_net_gates.  The thin 1->16 and 16->1 layers use FP32 FMAs.
// Activations are stored as BF16 with a 40-byte pixel stride, which makes
// the 8-byte A-operand reads of 16 consecutive pixels bank-conflict free;
// layer 3 writes over layer 1's buffer.  Gates are read as BF16 [N][2W]
// (g1, g2).  Zero padding: every layer's input is 0 outside the grid.
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
constexpr int kG = 32;        // gate channels per point (g1, g2)

__device__ __forceinline__ float bfval(short b) { return bf16_to_f32(bf16{(uint16_t)b}); }
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    return (uint32_t)f32_to_bf16(lo).b | ((uint32_t)f32_to_bf16(hi).b << 16);
}

// One MFMA layer 16 -> 16: input region edge RI (LDS in), output edge RO,
// output gates from channel gate_off of the [N][32] gate rows.
template <int RI, int RO>
__device__ __forceinline__ void mfma_layer(const short *__restrict__ sin, short *__restrict__ sout,
                                           const bf16x4 *wb, int gx0, int gy0, int nx, int ny,
                                           const uint16_t *__restrict__ G16, int gate_off) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int npx = RO * RO;
    constexpr int ngroups = (npx + 15) / 16;
    const int i_row = lane & 15;        // A row / D column index
    const int kq = (lane >> 4) * 4;     // channel quad of A, pixel quad of D
    const int co = lane & 15;
    for (int grp = wave; grp < ngroups; grp += 4) {
        const int pa = grp * 16 + i_row;            // this lane's A pixel
        const bool va = pa < npx;
        const int oy = va ? pa / RO : 0, ox = va ? pa % RO : 0;
        // the gates of this lane's four output pixels, fetched before the MFMAs
        float gv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int p = grp * 16 + kq + c;
            const int py = p / RO, px = p % RO;
            const int gx = gx0 + px, gy = gy0 + py;
            gv[c] = (p < npx && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
                        ? bf16_to_f32(bf16{G16[((long long)gy * nx + gx) * kG + gate_off + co]})
                        : 0.f;
        }
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ty = t / 3, tx = t % 3;
            const short *src = sin + ((oy + ty) * RI + (ox + tx)) * kStride + kq;
            bf16x4 a = *(const bf16x4 *)src;
            if (!va) a = bf16x4{0, 0, 0, 0};
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wb[t], d, 0, 0, 0);
        }
        // D: column j = co, rows (pixels) kq..kq+3
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int p = grp * 16 + kq + c;
            if (p < npx) sout[p * kStride + co] = (short)f32_to_bf16(d[c] * gv[c]).b;
        }
    }
}

__global__ __launch_bounds__(256) void k_net2d_fused(int nx, int ny, const float *__restrict__ r,
                                                     const float *__restrict__ F0,
                                                     const uint16_t *__restrict__ G16,
                                                     const float *__restrict__ W1,
                                                     const bf16x4 *__restrict__ wpack,
                                                     const float *__restrict__ W4,
                                                     float *__restrict__ z) {
    __shared__ float sr[kR0 * kR0];
    // layer 1 output, later layer 3 output (s1 is dead once layer 2 has run)
    __shared__ __attribute__((aligned(16))) short s13[kR1 * kR1 * kStride];
    __shared__ __attribute__((aligned(16))) short s2[kR2 * kR2 * kStride];
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
    const int tid = threadIdx.x, lane = tid & 63;

    // r on the 24x24 region, 0 outside the grid
    for (int k = tid; k < kR0 * kR0; k += 256) {
        const int gx = x0 - 4 + k % kR0, gy = y0 - 4 + k / kR0;
        sr[k] = (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? r[(long long)gy * nx + gx] : 0.f;
    }
    // B operands of the two MFMA layers, packed per lane: [layer][t][lane]
    bf16x4 wb2[9], wb3[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        wb2[t] = wpack[t * 64 + lane];
        wb3[t] = wpack[(9 + t) * 64 + lane];
    }
    __syncthreads();

    // layer 1 (1 -> 16, FP32 FMAs) on 22x22, times g1
    for (int k = tid; k < kR1 * kR1; k += 256) {
        const int py = k / kR1, px = k % kR1;
        const int gx = x0 - 3 + px, gy = y0 - 3 + py;
        uint2 *dst = (uint2 *)(s13 + k * kStride);
        if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) {
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = make_uint2(0u, 0u);
            continue;
        }
        float in[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) in[t] = sr[(py + t / 3) * kR0 + (px + t % 3)];
        const uint4 *grow = (const uint4 *)(G16 + ((long long)gy * nx + gx) * kG);
        const uint4 gq0 = grow[0], gq1 = grow[1];  // g1, 16 x BF16
        const uint32_t gw[8] = {gq0.x, gq0.y, gq0.z, gq0.w, gq1.x, gq1.y, gq1.z, gq1.w};
        float o[16];
#pragma unroll
        for (int co = 0; co < 16; ++co) {
            float a = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) a += W1[co * 9 + t] * in[t];
            const uint32_t gb = (co & 1) ? (gw[co >> 1] >> 16) : (gw[co >> 1] & 0xffffu);
            o[co] = a * bf16_to_f32(bf16{(uint16_t)gb});
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            dst[q] = make_uint2(pack2(o[4 * q], o[4 * q + 1]), pack2(o[4 * q + 2], o[4 * q + 3]));
    }
    __syncthreads();
    mfma_layer<kR1, kR2>(s13, s2, wb2, x0 - 2, y0 - 2, nx, ny, G16, 16);
    __syncthreads();
    mfma_layer<kR2, kR3>(s2, s13, wb3, x0 - 1, y0 - 1, nx, ny, G16, 0);
    __syncthreads();

    // layer 4 (16 -> 1, FP32 FMAs, no gate) on the 16x16 tile, then z
    {
        const int py = tid / kT, px = tid % kT;
        const int gx = x0 + px, gy = y0 + py;
        if (gx < nx && gy < ny) {
            float a = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const uint2 *src = (const uint2 *)(s13 + ((py + t / 3) * kR3 + (px + t % 3)) * kStride);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint2 v = src[q];
                    a += W4[(4 * q + 0) * 9 + t] * bfval((short)(v.x & 0xffffu));
                    a += W4[(4 * q + 1) * 9 + t] * bfval((short)(v.x >> 16));
                    a += W4[(4 * q + 2) * 9 + t] * bfval((short)(v.y & 0xffffu));
                    a += W4[(4 * q + 3) * 9 + t] * bfval((short)(v.y >> 16));
                }
            }
            const long long gi = (long long)gy * nx + gx;
            z[gi] = sr[(py + 4) * kR0 + (px + 4)] * F0[gi] + a;
        }
    }
}

// Pack the B operands of the two MFMA layers (expanded weights L2, L3) as
// BF16 in lane order: lane holds W[co = lane & 15][ci = 4 (lane >> 4) + c][t].
__global__ void k_pack_mfma(const float *__restrict__ L2, const float *__restrict__ L3,
                            bf16x4 *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (layer, t, lane)
    if (e >= 2 * 9 * 64) return;
    const int lane = e % 64, t = (e / 64) % 9, layer = e / (64 * 9);
    const float *W = layer ? L3 : L2;
    const int co = lane & 15, ci0 = (lane >> 4) * 4;
    bf16x4 v;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (short)f32_to_bf16(W[(co * 16 + ci0 + c) * 9 + t]).b;
    out[e] = v;
}

}  // namespace

// Offset (in floats) of the packed MFMA operands inside net->layers (2D).
constexpr size_t kPackOffset = 2 * 16 * 17 * 9;

int net_pack_mfma(const adlbr_net *net, hipStream_t s) {
    const float *L = net->layers;
    const size_t l2 = 16 * 9, l3 = l2 + 16 * 16 * 9;
    hipLaunchKernelGGL(k_pack_mfma, dim3((2 * 9 * 64 + 255) / 256), dim3(256), 0, s, L + l2, L + l3,
                       (bf16x4 *)(net->layers + kPackOffset));
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

int net_apply_mfma(const adlbr_net *net, const adlbr_operator *op, const float *r, float *z,
                   hipStream_t s) {
    const GridInfo &g = operator_grid(op);
    const float *L = net->layers;
    // expanded layer offsets for dim 2, width 16: [W1, W2, W3, W4, packed B operands]
    const size_t l4 = 16 * 9 + 2 * 16 * 16 * 9;
    dim3 grid((g.nx + kT - 1) / kT, (g.ny + kT - 1) / kT);
    hipLaunchKernelGGL(k_net2d_fused, grid, dim3(256), 0, s, g.nx, g.ny, r, net->features,
                       net->gates16, L, (const bf16x4 *)(L + kPackOffset), L + l4, z);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

}  // namespace adlbr
