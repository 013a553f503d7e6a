// Internal helpers shared by the HIP sources of libadlbr.so (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "adlbr.h"

namespace adlbr {

typedef long long ll;

// ---------------------------------------------------------------- errors --
void set_error(const char *fmt, ...);
void clear_error();

#define ADLBR_CHECK_HIP(expr)                                                  \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            ::adlbr::set_error("%s failed: %s", #expr, hipGetErrorString(e_)); \
            return ADLBR_E_HIP;                                                \
        }                                                                      \
    } while (0)

#define ADLBR_LAUNCH_CHECK()                                                   \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) {                                                \
            ::adlbr::set_error("kernel launch failed: %s", hipGetErrorString(e_)); \
            return ADLBR_E_HIP;                                                \
        }                                                                      \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Two timing events, destroyed on every exit path of the function that
// holds them.
struct EventPair {
    hipEvent_t e[2] = {nullptr, nullptr};
    hipError_t create() {
        hipError_t r = hipEventCreate(&e[0]);
        return r == hipSuccess ? hipEventCreate(&e[1]) : r;
    }
    ~EventPair() {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// ------------------------------------------------------------------ grid --
struct GridInfo {
    int dim;
    int periodic;
    int nx, ny, nz;
    long long N;
};

int check_grid(const adlbr_grid *g, GridInfo *gi);

// --------------------------------------------------------- 16-bit storage --
struct bf16 { uint16_t b; };

__host__ __device__ inline float bf16_to_f32(bf16 v) {
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)v.b << 16;
    return c.f;
}

__host__ __device__ inline bf16 f32_to_bf16(float f) {
    union { uint32_t u; float f; } c;
    c.f = f;
    uint32_t u = c.u;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) {
        return bf16{(uint16_t)((u >> 16) | 0x40)};  // quiet NaN
    }
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return bf16{(uint16_t)(u >> 16)};
}

// load storage type -> arithmetic type, and back (round to nearest even)
template <typename TS, typename TA> struct Conv;
template <> struct Conv<double, double> {
    __device__ static double ld(double v) { return v; }
    __device__ static double st(double v) { return v; }
};
template <> struct Conv<float, float> {
    __device__ static float ld(float v) { return v; }
    __device__ static float st(float v) { return v; }
};
template <> struct Conv<float, double> {
    __device__ static double ld(float v) { return (double)v; }
    __device__ static float st(double v) { return (float)v; }
};
template <> struct Conv<bf16, float> {
    __device__ static float ld(bf16 v) { return bf16_to_f32(v); }
    __device__ static bf16 st(float v) { return f32_to_bf16(v); }
};
template <> struct Conv<_Float16, float> {
    __device__ static float ld(_Float16 v) { return (float)v; }
    __device__ static _Float16 st(float v) { return (_Float16)v; }
};

inline size_t dtype_size(int dt) {
    switch (dt) {
    case ADLBR_F64: return 8;
    case ADLBR_F32: return 4;
    case ADLBR_BF16:
    case ADLBR_F16: return 2;
    default: return 0;
    }
}

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// ------------------------------------------------------- status helpers --
__global__ void k_status_init(int32_t *status);
__global__ void k_status_final(int32_t *status);

__device__ inline void report(int32_t *status, long long z, int flags) {
    if (!status || !flags) return;
    if (flags & (ADLBR_ST_NOT_SPD | ADLBR_ST_RANGE | ADLBR_ST_ITER | ADLBR_ST_STENCIL |
                 ADLBR_ST_INCOMING))
        atomicMin(&status[0], (int32_t)z);
    atomicOr(&status[1], flags);
}

// Blocks are dispatched round-robin over the 8 XCDs of an MI355X; remap the
// hardware block id so that XCD k works on one contiguous range of logical
// blocks (neighbouring rows share that XCD's L2).
__device__ inline long long xcd_block(long long b, long long nb) {
    const long long nx = 8;
    long long q = nb / nx, r = nb % nx;
    long long k = b % nx, j = b / nx;
    long long start = k * q + (k < r ? k : r);
    return start + j;
}

// 3D traversal in strips of kStripZ planes.  With blocks taken plane after
// plane, a block's neighbours one plane up or down were last touched a whole
// plane of blocks ago and have left the L2 by then.  When a plane is a whole
// number BP of blocks, logical block L is sent instead to a strip of kStripZ
// planes (fewer for the last strip) walked column by column: within a strip,
// the blocks at one in-plane position j of all its planes come one after
// the other, so blocks one plane apart run close together in time.  The
// map is a bijection of [0, nblocks).
#ifndef ADLBR_STRIP_Z
#define ADLBR_STRIP_Z 32
#endif
constexpr int kStripZ = ADLBR_STRIP_Z;

__device__ inline long long strip_block(long long L, const GridInfo &g, int points_per_block) {
    if (g.dim != 3 || kStripZ <= 1) return L;
    const unsigned plane = (unsigned)g.nx * (unsigned)g.ny;  // N < 2^28
    if (plane % (unsigned)points_per_block) return L;
    const unsigned bp = plane / (unsigned)points_per_block;
    const unsigned strip = (unsigned)kStripZ * bp;
    const unsigned s = (unsigned)L / strip;
    const unsigned z0 = s * (unsigned)kStripZ;
    const unsigned tz = min((unsigned)kStripZ, (unsigned)g.nz - z0);
    const unsigned i = (unsigned)L - s * strip;
    const unsigned j = i / tz, z = z0 + i % tz;
    return (long long)z * bp + j;
}

// Index of weight q of point z in an operator's weights.  2D (S = 3):
// point-major [N][3], so that the gather of an incoming edge's weight from
// its source finds the source's three weights on one line.  3D (S = 6),
// with ADLBR_W3D_INLINE (the default): slot-major planes [6][N], read
// coalesced by the own part only, and every incoming entry carries its
// weight beside it (an 8-byte record in FP32).  Without it the 3D weights
// are point-major too and gathered from the source, 4 bytes less per
// incoming edge but slower (256^3 step 709 -> 911 us).
#ifndef ADLBR_W3D_INLINE
#define ADLBR_W3D_INLINE 1
#endif
template <int S> __host__ __device__ __forceinline__ long long widx(int q, long long z, long long N) {
    return S == 3 || !ADLBR_W3D_INLINE ? z * S + q : (long long)q * N + z;
}
template <int S> __host__ __device__ __forceinline__ unsigned widx32(int q, int z, int N) {
    return S == 3 || !ADLBR_W3D_INLINE ? (unsigned)(z * S + q) : (unsigned)(q * N + z);
}

// First point of the calling wave's P consecutive 64-point groups in block
// blk.  Blocks cover 256 P consecutive points, except on a 2D grid whose
// rows are whole groups and whose row count is a multiple of 4 (with
// P = 1): there a block takes a 64 x 4 patch, its four waves one row apart,
// so that their neighbour gathers share the CU's L1 (2D apply on 2048^2:
// 124 -> 109 us).  Same block count either way.
__device__ __forceinline__ long long wave_group(const GridInfo &g, long long blk, int P) {
    const long long wv = threadIdx.x >> 6;
    if (P == 1 && g.dim == 2 && g.nx % 64 == 0 && g.ny % 4 == 0) {
        // 32-bit division (blocks < 2^22 for N < 2^28): a 64-bit one by a
        // runtime divisor costs a long scalar sequence in every wave
        const unsigned gpr = (unsigned)g.nx / 64u, b = (unsigned)blk;
        const unsigned by = b / gpr, bx = b - by * gpr;
        return (long long)(by * 4u + (unsigned)wv) * g.nx + (long long)bx * 64;
    }
    return blk * 256 * P + wv * 64 * P;
}

// Device-resident scalars of a (flexible) conjugate-gradient iteration.
struct CgState {
    double dt;      // K = I + dt A
    double rz;      // <z_k, r_k>
    double rz_old;  // <z_{k-1}, r_{k-1}>
    double zr_prev; // <z_k, r_{k-1}> (flexible CG)
    double pq;      // <p_k, K p_k>
    double alpha, beta;
    double rr;      // |r_k|^2
    double bb;      // |b|^2
    int32_t bad;    // non-descent direction or non-finite value
    int32_t iter;
    int32_t done;   // recurrence residual below tolerance: later kernels are no-ops
    int32_t pad;
};

struct adlbr_net_impl;
// Learned preconditioner z = N(r) for K = I + dt A (defined with the CNN).
int net_apply(const adlbr_net *net, const adlbr_operator *op, double dt, const void *r, void *z,
              hipStream_t s);
// z = preconditioned r (FP32) and the per-block FP64 partials of <z, r> in
// part[0 .. nparts) and of <z, rp> in part[nparts .. 2 nparts) (rp may be
// null); nparts (host out) depends on the inference path taken.  st (may be
// null): a solver state whose done or bad flag turns the fused inference
// into a no-op (the solver's later kernels ignore z and the partials then).
int net_apply_dots(const adlbr_net *net, const adlbr_operator *op, const float *r,
                   const float *rp, float *z, double *part, long long *nparts,
                   const CgState *st, hipStream_t s);

// Rows per block of the explicit-step kernels: every wave of a 256-thread
// block takes kApplyPPT groups of 64 consecutive rows.
constexpr int kApplyPPT = 1;
constexpr int kApplyPoints = 256 * kApplyPPT;

// Device descriptor of one problem of a batch (one operator and its two
// state buffers); first_block is the problem's first block in the batch's
// grid, nblocks its number of blocks and block_points the points a block
// covers in linear order (kApplyPoints rows for the list layout, one tile
// for the tiled layout).
struct BatchProb {
    GridInfo g;
    const void *sb;
    const void *w;
    const uint8_t *cnt;
    const int32_t *pos;
    const int32_t *ent;
    const void *went;
    const double *dtcfl;
    void *u[2];
    double dt;
    int32_t dt_mode;
    int32_t block_points;
    long long first_block;
    long long nblocks;
    const int32_t *hnear;    // tiled layout: halo of the near edges
    const double *maxdiag;   // tiled layout: max A_zz (fixed-point scale)
};
// Blocks of one explicit step of op, and the points each covers.
long long batch_blocks(const adlbr_operator *op, int *block_points);
// Class of an operator for batching (dim, offset width, boundary, storage):
// problems of one class share a kernel instance.
int batch_class(const adlbr_operator *op);
// Fill the operator part of a descriptor.
void batch_describe(const adlbr_operator *op, BatchProb *d);
// Device bytes one explicit step of op reads or writes (u, its successor and
// the operator's arrays), the working set that cache blocking budgets for.
size_t batch_footprint(const adlbr_operator *op);

// One step of the problems of one class (rep: any operator of the class):
// an explicit step from u[parity] to u[parity ^ 1], or (copy) u[0] = u[1].
// probs / hprobs: the descriptors on the device / on the host, in the same
// order.  variant bit 0: XCD-contiguous block order of the grouped launch;
// bit 2: one launch per problem instead of the grouped launch.
int batch_launch(const adlbr_operator *rep, const BatchProb *probs, const BatchProb *hprobs,
                 int nprob, long long nblocks, int parity, int variant, int copy, hipStream_t s);

// Internal entry points shared between translation units.
// Direction update q = K z + beta q, p = z + beta p and alpha = <z,r>/<p,q>
// (partial: one double per 256-point block).
int cg_direction(const adlbr_operator *op, const void *z, void *q, void *p, CgState *st,
                 double *partial, int first, hipStream_t s);
// |b - (I + dt A) x|^2 for an FP64 iterate x, accumulated in FP64 into
// *out (deterministic); the residual itself goes to rout (storage dtype) if
// rout is not null.  partial: one double per 256-point block.
int true_residual(const adlbr_operator *op, double dt, const void *b, const double *x,
                  double *out, double *partial, void *rout, hipStream_t s);

// Reductions are two-phase and atomic-free: every block of a grid-wide
// kernel writes its partial (block_partial_sum), then a one-block finisher
// kernel sums the partials in a fixed order (reduce_partials).  Same-address
// device-scope atomics serialize across the XCDs, so a "last block
// finishes" ticket costs far more than the extra launch; the fixed order
// also makes every reduction deterministic.
// Block sum of v over the block's threads (blockDim.x == 256) into
// partial[blockIdx.x].  All threads must call it.
__device__ inline void block_partial_sum(double v, double *partial) {
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
    __syncthreads();  // red[] may be reused by a second call
}

// Block sums of a and b into pa[blockIdx.x] and pb[blockIdx.x] in one pass
// (blockDim.x == 256): butterfly sums within each wave, then the four wave
// sums in wave order; fixed order, so deterministic.
__device__ inline void block_partial_sum2(double a, double b, double *pa, double *pb) {
    __shared__ double red2[2][4];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        a += __shfl_xor(a, d, 64);
        b += __shfl_xor(b, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red2[0][threadIdx.x >> 6] = a;
        red2[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        pa[blockIdx.x] = ((red2[0][0] + red2[0][1]) + red2[0][2]) + red2[0][3];
        pb[blockIdx.x] = ((red2[1][0] + red2[1][1]) + red2[1][2]) + red2[1][3];
    }
}

// Block maximum of v into partial[blockIdx.x] (blockDim.x == 256).
__device__ inline void block_partial_max(double v, double *partial) {
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
    __syncthreads();
}

// Sum (or max, when take_max) of partial[0 .. n) by a single block of 256
// threads in a fixed order; every thread gets the result.
__device__ inline double reduce_partials(const double *partial, long long n, bool take_max = false) {
    __shared__ double red[256];
    double acc = take_max ? -1.0e308 : 0.0;
    long long b = threadIdx.x;
    // eight independent loads in flight, then added in the same order as a
    // plain strided loop would
    for (; b + 7 * 256 < n; b += 8 * 256) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = partial[b + 256 * j];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc = take_max ? fmax(acc, v[j]) : acc + v[j];
    }
    for (; b < n; b += 256) acc = take_max ? fmax(acc, partial[b]) : acc + partial[b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            red[threadIdx.x] = take_max ? fmax(red[threadIdx.x], red[threadIdx.x + s])
                                        : red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

const GridInfo &operator_grid(const adlbr_operator *op);
int operator_storage(const adlbr_operator *op);
const void *operator_diag(const adlbr_operator *op);
// The operator's weights, in the storage dtype, at widx<S>(q, z, N).
const void *operator_weights(const adlbr_operator *op);
const void *operator_slots(const adlbr_operator *op);
int operator_wide(const adlbr_operator *op);
int operator_tiled(const adlbr_operator *op);

}  // namespace adlbr
