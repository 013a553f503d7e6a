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
    uint32_t ticket[4];
};

struct adlbr_net_impl;
// Learned preconditioner z = N(r) for K = I + dt A (defined with the CNN).
int net_apply(const adlbr_net *net, const adlbr_operator *op, double dt, const void *r, void *z,
              hipStream_t s);

// Internal entry points shared between translation units.
int cg_direction(const adlbr_operator *op, const void *z, void *q, void *p, CgState *st,
                 double *partial, int first, hipStream_t s);
// |b - (I + dt A) x|^2 for an FP64 iterate x, accumulated in FP64 into
// *out (deterministic); the residual itself goes to rout (storage dtype) if
// rout is not null.
int true_residual(const adlbr_operator *op, double dt, const void *b, const double *x,
                  double *out, double *partial, uint32_t *ticket, void *rout, hipStream_t s);

// Block sum of a double over 256 threads, then the last block to arrive sums
// the per-block partials in block order; returns true in that block's
// threads, with the total in `total`.
__device__ inline bool last_block_sum(double v, double *partial, uint32_t *ticket, double &total) {
    __shared__ double red[256];
    __shared__ int last;
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = red[0];
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double acc = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += 256)
        acc += __hip_atomic_load(&partial[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    total = red[0];
    if (threadIdx.x == 0) *ticket = 0u;
    __syncthreads();  // red[] is reused by the caller's next reduction
    return true;
}
const GridInfo &operator_grid(const adlbr_operator *op);
int operator_storage(const adlbr_operator *op);
const void *operator_diag(const adlbr_operator *op);
const void *operator_weights(const adlbr_operator *op);
const void *operator_slots(const adlbr_operator *op);
int operator_wide(const adlbr_operator *op);

}  // namespace adlbr
