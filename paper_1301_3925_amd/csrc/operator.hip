// AD-LBR operator A = 1/2 grad E_h (eq. (def:E*), h = 1) on the GPU:
// assembly of the gather form and the matrix-free apply / explicit step.
//
// Row z of A has two parts (Section 1; Neumann truncation V(z;h)):
//   own:      sum over slots o of z and s = +-1 with z + s o in the grid of
//             w_o(z) (u(z) - u(z + s o))
//   incoming: sum over directed edges (y, s o) of other points landing on z
//             of w_o(y) (u(z) - u(y)).
// The incoming edges are the transpose of the stencils; they are listed
// once per operator (count -> scan -> fill -> per-row sort), so every apply
// is a deterministic gather with no atomics.
//
// Data layout in the workspace (N points, S = 3 or 6 slots):
//   sb     compact slots: 2D (o0, o1) as 4 x int8 (or int16), o2 = -o0-o1;
//          3D (o0, o1, o2) as 12 x int8 (or int16), o3 = -(o0+o1),
//          o4 = o0-o2, o5 = o1+o2.  One vector load per point.
//   w      [S][N] weights in the storage dtype.
//   cnt    [N] uint8 number of incoming edges of each point.
//   pos    [N] int32 start of each point's incoming list; the apply only
//          reads the entry at the first point of each 64-point slice and
//          rebuilds the rest with a wavefront prefix sum of cnt.
//   ent    incoming entries, int32 ((y - z) << 9 | slot << 6 | lane), lane =
//          z mod 64 (the target's position in its wavefront), sorted per row;
//          |y - z| < 2^22.
//   diag   [N] A_zz (double for FP64 storage, float otherwise).
#include <new>

#include "common.h"

struct adlbr_operator {
    adlbr::GridInfo gi;
    int slots;    // 3 or 6
    int storage;  // adlbr_dtype
    int wide;     // int16 compact offsets
    void *sb;
    void *w;
    uint8_t *cnt;
    int32_t *pos;
    int32_t *ent;
    void *diag;
    unsigned long long *maxdiag;
    double *dtcfl;
    uint32_t *bincnt;  // edges per bin of targets
    uint32_t *bincur;  // placement cursor per bin
    uint32_t *binoff;  // exclusive scan of bincnt
    int2 *binbuf;      // (target, entry) grouped by bin
};

namespace adlbr {
namespace {

constexpr int kBS = 256;         // threads per block of the apply

// --------------------------------------------------------- compact slots --
template <int DIM, bool WIDE> struct Slots;
template <> struct Slots<2, false> {
    typedef char4 store_t;
    int o[3][2];
    __device__ void load(const store_t *p, long long z) {
        const char4 v = p[z];
        o[0][0] = v.x; o[0][1] = v.y; o[1][0] = v.z; o[1][1] = v.w;
        o[2][0] = -o[0][0] - o[1][0]; o[2][1] = -o[0][1] - o[1][1];
    }
    __device__ static bool pack(const int s[6][3], store_t *p, long long z) {
        for (int q = 0; q < 2; ++q)
            for (int c = 0; c < 2; ++c)
                if (s[q][c] > 127 || s[q][c] < -127) {
                    p[z] = make_char4(0, 0, 0, 0);
                    return false;
                }
        p[z] = make_char4(s[0][0], s[0][1], s[1][0], s[1][1]);
        return true;
    }
};
template <> struct Slots<2, true> {
    typedef short4 store_t;
    int o[3][2];
    __device__ void load(const store_t *p, long long z) {
        const short4 v = p[z];
        o[0][0] = v.x; o[0][1] = v.y; o[1][0] = v.z; o[1][1] = v.w;
        o[2][0] = -o[0][0] - o[1][0]; o[2][1] = -o[0][1] - o[1][1];
    }
    __device__ static bool pack(const int s[6][3], store_t *p, long long z) {
        p[z] = make_short4(s[0][0], s[0][1], s[1][0], s[1][1]);
        return true;
    }
};
struct __attribute__((aligned(4))) C3x8 { int8_t v[12]; };
struct __attribute__((aligned(8))) C3x16 { int16_t v[12]; };
template <> struct Slots<3, false> {
    typedef C3x8 store_t;
    int o[6][3];
    __device__ void load(const store_t *p, long long z) {
        const C3x8 v = p[z];
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) o[q][c] = v.v[3 * q + c];
        derive();
    }
    __device__ void derive() {
        for (int c = 0; c < 3; ++c) {
            o[3][c] = -(o[0][c] + o[1][c]);
            o[4][c] = o[0][c] - o[2][c];
            o[5][c] = o[1][c] + o[2][c];
        }
    }
    __device__ static bool pack(const int s[6][3], store_t *p, long long z) {
        C3x8 v;
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) {
                if (s[q][c] > 127 || s[q][c] < -127) {
                    for (int k = 0; k < 12; ++k) v.v[k] = 0;
                    p[z] = v;
                    return false;
                }
                v.v[3 * q + c] = (int8_t)s[q][c];
            }
        v.v[9] = v.v[10] = v.v[11] = 0;
        p[z] = v;
        return true;
    }
};
template <> struct Slots<3, true> {
    typedef C3x16 store_t;
    int o[6][3];
    __device__ void load(const store_t *p, long long z) {
        const C3x16 v = p[z];
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) o[q][c] = v.v[3 * q + c];
        for (int c = 0; c < 3; ++c) {
            o[3][c] = -(o[0][c] + o[1][c]);
            o[4][c] = o[0][c] - o[2][c];
            o[5][c] = o[1][c] + o[2][c];
        }
    }
    __device__ static bool pack(const int s[6][3], store_t *p, long long z) {
        C3x16 v;
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) v.v[3 * q + c] = (int16_t)s[q][c];
        v.v[9] = v.v[10] = v.v[11] = 0;
        p[z] = v;
        return true;
    }
};

// coordinates of a linear index
struct Coord {
    int x, y, z;
};
__device__ __forceinline__ Coord coords(long long i, const GridInfo &g) {
    Coord c;
    const unsigned ui = (unsigned)i;
    const unsigned t = ui / (unsigned)g.nx;
    c.x = (int)(ui - t * (unsigned)g.nx);
    if (g.dim == 2) {
        c.y = (int)t;
        c.z = 0;
    } else {
        const unsigned t2 = t / (unsigned)g.ny;
        c.y = (int)(t - t2 * (unsigned)g.ny);
        c.z = (int)t2;
    }
    return c;
}

__device__ __forceinline__ int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Target of the directed edge (p, s*o); returns false when it leaves a
// Neumann grid.
template <int DIM, bool PER>
__device__ __forceinline__ bool edge_target(const Coord &p, long long i, const int *o, int s,
                                            const GridInfo &g, long long &t) {
    if (PER) {
        const int x = wrap(p.x + s * o[0], g.nx);
        const int y = wrap(p.y + s * o[1], g.ny);
        const int zz = DIM == 3 ? wrap(p.z + s * o[2], g.nz) : 0;
        t = x + (long long)g.nx * (y + (long long)g.ny * zz);
        return t != i;  // an offset that wraps onto the point itself is no edge
    } else {
        const int x = p.x + s * o[0], y = p.y + s * o[1];
        const int zz = DIM == 3 ? p.z + s * o[2] : 0;
        if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || zz < 0 || zz >= g.nz) return false;
        t = i + s * (o[0] + (long long)g.nx * (o[1] + (long long)g.ny * (DIM == 3 ? o[2] : 0)));
        return true;
    }
}

// ---------------------------------------------------------------- build --

__global__ void k_fill_i32(int32_t *p, long long n, int32_t v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_init_scalars(unsigned long long *maxdiag) { *maxdiag = 0ull; }

template <typename TW> __device__ __forceinline__ double ld_w(const TW *w, long long i) {
    return (double)w[i];
}

// Pack the slots, convert the weights, count incoming edges per target.
// Assembly of the transpose (incoming lists) without per-edge global
// atomics.  Targets are grouped into bins of kBin consecutive points; the
// edges of a wavefront mostly land in one or two bins, so counting and
// placing them costs one atomic per distinct bin per wavefront (leader lane,
// ballot of the lanes that share its bin).  Each bin is then built by one
// block with LDS counters.
constexpr int kBinShift = 10;
constexpr int kBin = 1 << kBinShift;

// The edges (q, s) of point z, in a fixed order; returns the target of the
// k-th candidate edge or -1.
template <int DIM, bool PER>
__device__ __forceinline__ long long edge_k(const Coord &p, long long z, const int s[6][3],
                                           const double *wq, int k, const GridInfo &g) {
    const int q = k >> 1, sg = (k & 1) ? 1 : -1;
    if (!(wq[q] > 0.0)) return -1;
    long long t;
    if (!edge_target<DIM, PER>(p, z, s[q], sg, g, t)) return -1;
    // entries store z - t in 23 bits; such an edge is flagged and left out
    if (z - t >= (1ll << 22) || z - t <= -(1ll << 22)) return -2;
    return t;
}

// Wave-aggregated "append to bin": every lane with bin >= 0 gets a slot in
// its bin; the leader of each group of lanes sharing a bin does one atomic.
// With count_only the slot is not needed.
__device__ __forceinline__ unsigned bin_append(int bin, uint32_t *counter, bool count_only) {
    const int lane = (int)(threadIdx.x & 63u);
    unsigned long long pending = __ballot(bin >= 0);
    unsigned slot = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int bl = __shfl(bin, leader, 64);
        const unsigned long long m = __ballot(bin == bl);
        unsigned base = 0;
        if (lane == leader) base = atomicAdd(&counter[bl], (unsigned)__popcll(m));
        if (!count_only) {
            base = __shfl(base, leader, 64);
            if (bin == bl) slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
        }
        pending &= ~m;
    }
    return slot;
}

// Pack the slots, convert the weights, count the edges landing in each bin.
template <int DIM, bool WIDE, bool PER, typename TWin, typename TS, typename TA>
__global__ void k_compact(GridInfo g, const int16_t *__restrict__ off, const TWin *__restrict__ win,
                          typename Slots<DIM, WIDE>::store_t *__restrict__ sb, TS *__restrict__ w,
                          uint32_t *__restrict__ bincnt, int32_t *status) {
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = z < g.N;  // every lane takes part in the ballots
    constexpr int S = DIM == 2 ? 3 : 6;
    const long long N = g.N;
    int s[6][3];
    double wq[6];
    int st = 0;
    for (int q = 0; q < 6; ++q) {
        wq[q] = 0.0;
        for (int c = 0; c < 3; ++c) s[q][c] = 0;
    }
    Coord p{0, 0, 0};
    if (live) {
        for (int q = 0; q < S; ++q)
            for (int c = 0; c < 3; ++c) s[q][c] = c < DIM ? (int)off[(DIM * q + c) * N + z] : 0;
        bool rel = true;
        if (DIM == 2) {
            for (int c = 0; c < 2; ++c) rel = rel && s[2][c] == -s[0][c] - s[1][c];
        } else {
            for (int c = 0; c < 3; ++c)
                rel = rel && s[3][c] == -(s[0][c] + s[1][c]) && s[4][c] == s[0][c] - s[2][c] &&
                      s[5][c] == s[1][c] + s[2][c];
        }
        if (!rel) st |= ADLBR_ST_STENCIL;
        if (!Slots<DIM, WIDE>::pack(s, sb, z)) st |= ADLBR_ST_RANGE;
        p = coords(z, g);
        for (int q = 0; q < S; ++q) {
            wq[q] = (double)win[q * N + z];
            w[q * N + z] = Conv<TS, TA>::st((TA)wq[q]);
        }
    }
    for (int k = 0; k < 2 * S; ++k) {
        const long long t = live ? edge_k<DIM, PER>(p, z, s, wq, k, g) : -1;
        if (t == -2) st |= ADLBR_ST_RANGE;
        bin_append(t >= 0 ? (int)(t >> kBinShift) : -1, bincnt, true);
    }
    if (live) report(status, z, st);
}

// Place every edge (target, entry) in its bin's region of binbuf.
template <int DIM, bool WIDE, bool PER, typename TWin>
__global__ void k_bin_fill(GridInfo g, const int16_t *__restrict__ off, const TWin *__restrict__ win,
                           const uint32_t *__restrict__ binoff, uint32_t *__restrict__ bincur,
                           int2 *__restrict__ binbuf) {
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = z < g.N;
    constexpr int S = DIM == 2 ? 3 : 6;
    const long long N = g.N;
    int s[6][3];
    double wq[6];
    for (int q = 0; q < 6; ++q) {
        wq[q] = 0.0;
        for (int c = 0; c < 3; ++c) s[q][c] = 0;
    }
    Coord p{0, 0, 0};
    if (live) {
        for (int q = 0; q < S; ++q) {
            for (int c = 0; c < 3; ++c) s[q][c] = c < DIM ? (int)off[(DIM * q + c) * N + z] : 0;
            wq[q] = (double)win[q * N + z];
        }
        p = coords(z, g);
    }
    for (int k = 0; k < 2 * S; ++k) {
        const long long t = live ? edge_k<DIM, PER>(p, z, s, wq, k, g) : -1;
        const int bin = t >= 0 ? (int)(t >> kBinShift) : -1;
        const unsigned slot = bin_append(bin, bincur, false);
        if (bin >= 0) {
            const int32_t e = (int32_t)(((z - t) << 9) | ((k >> 1) << 6) | (t & 63));
            binbuf[(long long)binoff[bin] + slot] = make_int2((int)t, e);
        }
    }
}

// One block per bin: per-target counts and offsets in LDS, entries placed at
// their row, rows sorted by (source, slot), diagonal A_zz = own in-grid
// weights + incoming weights, and the maximum diagonal.
template <int DIM, bool WIDE, bool PER, typename TS, typename TA, typename TD>
__global__ __launch_bounds__(256) void k_bin_build(
    GridInfo g, const uint32_t *__restrict__ bincnt, const uint32_t *__restrict__ binoff,
    const int2 *__restrict__ binbuf, const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
    const TS *__restrict__ w, int32_t *__restrict__ pos, uint8_t *__restrict__ cnt,
    int32_t *__restrict__ ent, TD *__restrict__ diag, unsigned long long *maxdiag, int32_t *status) {
    __shared__ int32_t lcnt[kBin];
    __shared__ int32_t loff[kBin];
    __shared__ int32_t scan[256];
    __shared__ double red[256];
    constexpr int S = DIM == 2 ? 3 : 6;
    const long long N = g.N;
    const long long b = blockIdx.x;
    const long long t0 = b << kBinShift;
    const long long base = binoff[b];
    const unsigned E = bincnt[b];
    for (int k = threadIdx.x; k < kBin; k += 256) lcnt[k] = 0;
    __syncthreads();
    for (unsigned e = threadIdx.x; e < E; e += 256) atomicAdd(&lcnt[binbuf[base + e].x - t0], 1);
    __syncthreads();
    // exclusive scan of the clamped counts (4 per thread)
    int32_t c4[4], sum = 0;
    for (int k = 0; k < 4; ++k) {
        const int tl = threadIdx.x * 4 + k;
        c4[k] = lcnt[tl];
        sum += min(c4[k], 255);
    }
    scan[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int32_t add = threadIdx.x >= (unsigned)d ? scan[threadIdx.x - d] : 0;
        __syncthreads();
        scan[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = scan[threadIdx.x] - sum;
    for (int k = 0; k < 4; ++k) {
        const int tl = threadIdx.x * 4 + k;
        loff[tl] = run;
        const long long t = t0 + tl;
        if (t < N) {
            pos[t] = (int32_t)(base + run);
            cnt[t] = (uint8_t)min(c4[k], 255);
            if (c4[k] > 255) report(status, t, ADLBR_ST_INCOMING);
        }
        run += min(c4[k], 255);
        lcnt[tl] = 0;  // becomes the placement cursor
    }
    __syncthreads();
    for (unsigned e = threadIdx.x; e < E; e += 256) {
        const int2 v = binbuf[base + e];
        const int tl = v.x - (int)t0;
        const int k = atomicAdd(&lcnt[tl], 1);
        if (k < 255) ent[base + loff[tl] + k] = v.y;
    }
    __syncthreads();
    double dmax = 0.0;
    for (int k = 0; k < 4; ++k) {
        const int tl = threadIdx.x + 256 * k;
        const long long z = t0 + tl;
        if (z >= N) continue;
        const int c = min(lcnt[tl], 255);
        int32_t *e = ent + base + loff[tl];
        if (c <= 16) {  // odd-even transposition network on 16 registers
            int32_t r[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) r[i] = i < c ? e[i] : 0x7fffffff;
#pragma unroll
            for (int round = 0; round < 16; ++round) {
#pragma unroll
                for (int i = round & 1; i + 1 < 16; i += 2) {
                    const int32_t a = r[i], bb = r[i + 1];
                    r[i] = min(a, bb);
                    r[i + 1] = max(a, bb);
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < c) e[i] = r[i];
        } else {
            for (int i = 1; i < c; ++i) {  // insertion sort by (source, slot)
                const int32_t key = e[i];
                int j = i - 1;
                while (j >= 0 && e[j] > key) {
                    e[j + 1] = e[j];
                    --j;
                }
                e[j + 1] = key;
            }
        }
        double d = 0.0;
        Slots<DIM, WIDE> sl;
        sl.load(sb, z);
        const Coord p = coords(z, g);
        for (int q = 0; q < S; ++q) {
            const double wv = (double)Conv<TS, TA>::ld(w[q * N + z]);
            for (int sg = -1; sg <= 1; sg += 2) {
                long long t;
                if (edge_target<DIM, PER>(p, z, sl.o[q], sg, g, t)) d += wv;
            }
        }
        for (int i = 0; i < c; ++i) {
            const int32_t v = e[i];
            d += (double)Conv<TS, TA>::ld(w[(long long)((v >> 6) & 7) * N + z + (v >> 9)]);
        }
        diag[z] = (TD)d;
        dmax = fmax(dmax, d);
    }
    red[threadIdx.x] = dmax;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(maxdiag, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_copy_u32(const uint32_t *a, uint32_t *b, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// Block-level exclusive scan helpers (blockDim.x == 256, 4 items per thread).
__device__ int32_t block_excl_scan256(int32_t v, int32_t *lds, int32_t &total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int32_t add = t >= d ? lds[t - d] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    total = lds[255];
    const int32_t incl = lds[t];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_top(int32_t *bsum, long long nb) {
    __shared__ int32_t lds[256];
    int32_t carry = 0;
    for (long long b0 = 0; b0 < nb; b0 += 256) {
        const long long i = b0 + threadIdx.x;
        const int32_t v = i < nb ? bsum[i] : 0;
        int32_t total;
        const int32_t ex = block_excl_scan256(v, lds, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
}

__global__ void k_cfl(const unsigned long long *maxdiag, double *dtcfl) {
    const double m = __longlong_as_double((long long)*maxdiag);
    *dtcfl = m > 0.0 ? 1.0 / m : 0.0;
}

// ---------------------------------------------------------------- apply --
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
    const unsigned lane = threadIdx.x & 63u;
    unsigned x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned y = __shfl_up(x, d, 64);
        if (lane >= (unsigned)d) x += y;
    }
    return x;
}

// Where a wavefront's incoming lists are: the 64 consecutive rows of the
// wave own the entries [start, start + total) in row order; this lane's row
// owns [lo, hi) relative to start.
struct WaveLists {
    long long start;
    unsigned total, lo, hi;
};

__device__ __forceinline__ WaveLists wave_lists(const uint8_t *__restrict__ cnt,
                                                const int32_t *__restrict__ pos, long long z,
                                                long long N) {
    WaveLists L;
    const unsigned c = z < N ? cnt[z] : 0u;
    const unsigned incl = wave_incl_scan(c);
    L.total = __shfl(incl, 63, 64);
    L.lo = incl - c;
    L.hi = incl;
    const long long z0 = z & ~63ll;
    L.start = z0 < N ? (long long)pos[z0] : 0;
    return L;
}

// Own part of row z: sum over slots o and signs s with z + s o in the grid
// of w_o(z) (u(z) - u(z + s o)).
template <int DIM, bool WIDE, bool PER, typename TS, typename TA, typename TU>
__device__ __forceinline__ TA row_own(const GridInfo &g, long long z, TA uz, const TU *__restrict__ u,
                                      const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                      const TS *__restrict__ w) {
    constexpr int S = DIM == 2 ? 3 : 6;
    const long long N = g.N;
    TA acc = (TA)0;
    Slots<DIM, WIDE> sl;
    sl.load(sb, z);
    const Coord p = coords(z, g);
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const TA wq = Conv<TS, TA>::ld(w[q * N + z]);
        TA part = (TA)0;
#pragma unroll
        for (int sg = -1; sg <= 1; sg += 2) {
            long long t;
            if (edge_target<DIM, PER>(p, z, sl.o[q], sg, g, t))
                part += uz - Conv<TU, TA>::ld(u[t]);
        }
        acc += wq * part;
    }
    return acc;
}

// Incoming part of the rows of one wavefront, computed cooperatively: the
// wave's entries are taken 64 at a time (coalesced loads, every lane busy),
// each lane evaluates one edge w_slot(y) (u(row) - u(y)), and a segmented
// inclusive scan over the lanes (entries are grouped by row, rows ascend)
// sums each row's run; every lane then picks up its own row's sum from the
// lane holding the end of that run.  The order of additions is fixed, so the
// result is deterministic.  All 64 lanes must call this.
template <typename TS, typename TA, typename TU>
__device__ __forceinline__ TA wave_incoming(const WaveLists &L, long long z, long long N, TA uz,
                                            const TU *__restrict__ u, const TS *__restrict__ w,
                                            const int32_t *__restrict__ ent) {
    const int lane = (int)(threadIdx.x & 63u);
    const long long z0 = z & ~63ll;
    TA acc = (TA)0;
    for (unsigned e0 = 0; e0 < L.total; e0 += 64) {
        const unsigned e = e0 + lane;
        const bool valid = e < L.total;
        const int32_t v = valid ? ent[L.start + e] : 0;
        const int row = valid ? (v & 63) : 64;
        const TA ur = __shfl(uz, row & 63, 64);
        TA val = (TA)0;
        if (valid) {
            const long long y = z0 + (v & 63) + (v >> 9);
            val = Conv<TS, TA>::ld(w[(long long)((v >> 6) & 7) * N + y]) * (ur - Conv<TU, TA>::ld(u[y]));
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const TA vu = __shfl_up(val, d, 64);
            const int ru = __shfl_up(row, d, 64);
            if (lane >= d && ru == row) val += vu;
        }
        const unsigned lo = L.lo > e0 ? L.lo : e0;
        const unsigned hi = L.hi < e0 + 64 ? L.hi : e0 + 64;
        const TA mine = __shfl(val, (int)((hi - 1 - e0) & 63u), 64);
        if (hi > lo) acc += mine;
    }
    return acc;
}

// out = A u (STEP = false) or u - dt A u (STEP = true).
template <int DIM, bool WIDE, bool PER, bool STEP, typename TS, typename TA>
__global__ __launch_bounds__(kBS) void k_apply(
    GridInfo g, const TS *__restrict__ u, TS *__restrict__ out,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const TS *__restrict__ w,
    const uint8_t *__restrict__ cnt, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ ent, double dt, const double *__restrict__ dtcfl, int dt_mode) {
    const long long N = g.N;
    const long long blk = xcd_block(blockIdx.x, gridDim.x);
    const long long z = blk * kBS + threadIdx.x;
    const bool live = z < N;
    const WaveLists L = wave_lists(cnt, pos, z, N);
    const TA uz = live ? Conv<TS, TA>::ld(u[z]) : (TA)0;
    TA acc = wave_incoming<TS, TA, TS>(L, z, N, uz, u, w, ent);
    if (!live) return;
    acc += row_own<DIM, WIDE, PER, TS, TA, TS>(g, z, uz, u, sb, w);
    if (STEP) {
        const TA h = (TA)(dt_mode == ADLBR_DT_CFL ? dt * dtcfl[0] : dt);
        out[z] = Conv<TS, TA>::st(uz - h * acc);
    } else {
        out[z] = Conv<TS, TA>::st(acc);
    }
}

// Conjugate-gradient direction with K = I + dt A (dt from the state):
//   q = K z + beta q,  p = z + beta p  (beta = 0 on the first iteration),
// so that q = K p without a second gather.  Each block writes its partial
// <p, q> in FP64; the last block to finish sums the partials in block order
// (deterministic) and sets alpha = <z, r> / <p, q>.
template <int DIM, bool WIDE, bool PER, typename T>
__global__ __launch_bounds__(kBS) void k_cg_direction(
    GridInfo g, const T *__restrict__ zv, T *__restrict__ q, T *__restrict__ p,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const T *__restrict__ w,
    const uint8_t *__restrict__ cnt, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ ent, CgState *st, double *partial, int first) {
    __shared__ double red[kBS];
    const long long N = g.N;
    const long long blk = xcd_block(blockIdx.x, gridDim.x);
    const long long z = blk * kBS + threadIdx.x;
    const bool live = z < N;
    double pqz = 0.0;
    const bool skip = st->bad || st->done;
    const WaveLists L = wave_lists(cnt, pos, z, N);
    const T zz = live ? zv[z] : (T)0;
    T acc = skip ? (T)0 : wave_incoming<T, T, T>(L, z, N, zz, zv, w, ent);
    if (live && !skip) {
        acc += row_own<DIM, WIDE, PER, T, T, T>(g, z, zz, zv, sb, w);
        const T dt = (T)st->dt;
        const T beta = first ? (T)0 : (T)st->beta;
        const T qn = zz + dt * acc + (first ? (T)0 : beta * q[z]);
        const T pn = zz + (first ? (T)0 : beta * p[z]);
        q[z] = qn;
        p[z] = pn;
        pqz = (double)pn * (double)qn;
    }
    red[threadIdx.x] = pqz;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blk] = red[0];
        __threadfence();
        const unsigned t = atomicAdd(&st->ticket[0], 1u);
        red[0] = (t == gridDim.x - 1) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (red[0] != 0.0) {  // last block: ordered sum of all partials
        __threadfence();
        double acc = 0.0;
        for (long long b = threadIdx.x; b < gridDim.x; b += kBS)
            acc += __hip_atomic_load(&partial[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = kBS / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (!skip) {
                const double pq = red[0];
                st->pq = pq;
                if (!(pq > 0.0) || !isfinite(pq)) st->bad = 1;
                st->alpha = st->bad ? 0.0 : st->rz / pq;
            }
            st->ticket[0] = 0u;
        }
    }
}

// |b - (x + dt A x)|^2 with FP64 arithmetic (weights promoted).
template <int DIM, bool WIDE, bool PER, typename T>
__global__ __launch_bounds__(kBS) void k_residual(
    GridInfo g, const T *__restrict__ b, const double *__restrict__ x,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const T *__restrict__ w,
    const uint8_t *__restrict__ cnt, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ ent, double dt, double *out, double *partial, uint32_t *ticket,
    T *__restrict__ rout) {
    const long long N = g.N;
    const long long z = (long long)blockIdx.x * kBS + threadIdx.x;
    const bool live = z < N;
    double r2 = 0.0;
    const WaveLists L = wave_lists(cnt, pos, z, N);
    const double xz = live ? x[z] : 0.0;
    double ax = wave_incoming<T, double, double>(L, z, N, xz, x, w, ent);
    if (live) {
        ax += row_own<DIM, WIDE, PER, T, double, double>(g, z, xz, x, sb, w);
        const double r = (double)b[z] - (xz + dt * ax);
        r2 = r * r;
        if (rout) rout[z] = (T)r;
    }
    double tot;
    if (last_block_sum(r2, partial, ticket, tot) && threadIdx.x == 0) *out = tot;
}

template <int DIM, bool WIDE, bool PER, typename TS, typename TA>
int build_impl(adlbr_operator *op, const int16_t *off, const void *win, int win_f64,
               int32_t *status, hipStream_t s) {
    typedef typename Slots<DIM, WIDE>::store_t store_t;
    const GridInfo g = op->gi;
    const long long N = g.N;
    const unsigned nb = (unsigned)((N + kBS - 1) / kBS);
    const long long nbins = (N + kBin - 1) / kBin;
    const unsigned nbb = (unsigned)((nbins + kBS - 1) / kBS);
    TS *w = (TS *)op->w;
    store_t *sb = (store_t *)op->sb;
    hipLaunchKernelGGL(k_fill_i32, dim3(nbb), dim3(kBS), 0, s, (int32_t *)op->bincnt, nbins, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(nbb), dim3(kBS), 0, s, (int32_t *)op->bincur, nbins, 0);
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(1), 0, s, op->maxdiag);
    if (win_f64)
        hipLaunchKernelGGL((k_compact<DIM, WIDE, PER, double, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           off, (const double *)win, sb, w, op->bincnt, status);
    else
        hipLaunchKernelGGL((k_compact<DIM, WIDE, PER, float, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           off, (const float *)win, sb, w, op->bincnt, status);
    hipLaunchKernelGGL(k_copy_u32, dim3(nbb), dim3(kBS), 0, s, op->bincnt, op->binoff, nbins);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, (int32_t *)op->binoff, nbins);
    if (win_f64)
        hipLaunchKernelGGL((k_bin_fill<DIM, WIDE, PER, double>), dim3(nb), dim3(kBS), 0, s, g, off,
                           (const double *)win, op->binoff, op->bincur, op->binbuf);
    else
        hipLaunchKernelGGL((k_bin_fill<DIM, WIDE, PER, float>), dim3(nb), dim3(kBS), 0, s, g, off,
                           (const float *)win, op->binoff, op->bincur, op->binbuf);
    if (op->storage == ADLBR_F64)
        hipLaunchKernelGGL((k_bin_build<DIM, WIDE, PER, TS, TA, double>), dim3((unsigned)nbins),
                           dim3(256), 0, s, g, op->bincnt, op->binoff, op->binbuf, sb, w, op->pos,
                           op->cnt, op->ent, (double *)op->diag, op->maxdiag, status);
    else
        hipLaunchKernelGGL((k_bin_build<DIM, WIDE, PER, TS, TA, float>), dim3((unsigned)nbins),
                           dim3(256), 0, s, g, op->bincnt, op->binoff, op->binbuf, sb, w, op->pos,
                           op->cnt, op->ent, (float *)op->diag, op->maxdiag, status);
    hipLaunchKernelGGL(k_cfl, dim3(1), dim3(1), 0, s, op->maxdiag, op->dtcfl);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

template <int DIM, bool WIDE, bool PER, typename TS, typename TA>
int apply_impl(const adlbr_operator *op, const void *u, void *out, bool step, double dt, int dt_mode,
               hipStream_t s) {
    typedef typename Slots<DIM, WIDE>::store_t store_t;
    const GridInfo g = op->gi;
    const unsigned nb = (unsigned)((g.N + kBS - 1) / kBS);
    if (step)
        hipLaunchKernelGGL((k_apply<DIM, WIDE, PER, true, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           (const TS *)u, (TS *)out, (const store_t *)op->sb, (const TS *)op->w,
                           op->cnt, op->pos, op->ent, dt, op->dtcfl, dt_mode);
    else
        hipLaunchKernelGGL((k_apply<DIM, WIDE, PER, false, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           (const TS *)u, (TS *)out, (const store_t *)op->sb, (const TS *)op->w,
                           op->cnt, op->pos, op->ent, dt, op->dtcfl, dt_mode);
    return ADLBR_OK;
}

// Expand the (dim, wide, periodic, storage) choice into template instances.
template <template <int, bool, bool, typename, typename> class F, typename OpT,
          typename... Args>
int dispatch(OpT *op, Args... args) {
#define ADLBR_D3(DIM, WIDE, PER)                                                         \
    switch (op->storage) {                                                               \
    case ADLBR_F64: return F<DIM, WIDE, PER, double, double>::run(op, args...);          \
    case ADLBR_F32: return F<DIM, WIDE, PER, float, float>::run(op, args...);            \
    case ADLBR_BF16: return F<DIM, WIDE, PER, bf16, float>::run(op, args...);            \
    case ADLBR_F16: return F<DIM, WIDE, PER, _Float16, float>::run(op, args...);         \
    default: return ADLBR_E_UNSUPPORTED;                                                 \
    }
    const int dim = op->gi.dim, wide = op->wide, per = op->gi.periodic;
    if (dim == 2 && !wide && !per) { ADLBR_D3(2, false, false) }
    if (dim == 2 && !wide && per) { ADLBR_D3(2, false, true) }
    if (dim == 2 && wide && !per) { ADLBR_D3(2, true, false) }
    if (dim == 2 && wide && per) { ADLBR_D3(2, true, true) }
    if (dim == 3 && !wide && !per) { ADLBR_D3(3, false, false) }
    if (dim == 3 && !wide && per) { ADLBR_D3(3, false, true) }
    if (dim == 3 && wide && !per) { ADLBR_D3(3, true, false) }
    if (dim == 3 && wide && per) { ADLBR_D3(3, true, true) }
#undef ADLBR_D3
    return ADLBR_E_UNSUPPORTED;
}

template <int DIM, bool WIDE, bool PER, typename TS, typename TA> struct BuildF {
    static int run(adlbr_operator *op, const int16_t *off, const void *win, int f64, int32_t *st,
                   hipStream_t s) {
        return build_impl<DIM, WIDE, PER, TS, TA>(op, off, win, f64, st, s);
    }
};
template <int DIM, bool WIDE, bool PER, typename TS, typename TA> struct ApplyF {
    static int run(const adlbr_operator *op, const void *u, void *out, bool step, double dt,
                   int mode, hipStream_t s) {
        return apply_impl<DIM, WIDE, PER, TS, TA>(op, u, out, step, dt, mode, s);
    }
};

template <int DIM, bool WIDE, bool PER, typename TS, typename TA> struct CgDirF {
    static int run(const adlbr_operator *op, const void *z, void *q, void *p, CgState *st,
                   double *partial, int first, hipStream_t s) {
        typedef typename Slots<DIM, WIDE>::store_t store_t;
        const GridInfo g = op->gi;
        const unsigned nb = (unsigned)((g.N + kBS - 1) / kBS);
        if (op->storage != ADLBR_F32 && op->storage != ADLBR_F64) return ADLBR_E_UNSUPPORTED;
        hipLaunchKernelGGL((k_cg_direction<DIM, WIDE, PER, TS>), dim3(nb), dim3(kBS), 0, s, g,
                           (const TS *)z, (TS *)q, (TS *)p, (const store_t *)op->sb,
                           (const TS *)op->w, op->cnt, op->pos, op->ent, st, partial, first);
        return ADLBR_OK;
    }
};
template <int DIM, bool WIDE, bool PER> struct CgDirF<DIM, WIDE, PER, bf16, float> {
    static int run(const adlbr_operator *, const void *, void *, void *, CgState *, double *, int,
                   hipStream_t) {
        return ADLBR_E_UNSUPPORTED;
    }
};
template <int DIM, bool WIDE, bool PER> struct CgDirF<DIM, WIDE, PER, _Float16, float> {
    static int run(const adlbr_operator *, const void *, void *, void *, CgState *, double *, int,
                   hipStream_t) {
        return ADLBR_E_UNSUPPORTED;
    }
};

template <int DIM, bool WIDE, bool PER, typename TS, typename TA> struct ResidualF {
    static int run(const adlbr_operator *op, double dt, const void *b, const double *x,
                   double *out, double *partial, uint32_t *ticket, void *rout, hipStream_t s) {
        typedef typename Slots<DIM, WIDE>::store_t store_t;
        const GridInfo g = op->gi;
        const unsigned nb = (unsigned)((g.N + kBS - 1) / kBS);
        hipLaunchKernelGGL((k_residual<DIM, WIDE, PER, TS>), dim3(nb), dim3(kBS), 0, s, g,
                           (const TS *)b, x, (const store_t *)op->sb, (const TS *)op->w, op->cnt,
                           op->pos, op->ent, dt, out, partial, ticket, (TS *)rout);
        return ADLBR_OK;
    }
};
template <int DIM, bool WIDE, bool PER> struct ResidualF<DIM, WIDE, PER, bf16, float> {
    static int run(const adlbr_operator *, double, const void *, const double *, double *,
                   double *, uint32_t *, void *, hipStream_t) {
        return ADLBR_E_UNSUPPORTED;
    }
};
template <int DIM, bool WIDE, bool PER> struct ResidualF<DIM, WIDE, PER, _Float16, float> {
    static int run(const adlbr_operator *, double, const void *, const double *, double *,
                   double *, uint32_t *, void *, hipStream_t) {
        return ADLBR_E_UNSUPPORTED;
    }
};

struct Layout {
    size_t sb, w, cnt, pos, ent, diag, scal, bincnt, bincur, binoff, binbuf, total;
};

Layout layout(const GridInfo &g, int storage, int wide) {
    const long long N = g.N;
    const int S = g.dim == 2 ? 3 : 6;
    const size_t sbsz = g.dim == 2 ? (wide ? 8 : 4) : (wide ? 24 : 12);
    const size_t nbins = (size_t)((N + kBin - 1) / kBin);
    Layout L;
    size_t o = 0;
    L.sb = o;   o += align_up(sbsz * N);
    L.w = o;    o += align_up(dtype_size(storage) * S * N);
    L.cnt = o;  o += align_up((size_t)N + 64);
    L.pos = o;  o += align_up(4 * (size_t)N + 256);
    L.ent = o;  o += align_up(4 * (size_t)(2 * S) * N);
    L.diag = o; o += align_up((storage == ADLBR_F64 ? 8 : 4) * (size_t)N);
    L.scal = o; o += 256;
    L.bincnt = o; o += align_up(4 * nbins + 4);
    L.bincur = o; o += align_up(4 * nbins + 4);
    L.binoff = o; o += align_up(4 * nbins + 4);
    L.binbuf = o; o += align_up(8 * (size_t)(2 * S) * N);
    L.total = o;
    return L;
}

}  // namespace

int cg_direction(const adlbr_operator *op, const void *z, void *q, void *p, CgState *st,
                 double *partial, int first, hipStream_t s) {
    return dispatch<CgDirF>(op, z, q, p, st, partial, first, s);
}

// out = (I + dt A) u, written as one explicit step with step -dt.
int apply_K(const adlbr_operator *op, const void *u, void *out, double dt, hipStream_t s) {
    return dispatch<ApplyF>(op, u, out, true, -dt, (int)ADLBR_DT_ABS, s);
}

int true_residual(const adlbr_operator *op, double dt, const void *b, const double *x,
                  double *out, double *partial, uint32_t *ticket, void *rout, hipStream_t s) {
    return dispatch<ResidualF>(op, dt, b, x, out, partial, ticket, rout, s);
}

const GridInfo &operator_grid(const adlbr_operator *op) { return op->gi; }
int operator_storage(const adlbr_operator *op) { return op->storage; }
const void *operator_diag(const adlbr_operator *op) { return op->diag; }
const void *operator_weights(const adlbr_operator *op) { return op->w; }
const void *operator_slots(const adlbr_operator *op) { return op->sb; }
int operator_wide(const adlbr_operator *op) { return op->wide; }

}  // namespace adlbr

using namespace adlbr;

extern "C" int adlbr_operator_workspace(const adlbr_grid *g, int storage, int flags,
                                        size_t *bytes) {
    clear_error();
    GridInfo gi;
    int rc = check_grid(g, &gi);
    if (rc) return rc;
    if (!bytes || dtype_size(storage) == 0) {
        set_error("adlbr_operator_workspace: bad storage dtype or null output");
        return ADLBR_E_INVALID;
    }
    *bytes = layout(gi, storage, flags & ADLBR_OP_WIDE).total;
    return ADLBR_OK;
}

extern "C" int adlbr_operator_create(const adlbr_grid *g, const int16_t *offsets,
                                     const void *weights, int w_dtype, int storage, int flags,
                                     void *workspace, size_t ws_bytes, int32_t *status,
                                     void *stream, adlbr_operator **op_out) {
    clear_error();
    GridInfo gi;
    int rc = check_grid(g, &gi);
    if (rc) return rc;
    if (!offsets || !weights || !workspace || !status || !op_out) {
        set_error("adlbr_operator_create: null pointer argument");
        return ADLBR_E_INVALID;
    }
    if ((w_dtype != ADLBR_F64 && w_dtype != ADLBR_F32) || dtype_size(storage) == 0) {
        set_error("adlbr_operator_create: weights must be F64/F32, storage F64/F32/BF16/F16");
        return ADLBR_E_INVALID;
    }
    const int wide = flags & ADLBR_OP_WIDE ? 1 : 0;
    if ((long long)(gi.dim == 2 ? 6 : 12) * gi.N >= (1ll << 31)) {
        set_error("adlbr_operator_create: too many edges for 32-bit list positions");
        return ADLBR_E_RANGE;
    }
    const Layout L = layout(gi, storage, wide);
    if (ws_bytes < L.total) {
        set_error("adlbr_operator_create: workspace has %zu bytes, %zu needed", ws_bytes, L.total);
        return ADLBR_E_NOMEM;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
        set_error("adlbr_operator_create: workspace must be 256-byte aligned");
        return ADLBR_E_INVALID;
    }
    adlbr_operator *op = new (std::nothrow) adlbr_operator;
    if (!op) {
        set_error("adlbr_operator_create: out of host memory");
        return ADLBR_E_NOMEM;
    }
    char *b = (char *)workspace;
    op->gi = gi;
    op->slots = gi.dim == 2 ? 3 : 6;
    op->storage = storage;
    op->wide = wide;
    op->sb = b + L.sb;
    op->w = b + L.w;
    op->cnt = (uint8_t *)(b + L.cnt);
    op->pos = (int32_t *)(b + L.pos);
    op->ent = (int32_t *)(b + L.ent);
    op->diag = b + L.diag;
    op->maxdiag = (unsigned long long *)(b + L.scal);
    op->dtcfl = (double *)(b + L.scal + 8);
    op->bincnt = (uint32_t *)(b + L.bincnt);
    op->bincur = (uint32_t *)(b + L.bincur);
    op->binoff = (uint32_t *)(b + L.binoff);
    op->binbuf = (int2 *)(b + L.binbuf);
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, s, status);
    rc = dispatch<BuildF>(op, offsets, weights, (int)(w_dtype == ADLBR_F64), status, s);
    hipLaunchKernelGGL(k_status_final, dim3(1), dim3(1), 0, s, status);
    if (rc) {
        delete op;
        return rc;
    }
    ADLBR_LAUNCH_CHECK();
    *op_out = op;
    return ADLBR_OK;
}

extern "C" int adlbr_operator_destroy(adlbr_operator *op) {
    delete op;
    return ADLBR_OK;
}

extern "C" int adlbr_operator_dt_cfl(adlbr_operator *op, double *dt_max, void *stream) {
    clear_error();
    if (!op || !dt_max) {
        set_error("adlbr_operator_dt_cfl: null argument");
        return ADLBR_E_INVALID;
    }
    hipStream_t s = as_stream(stream);
    ADLBR_CHECK_HIP(hipMemcpyAsync(dt_max, op->dtcfl, sizeof(double), hipMemcpyDeviceToHost, s));
    ADLBR_CHECK_HIP(hipStreamSynchronize(s));
    return ADLBR_OK;
}

namespace {
template <typename TI, typename TO>
__global__ void k_convert(const TI *in, TO *out, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (TO)in[i];
}
}  // namespace

extern "C" int adlbr_operator_diagonal(adlbr_operator *op, void *diag, int dtype, void *stream) {
    clear_error();
    if (!op || !diag || (dtype != ADLBR_F64 && dtype != ADLBR_F32)) {
        set_error("adlbr_operator_diagonal: bad argument");
        return ADLBR_E_INVALID;
    }
    hipStream_t s = as_stream(stream);
    const long long N = op->gi.N;
    const unsigned nb = (unsigned)((N + 255) / 256);
    const bool src64 = op->storage == ADLBR_F64;
    if (src64 && dtype == ADLBR_F64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(nb), dim3(256), 0, s, (const double *)op->diag, (double *)diag, N);
    else if (src64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nb), dim3(256), 0, s, (const double *)op->diag, (float *)diag, N);
    else if (dtype == ADLBR_F64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(nb), dim3(256), 0, s, (const float *)op->diag, (double *)diag, N);
    else
        hipLaunchKernelGGL((k_convert<float, float>), dim3(nb), dim3(256), 0, s, (const float *)op->diag, (float *)diag, N);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_apply(adlbr_operator *op, const void *u, void *Au, void *stream) {
    clear_error();
    if (!op || !u || !Au || u == Au) {
        set_error("adlbr_apply: null or aliased argument");
        return ADLBR_E_INVALID;
    }
    int rc = dispatch<ApplyF>(op, u, Au, false, 0.0, 0, as_stream(stream));
    if (rc) return rc;
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

extern "C" int adlbr_step(adlbr_operator *op, void *u, void *u_tmp, double dt, int dt_mode,
                          int64_t nsteps, void *stream) {
    clear_error();
    if (!op || !u || !u_tmp || u == u_tmp || nsteps < 0 ||
        (dt_mode != ADLBR_DT_ABS && dt_mode != ADLBR_DT_CFL)) {
        set_error("adlbr_step: bad argument");
        return ADLBR_E_INVALID;
    }
    hipStream_t s = as_stream(stream);
    void *a = u, *b = u_tmp;
    for (int64_t k = 0; k < nsteps; ++k) {
        int rc = dispatch<ApplyF>(op, (const void *)a, b, true, dt, dt_mode, s);
        if (rc) return rc;
        void *t = a;
        a = b;
        b = t;
    }
    ADLBR_LAUNCH_CHECK();
    if (a != u)
        ADLBR_CHECK_HIP(hipMemcpyAsync(u, a, (size_t)op->gi.N * dtype_size(op->storage),
                                       hipMemcpyDeviceToDevice, s));
    return ADLBR_OK;
}
