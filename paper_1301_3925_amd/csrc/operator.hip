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
// is a deterministic gather with no atomics.  2D grids are assembled by
// target tiles that gather their edges from a window of sources (LDS
// atomics only); 3D grids by bins of targets (wave-aggregated global
// atomics, then one block per bin).
//
// Data layout in the workspace (N points, S = 3 or 6 slots):
//   sb     compact slots: 2D (o0, o1) as 4 x int8 (or int16), o2 = -o0-o1;
//          3D (o0, o1, o2) as 12 x int8 (or int16), o3 = -(o0+o1),
//          o4 = o0-o2, o5 = o1+o2.  One vector load per point.
//   w      [S][N] weights in the storage dtype.
//   cnt    [N] uint8 number of incoming edges of each point.
//   pos    [N + 1] int32 start of each point's incoming list; pos[N] is the
//          total number of entries.
//   ent    incoming entries, int32 ((y - z) << 9 | slot << 6 | lane), lane =
//          z mod 64 (the target's position in its wavefront), sorted per row;
//          |y - z| < 2^22.
//   diag   [N] A_zz (double for FP64 storage, float otherwise).
#include <algorithm>
#include <cstddef>
#include <type_traits>
#include <new>

#include "common.h"

struct adlbr_operator {
    adlbr::GridInfo gi;
    int slots;    // 3 or 6
    int storage;  // adlbr_dtype
    int wide;     // int16 compact offsets
    int tiled;    // tiled layout: near edges from LDS tiles, far edges listed
    void *sb;
    void *w;
    uint8_t *cnt;
    int32_t *pos;
    int32_t *ent;
    void *went;        // 3D: [entries] the weight of every incoming entry (EntRec)
    void *diag;
    double *maxdiag;
    double *dtcfl;
    int32_t *rmax;     // 2D: largest tile reach
    int32_t *hnear;    // edges with every offset component <= hnear are not listed (tiled)
    double *wmax;      // largest weight (tiled: scale of the diagonal pass)
    double *rpart;     // per-block reach partials (tiled)
    uint8_t *mask;     // bit q: slot q has a positive weight
    double *part;      // per-block partials of the assembly
    int32_t *trmax;    // 2D: reach of every 64 x 64 tile
    int32_t *brmax;    // 2D: reach of every 4 x 4 brick
    uint8_t *rank;     // 2D: [6][N] rank of every edge in its target's row
    uint32_t *bincnt;  // 3D: edges per bin of targets; 2D: cnt sums per 1024-point chunk
    uint32_t *bincur;  // 3D: placement cursor per bin
    uint32_t *binoff;  // 3D: exclusive scan of bincnt
    int2 *binbuf;      // 3D: (target, entry) grouped by bin
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

// A coordinate outside [0, n) brought back: wrapped (periodic grid,
// mode 1) or mirrored at the half-sample points -1/2 and n - 1/2 (the
// reflecting boundary, mode 2: -1 -> 0, n -> n - 1, period 2n).
__device__ __forceinline__ int fold(int v, int n, int mode) {
    if (mode != 2) return wrap(v, n);
    const int m = wrap(v, 2 * n);
    return m < n ? m : 2 * n - 1 - m;
}

// Target of the directed edge (p, s*o); returns false when it leaves a
// Neumann grid.
template <int DIM, bool PER>
__device__ __forceinline__ bool edge_target(const Coord &p, long long i, const int *o, int s,
                                            const GridInfo &g, long long &t) {
    if (PER) {
        const int x = fold(p.x + s * o[0], g.nx, g.periodic);
        const int y = fold(p.y + s * o[1], g.ny, g.periodic);
        const int zz = DIM == 3 ? fold(p.z + s * o[2], g.nz, g.periodic) : 0;
        t = x + (long long)g.nx * (y + (long long)g.ny * zz);
        return t != i;  // an offset folded onto the point itself is no edge
    } else {
        const int x = p.x + s * o[0], y = p.y + s * o[1];
        const int zz = DIM == 3 ? p.z + s * o[2] : 0;
        if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || zz < 0 || zz >= g.nz) return false;
        t = i + s * (o[0] + (long long)g.nx * (o[1] + (long long)g.ny * (DIM == 3 ? o[2] : 0)));
        return true;
    }
}

// edge_target in 32-bit arithmetic (N < 2^28), for the apply kernels.
template <int DIM, bool PER>
__device__ __forceinline__ bool edge_target32(const Coord &p, int i, const int *o, int s,
                                              const GridInfo &g, int &t) {
    if (PER) {
        const int x = fold(p.x + s * o[0], g.nx, g.periodic);
        const int y = fold(p.y + s * o[1], g.ny, g.periodic);
        const int zz = DIM == 3 ? fold(p.z + s * o[2], g.nz, g.periodic) : 0;
        t = x + g.nx * (y + g.ny * zz);
        return t != i;
    } else {
        const int x = p.x + s * o[0], y = p.y + s * o[1];
        const int zz = DIM == 3 ? p.z + s * o[2] : 0;
        if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || zz < 0 || zz >= g.nz) return false;
        t = i + s * (o[0] + g.nx * (o[1] + g.ny * (DIM == 3 ? o[2] : 0)));
        return true;
    }
}

// ---------------------------------------------------------------- build --

__global__ void k_fill_i32(int32_t *p, long long n, int32_t v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename TW> __device__ __forceinline__ double ld_w(const TW *w, long long i) {
    return (double)w[i];
}

// 3D assembly of the transpose (incoming lists) without per-edge global
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
                                           const double *wq, int k, const GridInfo &g,
                                           int hnear = 0) {
    const int q = k >> 1, sg = (k & 1) ? 1 : -1;
    if (!(wq[q] > 0.0)) return -1;
    if (hnear > 0 && max(max(abs(s[q][0]), abs(s[q][1])), abs(s[q][2])) <= hnear)
        return -1;  // a near edge of the tiled layout: not listed
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

// Pack the slots, convert the weights and record which slots carry a
// positive weight (mask bit q).
template <int DIM, bool WIDE, bool PER, typename TWin, typename TS, typename TA>
__global__ __launch_bounds__(256) void k_compact(
    GridInfo g, const int16_t *__restrict__ off, const TWin *__restrict__ win,
    typename Slots<DIM, WIDE>::store_t *__restrict__ sb, TS *__restrict__ w,
    uint8_t *__restrict__ mask, int32_t *status) {
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
        // a point whose slots do not fit the compact format keeps no edge
        // (zero weights, empty mask), so the operator stays symmetric and
        // its diagonal is not inflated by self-edges; the flag reports it
        const bool packed = Slots<DIM, WIDE>::pack(s, sb, z);
        if (!packed) st |= ADLBR_ST_RANGE;
        p = coords(z, g);
        unsigned m = 0;
        for (int q = 0; q < S; ++q) {
            wq[q] = packed ? (double)win[q * N + z] : 0.0;
            w[widx<S>(q, z, N)] = Conv<TS, TA>::st((TA)wq[q]);
            if (wq[q] > 0.0) m |= 1u << q;
        }
        mask[z] = (uint8_t)m;
    }
    for (int k = 0; k < 2 * S; ++k)
        if (live && edge_k<DIM, PER>(p, z, s, wq, k, g) == -2) st |= ADLBR_ST_RANGE;
    if (live) report(status, z, st);
}

// The listed edges of point z, k = 2q + (sign > 0) in order: f(k, target)
// with target -1 for an edge that is not listed (zero weight, leaves a
// Neumann grid, beyond the 22-bit entry range, or near in the tiled layout).
template <int DIM, bool WIDE, bool PER, typename F>
__device__ __forceinline__ void listed_edges(const GridInfo &g, long long z, bool live,
                                             const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                             const uint8_t *__restrict__ mask, int hnear, F f) {
    constexpr int S = DIM == 2 ? 3 : 6;
    int s[6][3];
    double wq[6];
    for (int q = 0; q < 6; ++q) {
        wq[q] = 0.0;
        for (int c = 0; c < 3; ++c) s[q][c] = 0;
    }
    Coord p{0, 0, 0};
    if (live) {
        Slots<DIM, WIDE> sl;
        sl.load(sb, z);
        const unsigned m = mask[z];
        for (int q = 0; q < S; ++q) {
            for (int c = 0; c < DIM; ++c) s[q][c] = sl.o[q][c];
            wq[q] = (m >> q) & 1u ? 1.0 : 0.0;
        }
        p = coords(z, g);
    }
    for (int k = 0; k < 2 * S; ++k) f(k, live ? edge_k<DIM, PER>(p, z, s, wq, k, g, hnear) : -1ll);
}

// The bins of a block's edge targets lie near the block's own bin (offsets
// are short against the grid), so both binning passes count them first in
// an LDS window of kWinBins bins centred there: one global atomic per
// window bin and block instead of one per bin, wavefront and edge slot,
// which took the global counters of the busy bins out of contention.
// Targets outside the window go to the global counters directly.
constexpr int kWinBins = 2048;

struct BinWindow {
    long long b0;  // bin of window index 0 (may be negative)
    __device__ explicit BinWindow(unsigned block) {
        b0 = (((long long)block * kBS) >> kBinShift) - kWinBins / 2;
    }
    // window index of target t's bin, -1 outside (or no target)
    __device__ int rel(long long t) const {
        if (t < 0) return -1;
        const long long r = (t >> kBinShift) - b0;
        return r >= 0 && r < kWinBins ? (int)r : -1;
    }
};

// Count the listed edges landing in each bin of targets.
template <int DIM, bool WIDE, bool PER>
__global__ __launch_bounds__(256) void k_bin_count(GridInfo g,
                                                   const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                                   const uint8_t *__restrict__ mask,
                                                   const int32_t *__restrict__ hnear,
                                                   uint32_t *__restrict__ bincnt) {
    __shared__ uint32_t hist[kWinBins];
    for (int i = threadIdx.x; i < kWinBins; i += 256) hist[i] = 0;
    __syncthreads();
    const BinWindow win(blockIdx.x);
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    listed_edges<DIM, WIDE, PER>(g, z, z < g.N, sb, mask, *hnear, [&](int, long long t) {
        const int r = win.rel(t);
        bin_append(r, hist, true);  // every lane
        if (t >= 0 && r < 0) atomicAdd(&bincnt[t >> kBinShift], 1u);
    });
    __syncthreads();
    for (int i = threadIdx.x; i < kWinBins; i += 256)
        if (hist[i]) atomicAdd(&bincnt[win.b0 + i], hist[i]);
}

// Sort one row's entries ascending (the order is then independent of the
// order of placement): a transposition network for up to 16 entries,
// insertion sort beyond.
__device__ inline void sort_row(int32_t *e, int c) {
    if (c <= 16) {
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
        for (int i = 1; i < c; ++i) {
            const int32_t key = e[i];
            int j = i - 1;
            while (j >= 0 && e[j] > key) {
                e[j + 1] = e[j];
                --j;
            }
            e[j + 1] = key;
        }
    }
}

// The weights of the 3D incoming entries, one EntRec per entry.  FP32: the
// entry again with its weight in one 8-byte record, so that one vector load
// brings both; other dtypes: the weight alone, beside ent.  (A 16-bit weight
// padded into an 8-byte record was measured slower than the two arrays, 6
// bytes per entry: 637 against 561 us per step of 256^3 in BF16.  FP64
// would need 16 bytes.)
template <typename TS> struct alignas(8) EntW {
    int32_t e;
    TS w;
};
template <typename TS> constexpr bool kPackedEW = sizeof(TS) == 4;
template <typename TS, bool PACKED = kPackedEW<TS>> struct EntRecT {
    typedef TS type;
};
template <typename TS> struct EntRecT<TS, true> {
    typedef EntW<TS> type;
};
template <typename TS> using EntRec = typename EntRecT<TS>::type;

template <typename TS> __device__ __forceinline__ EntRec<TS> make_rec(int32_t e, TS w) {
    if constexpr (kPackedEW<TS>) return EntRec<TS>{e, w};
    else return w;
}
// A 16-bit value read under a per-lane condition is widened by the compiler
// inside the conditional block, which then waits for that one load: the
// loads of a chunk would be serialized.  16-bit reads are therefore made
// unconditional, from an address that is always valid, and the values that
// do not count are dropped afterwards.
template <typename TS> constexpr bool kNarrow = sizeof(TS) == 2;

// Entry i and its weight (-1 and 0 when !ok).
template <typename TS>
__device__ __forceinline__ void load_rec(const EntRec<TS> *__restrict__ went,
                                         const int32_t *__restrict__ ent, long long i, bool ok,
                                         int32_t &v, TS &w) {
    if constexpr (kPackedEW<TS>) {
        // one 8-byte load: the entry, then the weight's bits
        static_assert(sizeof(EntRec<TS>) == 8 && offsetof(EntW<TS>, w) == 4, "record layout");
        const uint2 r = ok ? reinterpret_cast<const uint2 *>(went)[i] : make_uint2(~0u, 0u);
        v = (int32_t)r.x;
        w = __builtin_bit_cast(TS, r.y);
    } else if constexpr (kNarrow<TS>) {
        // entry 0 always exists (the arrays are sized for every possible edge)
        v = ent[ok ? i : 0];
        w = went[ok ? i : 0];
        if (!ok) {
            v = -1;
            w = TS{};
        }
    } else {
        v = ok ? ent[i] : -1;
        w = ok ? went[i] : TS{};
    }
}

// Sort row z (entries e[0..c)), store every entry again with its weight
// (we[i], the weight in the storage dtype; not when we is null) and return
// A_zz, summed as row_diag does.  A row of up to 16 entries is sorted in
// registers and its incoming weights are all requested before any is added.
// cw: a wave-uniform bound on c over the lanes that call this together (16
// when unknown); with cw <= 8 (12) the sort takes 8 (12) rounds instead of
// 16, and only cw weights are requested.
template <int DIM, bool WIDE, bool PER, typename TS, typename TA>
__device__ inline double sort_row_diag(const GridInfo &g, long long z, int32_t *e, int c, int cw,
                                       const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                       const TS *__restrict__ w, EntRec<TS> *__restrict__ we);

// A_zz = own in-grid weights (both signs) + weights of the incoming edges.
template <int DIM, bool WIDE, bool PER, typename TS, typename TA>
__device__ inline double row_diag(const GridInfo &g, long long z, const int32_t *e, int c,
                                  const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                  const TS *__restrict__ w) {
    constexpr int S = DIM == 2 ? 3 : 6;
    const long long N = g.N;
    double d = 0.0;
    Slots<DIM, WIDE> sl;
    sl.load(sb, z);
    const Coord p = coords(z, g);
    for (int q = 0; q < S; ++q) {
        const double wv = (double)Conv<TS, TA>::ld(w[widx<S>(q, z, N)]);
        for (int sg = -1; sg <= 1; sg += 2) {
            long long t;
            if (edge_target<DIM, PER>(p, z, sl.o[q], sg, g, t)) d += wv;
        }
    }
    for (int i = 0; i < c; ++i) {
        const int32_t v = e[i];
        d += (double)Conv<TS, TA>::ld(w[widx<S>((v >> 6) & 7, z + (v >> 9), N)]);
    }
    return d;
}

// Odd-even transposition sort of r[0 .. n) in registers.
template <int n> __device__ __forceinline__ void oe_sort(int32_t *r) {
#pragma unroll
    for (int round = 0; round < n; ++round) {
#pragma unroll
        for (int i = round & 1; i + 1 < n; i += 2) {
            const int32_t a = r[i], bb = r[i + 1];
            r[i] = min(a, bb);
            r[i + 1] = max(a, bb);
        }
    }
}

template <int DIM, bool WIDE, bool PER, typename TS, typename TA>
__device__ inline double sort_row_diag(const GridInfo &g, long long z, int32_t *e, int c, int cw,
                                       const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                       const TS *__restrict__ w, EntRec<TS> *__restrict__ we) {
    const long long N = g.N;
    if (c > 16) {
        sort_row(e, c);
        if (we)
            for (int i = 0; i < c; ++i)
                we[i] = make_rec<TS>(e[i], w[widx<DIM == 2 ? 3 : 6>((e[i] >> 6) & 7, z + (e[i] >> 9), N)]);
        return row_diag<DIM, WIDE, PER, TS, TA>(g, z, e, c, sb, w);
    }
    constexpr int S = DIM == 2 ? 3 : 6;
    // the row's own slots and weights do not depend on the sort: requested
    // first, so they arrive while it runs
    Slots<DIM, WIDE> sl;
    sl.load(sb, z);
    TS wown[S];
#pragma unroll
    for (int q = 0; q < S; ++q) wown[q] = w[widx<S>(q, z, N)];
    int32_t r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) r[i] = i < c ? e[i] : 0x7fffffff;
    // odd-even transposition sort of the first 8, 12 or 16 keys (n rounds
    // sort n keys; keys are distinct and the padding sorts last)
    if (cw <= 8)
        oe_sort<8>(r);
    else if (cw <= 12)
        oe_sort<12>(r);
    else
        oe_sort<16>(r);
    // the weights: up to the wave's bound, from in-grid addresses (the
    // row's own first weight past c) with no per-lane branch, so they are
    // all in flight at once
    TS wr[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        wr[i] = TS{};
        if (i < cw)
            wr[i] = w[i < c ? widx<S>((r[i] >> 6) & 7, z + (r[i] >> 9), N) : widx<S>(0, z, N)];
    }
    TA wi[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i < c) {
            e[i] = r[i];
            if (we) we[i] = make_rec<TS>(r[i], wr[i]);
        }
        wi[i] = i < c ? Conv<TS, TA>::ld(wr[i]) : (TA)0;
    }
    double d = 0.0;
    const Coord p = coords(z, g);
    for (int q = 0; q < S; ++q) {
        const double wv = (double)Conv<TS, TA>::ld(wown[q]);
        for (int sg = -1; sg <= 1; sg += 2) {
            long long t;
            if (edge_target<DIM, PER>(p, z, sl.o[q], sg, g, t)) d += wv;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (i < c) d += (double)wi[i];
    return d;
}

// Place every listed edge (target, entry) in its bin's region of binbuf
// (the same edges as k_bin_count): the block counts its window bins in LDS,
// reserves each bin's range with one global atomic, then places its edges
// within the ranges by LDS cursors.  The order within a bin depends on
// timing; k_bin_build sorts every row.
template <int DIM, bool WIDE, bool PER>
__global__ __launch_bounds__(256) void k_bin_fill(GridInfo g, const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                           const uint8_t *__restrict__ mask, const int32_t *__restrict__ hnear,
                           const uint32_t *__restrict__ binoff, uint32_t *__restrict__ bincur,
                           int2 *__restrict__ binbuf) {
    __shared__ uint32_t hist[kWinBins];  // counts, then cursors
    __shared__ uint32_t base[kWinBins];  // the block's range start in each bin
    for (int i = threadIdx.x; i < kWinBins; i += 256) hist[i] = 0;
    __syncthreads();
    const BinWindow win(blockIdx.x);
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int hn = *hnear;
    listed_edges<DIM, WIDE, PER>(g, z, z < g.N, sb, mask, hn, [&](int, long long t) {
        bin_append(win.rel(t), hist, true);  // every lane
    });
    __syncthreads();
    for (int i = threadIdx.x; i < kWinBins; i += 256) {
        const uint32_t c = hist[i];
        base[i] = c ? atomicAdd(&bincur[win.b0 + i], c) : 0u;
        hist[i] = 0;
    }
    __syncthreads();
    listed_edges<DIM, WIDE, PER>(g, z, z < g.N, sb, mask, hn, [&](int k, long long t) {
        const int r = win.rel(t);
        const int far = t >= 0 && r < 0 ? (int)(t >> kBinShift) : -1;
        const unsigned near_slot = bin_append(r, hist, false);   // every lane
        const unsigned far_slot = bin_append(far, bincur, false);  // every lane
        if (t >= 0) {
            const long long bin = t >> kBinShift;
            const unsigned slot = r >= 0 ? base[r] + near_slot : far_slot;
            const int32_t e = (int32_t)(((z - t) << 9) | ((k >> 1) << 6) | (t & 63));
            binbuf[(long long)binoff[bin] + slot] = make_int2((int)t, e);
        }
    });
}

// One block per bin: per-target counts and offsets in LDS, entries placed at
// their row, rows sorted by (source, slot), diagonal A_zz = own in-grid
// weights + incoming weights, and the maximum diagonal.
template <int DIM, bool WIDE, bool PER, typename TS, typename TA, typename TD>
__global__ __launch_bounds__(256) void k_bin_build(
    GridInfo g, const uint32_t *__restrict__ bincnt, const uint32_t *__restrict__ binoff,
    const int2 *__restrict__ binbuf, const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
    const TS *__restrict__ w, int32_t *__restrict__ pos, uint8_t *__restrict__ cnt,
    int32_t *__restrict__ ent, EntRec<TS> *__restrict__ went, TD *__restrict__ diag,
    double *__restrict__ dpart, int32_t *status) {
    __shared__ int32_t lcnt[kBin];
    __shared__ int32_t loff[kBin];
    __shared__ int32_t scan[256];
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
        if (t == N - 1) pos[N] = (int32_t)(base + run);  // total entry count
        lcnt[tl] = 0;  // becomes the placement cursor
    }
    __syncthreads();
    for (unsigned e = threadIdx.x; e < E; e += 256) {
        const int2 v = binbuf[base + e];
        const int tl = v.x - (int)t0;
        const int k = atomicAdd(&lcnt[tl], 1);
        if (k < 255) ent[base + loff[tl] + k] = v.y;
    }
    // Rows clamped at 255 entries (flagged above) leave the bin's region
    // [base + clamped total, base + E) unwritten, and the apply reads it as
    // the tail of the bin's last row (the next bin starts at base + E).  It
    // is filled with entries that contribute exactly 0: offset 0 on the last
    // row's lane (kBin is a multiple of 64, so that lane is 63), weight 0.
    const int32_t clamped_total = scan[255];
    for (unsigned e = (unsigned)clamped_total + threadIdx.x; e < E; e += 256) {
        ent[base + e] = 63;
        if (went) went[base + e] = make_rec<TS>(63, TS{});
    }
    __syncthreads();
    double dmax = 0.0;
    for (int k = 0; k < 4; ++k) {
        const int tl = threadIdx.x + 256 * k;
        const long long z = t0 + tl;
        if (z >= N) continue;
        const int c = min(lcnt[tl], 255);
        const double d = sort_row_diag<DIM, WIDE, PER, TS, TA>(g, z, ent + base + loff[tl], c, 16,
                                                               sb, w, went ? went + base + loff[tl] : nullptr);
        diag[z] = (TD)d;
        dmax = fmax(dmax, d);
    }
    block_partial_max(dmax, dpart);
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

// ------------------------------------------- 2D tile-gather assembly --
// The incoming lists of a 2D grid are built without any global atomics.
// Every block owns a kTile x kTile tile of targets and scans the sources of
// the edges that can land in it, counting (pass 1) or placing (pass 2) those
// that do with LDS atomics.  On a Neumann grid each source tile S carries its
// own reach r_S (largest offset component over its edges of positive
// weight), so only the band of S within r_S of the target tile is scanned:
// where the tensor field is near isotropic the bands are one point wide and
// the sources are read about once, whatever the largest offset elsewhere.
// On a periodic grid the window is the tile grown by the global R on each
// side (wrapped and capped at the grid size).
constexpr int kTile = 64;
constexpr int kBrick = 4;

// The window of sources along one axis for the tile [t0, t0 + tw).
struct Window {
    int start, len;
};
template <bool PER> __device__ inline Window window_axis(int t0, int tw, int R, int n) {
    Window w;
    if (PER) {
        w.len = min(n, tw + 2 * R);
        w.start = w.len == n ? 0 : t0 - R;
    } else {
        w.start = max(0, t0 - R);
        w.len = min(n, t0 + tw + R) - w.start;
    }
    return w;
}

// Visit every edge (source -> target in this tile) once: f(target local
// index, target linear index, entry).
template <bool WIDE, bool PER, typename F>
__device__ inline void tile_edges(const GridInfo &g, int x0, int y0, int tw, int th, int stride,
                                  int R, const typename Slots<2, WIDE>::store_t *__restrict__ sb,
                                  const uint8_t *__restrict__ mask, int hnear, F f) {
    const Window wx = window_axis<PER>(x0, tw, R, g.nx);
    const Window wy = window_axis<PER>(y0, th, R, g.ny);
    const long long W = (long long)wx.len * wy.len;
    for (long long k = threadIdx.x; k < W; k += blockDim.x) {
        int x = wx.start + (int)(k % wx.len), y = wy.start + (int)(k / wx.len);
        if (PER) {
            x = wrap(x, g.nx);
            y = wrap(y, g.ny);
        }
        const long long z = x + (long long)g.nx * y;
        const unsigned m = mask[z];
        if (!m) continue;
        Slots<2, WIDE> sl;
        sl.load(sb, z);
        const Coord p{x, y, 0};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (!(m & (1u << q))) continue;
            if (max(abs(sl.o[q][0]), abs(sl.o[q][1])) <= hnear) continue;  // near (tiled)
#pragma unroll
            for (int sg = -1; sg <= 1; sg += 2) {
                int tx = x + sg * sl.o[q][0], ty = y + sg * sl.o[q][1];
                if (PER) {
                    tx = fold(tx, g.nx, g.periodic);
                    ty = fold(ty, g.ny, g.periodic);
                }
                if (tx < x0 || tx >= x0 + tw || ty < y0 || ty >= y0 + th) continue;
                long long t;
                if (!edge_target<2, PER>(p, z, sl.o[q], sg, g, t)) continue;
                if (z - t >= (1ll << 22) || z - t <= -(1ll << 22)) continue;  // flagged earlier
                const int32_t e = (int32_t)(((z - t) << 9) | (q << 6) | (t & 63));
                f((ty - y0) * stride + (tx - x0), t, e, z, 2 * q + (sg > 0));
            }
        }
    }
}

template <bool WIDE, typename F>
__device__ inline void source_edges_of(const GridInfo &g, int x, int y, const Slots<2, WIDE> &sl,
                                       unsigned m, int x0, int y0, int tw, int th, int stride,
                                       int hnear, F f);

// The edges of positive weight from source (x, y) into the rectangle
// [x0, x0 + tw) x [y0, y0 + th) (Neumann grid): f(local index, target,
// entry, source, edge index 2q + (sign > 0)).
template <bool WIDE, typename F>
__device__ inline void source_edges(const GridInfo &g, int x, int y, int x0, int y0, int tw,
                                    int th, int stride,
                                    const typename Slots<2, WIDE>::store_t *__restrict__ sb,
                                    const uint8_t *__restrict__ mask, F f) {
    const long long z = x + (long long)g.nx * y;
    Slots<2, WIDE> sl;
    sl.load(sb, z);  // issued with the mask load, not after it
    const unsigned m = mask[z];
    if (!m) return;
    source_edges_of<WIDE>(g, x, y, sl, m, x0, y0, tw, th, stride, 0, f);
}

// source_edges with the source's slots and mask already loaded; edges
// whose offset components are all <= hnear (near edges of the tiled
// layout) are left out.
template <bool WIDE, typename F>
__device__ inline void source_edges_of(const GridInfo &g, int x, int y, const Slots<2, WIDE> &sl,
                                       unsigned m, int x0, int y0, int tw, int th, int stride,
                                       int hnear, F f) {
    const long long z = x + (long long)g.nx * y;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (!(m & (1u << q))) continue;
        if (max(abs(sl.o[q][0]), abs(sl.o[q][1])) <= hnear) continue;
#pragma unroll
        for (int sg = -1; sg <= 1; sg += 2) {
            const int tx = x + sg * sl.o[q][0], ty = y + sg * sl.o[q][1];
            if (tx < x0 || tx >= x0 + tw || ty < y0 || ty >= y0 + th) continue;
            const long long t = tx + (long long)g.nx * ty;
            if (z - t >= (1ll << 22) || z - t <= -(1ll << 22)) continue;  // flagged earlier
            const int32_t e = (int32_t)(((z - t) << 9) | (q << 6) | (t & 63));
            f((ty - y0) * stride + (tx - x0), t, e, z, 2 * q + (sg > 0));
        }
    }
}

// The bricks of [bxa, bxa + nbw) x [bya, bya + nbh) whose reach box meets
// the target rectangle go to the LDS list (at most `nbw * nbh` entries), then
// every point of every listed brick is visited, one thread per point.
// Block-uniform (barriers).
template <bool WIDE, typename F>
__device__ inline void brick_pass(const GridInfo &g, int x0, int y0, int tw, int th, int stride,
                                  int bxa, int bya, int nbw, int nbh,
                                  const int32_t *__restrict__ brmax,
                                  const typename Slots<2, WIDE>::store_t *__restrict__ sb,
                                  const uint8_t *__restrict__ mask, int32_t *list, int32_t *nlist,
                                  int hnear, F f) {
    const int nbx = (g.nx + kBrick - 1) / kBrick;
    if (threadIdx.x == 0) *nlist = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < nbw * nbh; k += blockDim.x) {
        const int bi = bxa + k % nbw, bj = bya + k / nbw;
        const int rb = brmax[bj * nbx + bi];
        if (bi * kBrick - rb < x0 + tw && (bi + 1) * kBrick + rb > x0 &&
            bj * kBrick - rb < y0 + th && (bj + 1) * kBrick + rb > y0)
            list[atomicAdd(nlist, 1)] = bj * nbx + bi;
    }
    __syncthreads();
    const int n = *nlist;
    constexpr int BB = kBrick * kBrick, G = 4;
    // G sources per thread at a time: their slots and masks are requested
    // together (from point 0 for a lane with no source, whose mask is then
    // taken as 0), then their edges are visited
    for (int kb = 0; kb < n * BB; kb += G * (int)blockDim.x) {  // block-uniform
        Slots<2, WIDE> sl[G];
        unsigned m[G];
        int xs[G], ys[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int k = kb + j * (int)blockDim.x + (int)threadIdx.x;
            int x = 0, y = 0;
            bool ok = false;
            if (k < n * BB) {
                const int br = list[k / BB], p = k % BB;
                x = (br % nbx) * kBrick + p % kBrick;
                y = (br / nbx) * kBrick + p / kBrick;
                ok = x < g.nx && y < g.ny;
            }
            const long long z = ok ? x + (long long)g.nx * y : 0;
            sl[j].load(sb, z);
            const unsigned mm = mask[z];
            m[j] = ok ? mm : 0u;
            xs[j] = x;
            ys[j] = y;
        }
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (m[j])
                source_edges_of<WIDE>(g, xs[j], ys[j], sl[j], m[j], x0, y0, tw, th, stride, hnear, f);
    }
    __syncthreads();
}

// Every edge into the target rectangle [x0, x0 + tw) x [y0, y0 + th) (f gets
// the local index (ty - y0) * stride + (tx - x0)).  Neumann grid: a
// kBrick x kBrick brick of sources is visited only if its reach brmax
// reaches the rectangle.  When the bricks within the global reach R of the
// rectangle are at most CAP, they are tested in one pass; otherwise kTile
// source tile by source tile, skipping the part of each tile beyond its own
// reach trmax.  list: LDS scratch of CAP + 1 ints (CAP >= (kTile/kBrick)^2).
// Block-uniform control flow (contains barriers).
template <bool WIDE, bool PER, int CAP, typename F>
__device__ inline void tile_sources(const GridInfo &g, int x0, int y0, int tw, int th, int stride,
                                    int R, const int32_t *__restrict__ trmax,
                                    const int32_t *__restrict__ brmax,
                                    const typename Slots<2, WIDE>::store_t *__restrict__ sb,
                                    const uint8_t *__restrict__ mask, int32_t *list, int hnear,
                                    F f) {
    static_assert(CAP >= (kTile / kBrick) * (kTile / kBrick), "a tile's bricks fit the list");
    if (PER) {
        tile_edges<WIDE, PER>(g, x0, y0, tw, th, stride, R, sb, mask, hnear, f);
        return;
    }
    int32_t *nlist = list + CAP;
    {
        const int bxa = max(0, x0 - R) / kBrick, bxb = min(g.nx - 1, x0 + tw - 1 + R) / kBrick;
        const int bya = max(0, y0 - R) / kBrick, byb = min(g.ny - 1, y0 + th - 1 + R) / kBrick;
        const long long nc = (long long)(bxb - bxa + 1) * (byb - bya + 1);
        if (nc <= CAP) {
            brick_pass<WIDE>(g, x0, y0, tw, th, stride, bxa, bya, bxb - bxa + 1, byb - bya + 1,
                             brmax, sb, mask, list, nlist, hnear, f);
            return;
        }
    }
    const int ntx = (g.nx + kTile - 1) / kTile, nty = (g.ny + kTile - 1) / kTile;
    const int sxa = max(0, x0 - R) / kTile, sxb = min(ntx - 1, (x0 + tw - 1 + R) / kTile);
    const int sya = max(0, y0 - R) / kTile, syb = min(nty - 1, (y0 + th - 1 + R) / kTile);
    for (int sy = sya; sy <= syb; ++sy)
        for (int sx = sxa; sx <= sxb; ++sx) {
            const int r = trmax[sy * ntx + sx];
            const int sx0 = sx * kTile, sy0 = sy * kTile;
            const int ax = max(sx0, x0 - r), bx = min(min(sx0 + kTile, g.nx), x0 + tw + r);
            const int ay = max(sy0, y0 - r), by = min(min(sy0 + kTile, g.ny), y0 + th + r);
            if (ax >= bx || ay >= by) continue;
            const int bxa = ax / kBrick, bya = ay / kBrick;
            brick_pass<WIDE>(g, x0, y0, tw, th, stride, bxa, bya, (bx - 1) / kBrick - bxa + 1,
                             (by - 1) / kBrick - bya + 1, brmax, sb, mask, list, nlist, hnear, f);
        }
}

// Reach of every kBrick x kBrick brick (brmax) and of every kTile x kTile
// tile (trmax): the largest offset component over the edges of positive
// weight that start in it.  One block per tile, one thread per brick.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_tile_rmax(GridInfo g,
                                                   const typename Slots<2, WIDE>::store_t *__restrict__ sb,
                                                   const uint8_t *__restrict__ mask,
                                                   int32_t *__restrict__ trmax,
                                                   int32_t *__restrict__ brmax) {
    static_assert((kTile / kBrick) * (kTile / kBrick) == 256, "one brick per thread");
    __shared__ int red[4];
    const int ntx = (g.nx + kTile - 1) / kTile;
    const int nbx = (g.nx + kBrick - 1) / kBrick, nby = (g.ny + kBrick - 1) / kBrick;
    const int bi = (int)(blockIdx.x % ntx) * (kTile / kBrick) + (int)threadIdx.x % (kTile / kBrick);
    const int bj = (int)(blockIdx.x / ntx) * (kTile / kBrick) + (int)threadIdx.x / (kTile / kBrick);
    int r = 0;
    if (bi < nbx && bj < nby) {
        for (int p = 0; p < kBrick * kBrick; ++p) {
            const int x = bi * kBrick + p % kBrick, y = bj * kBrick + p / kBrick;
            if (x >= g.nx || y >= g.ny) continue;
            const long long z = x + (long long)g.nx * y;
            const unsigned m = mask[z];
            if (!m) continue;
            Slots<2, WIDE> sl;
            sl.load(sb, z);
            for (int q = 0; q < 3; ++q)
                if (m & (1u << q)) r = max(r, max(abs(sl.o[q][0]), abs(sl.o[q][1])));
        }
        brmax[bj * nbx + bi] = r;
    }
    for (int d = 32; d > 0; d >>= 1) r = max(r, __shfl_xor(r, d));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) trmax[blockIdx.x] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// R = the largest tile reach.
__global__ __launch_bounds__(256) void k_rmax_tiles(const int32_t *__restrict__ trmax, long long n,
                                                    int32_t *R) {
    __shared__ int red[4];
    int r = 0;
    for (long long k = threadIdx.x; k < n; k += blockDim.x) r = max(r, trmax[k]);
    for (int d = 32; d > 0; d >>= 1) r = max(r, __shfl_xor(r, d));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) *R = max(max(red[0], red[1]), max(red[2], red[3]));
}

// Pass 1: incoming count of every target (clamped to 255, flagged above),
// and the rank of every edge in its target's row (rank[2q + (sign > 0)][z]
// for the edge of slot q and that sign from source z; 255 = beyond the
// clamp).  The ranks of one row are distinct and in no fixed order: the row
// is sorted once placed.
template <bool WIDE, bool PER>
__global__ __launch_bounds__(256) void k_tile_count(GridInfo g,
                                                    const typename Slots<2, WIDE>::store_t *__restrict__ sb,
                                                    const uint8_t *__restrict__ mask,
                                                    const int32_t *__restrict__ Rp,
                                                    const int32_t *__restrict__ trmax,
                                                    const int32_t *__restrict__ brmax,
                                                    const int32_t *__restrict__ hnear,
                                                    uint8_t *__restrict__ cnt,
                                                    uint8_t *__restrict__ rank, int32_t *status) {
    __shared__ int32_t lc[kTile * kTile];
    constexpr int CAP = (kTile + 128) / kBrick * ((kTile + 128) / kBrick);  // one pass for R <= 64
    __shared__ int32_t list[CAP + 1];
    const int ntx = (g.nx + kTile - 1) / kTile;
    const int x0 = (int)(blockIdx.x % ntx) * kTile, y0 = (int)(blockIdx.x / ntx) * kTile;
    const int tw = min(kTile, g.nx - x0), th = min(kTile, g.ny - y0);
    for (int k = threadIdx.x; k < kTile * kTile; k += blockDim.x) lc[k] = 0;
    __syncthreads();
    const long long N = g.N;
    tile_sources<WIDE, PER, CAP>(g, x0, y0, tw, th, kTile, *Rp, trmax, brmax, sb, mask, list,
                                 *hnear, [&](int tl, long long, int32_t, long long z, int k) {
                                     const int r = atomicAdd(&lc[tl], 1);
                                     rank[k * N + z] = (uint8_t)min(r, 255);
                                 });
    __syncthreads();
    for (int k = threadIdx.x; k < tw * th; k += blockDim.x) {
        const int lx = k % tw, ly = k / tw;
        const long long t = (x0 + lx) + (long long)g.nx * (y0 + ly);
        const int c = lc[ly * kTile + lx];
        cnt[t] = (uint8_t)min(c, 255);
        if (c > 255) report(status, t, ADLBR_ST_INCOMING);
    }
}

// Sum of cnt over each chunk of 1024 consecutive points.
__global__ __launch_bounds__(256) void k_chunk_sum(const uint8_t *__restrict__ cnt, long long N,
                                                   int32_t *__restrict__ csum) {
    __shared__ int32_t red[256];
    const long long base = (long long)blockIdx.x * 1024;
    int32_t v = 0;
    for (int k = 0; k < 4; ++k) {
        const long long z = base + threadIdx.x * 4 + k;
        if (z < N) v += cnt[z];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) csum[blockIdx.x] = red[0];
}

// pos[z] = exclusive prefix of cnt in linear order (chunk offsets coff from
// the scan of the chunk sums).
__global__ __launch_bounds__(256) void k_chunk_pos(const uint8_t *__restrict__ cnt, long long N,
                                                   const int32_t *__restrict__ coff,
                                                   int32_t *__restrict__ pos) {
    __shared__ int32_t scan[256];
    const long long base = (long long)blockIdx.x * 1024;
    int32_t c4[4], sum = 0;
    for (int k = 0; k < 4; ++k) {
        const long long z = base + threadIdx.x * 4 + k;
        c4[k] = z < N ? cnt[z] : 0;
        sum += c4[k];
    }
    scan[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const int32_t add = threadIdx.x >= (unsigned)d ? scan[threadIdx.x - d] : 0;
        __syncthreads();
        scan[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = coff[blockIdx.x] + scan[threadIdx.x] - sum;
    for (int k = 0; k < 4; ++k) {
        const long long z = base + threadIdx.x * 4 + k;
        if (z < N) pos[z] = run;
        run += c4[k];
        if (z == N - 1) pos[N] = run;  // total entry count
    }
}

// Pass 2: every source places its edges at pos[target] + rank (no atomics,
// one thread per source, the same edges as pass 1).
template <bool WIDE, bool PER>
__global__ __launch_bounds__(256) void k_place2d(GridInfo g,
                                                 const typename Slots<2, WIDE>::store_t *__restrict__ sb,
                                                 const uint8_t *__restrict__ mask,
                                                 const uint8_t *__restrict__ rank,
                                                 const int32_t *__restrict__ pos,
                                                 const int32_t *__restrict__ hnear,
                                                 int32_t *__restrict__ ent) {
    const long long N = g.N;
    const int h = *hnear;
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= N) return;
    Slots<2, WIDE> sl;
    sl.load(sb, z);
    const unsigned m = mask[z];
    if (!m) return;
    uint8_t rk[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) rk[k] = rank[k * N + z];
    const Coord p = coords(z, g);
    // the six targets first, then their row starts from in-grid addresses
    // (z itself for an edge that is not placed) with no branch around the
    // loads, so all six are in flight at once, then the stores
    long long tt[6];
    bool ok[6];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            long long t = z;
            bool v = (m >> q) & 1u;
            v = v && max(abs(sl.o[q][0]), abs(sl.o[q][1])) > h;  // near edges (tiled) unlisted
            v = v && edge_target<2, PER>(p, z, sl.o[q], k ? 1 : -1, g, t);
            v = v && z - t < (1ll << 22) && z - t > -(1ll << 22);  // else flagged earlier
            v = v && rk[2 * q + k] != 255;
            ok[2 * q + k] = v;
            tt[2 * q + k] = v ? t : z;
        }
    int32_t pt[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) pt[e] = pos[tt[e]];
#pragma unroll
    for (int e = 0; e < 6; ++e)
        if (ok[e])
            ent[(long long)pt[e] + rk[e]] =
                (int32_t)(((z - tt[e]) << 9) | ((e >> 1) << 6) | (tt[e] & 63));
}

// Maximum of v over the wavefront, in every lane (all 64 lanes must call it).
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// Pass 3: sort every row, store the weight of each entry beside it (went,
// where not null), take the diagonal A_zz and the block's largest diagonal
// (dpart), one thread per target.  The rows of a block's 256 consecutive
// targets are one run of ent; when it fits, it is staged in LDS with
// coalesced loads and stores around the per-thread sort.
template <int DIM, bool WIDE, bool PER, typename TS, typename TA, typename TD>
__global__ __launch_bounds__(256) void k_rows(GridInfo g,
                                              const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                              const TS *__restrict__ w,
                                              const uint8_t *__restrict__ cnt,
                                              const int32_t *__restrict__ pos,
                                              int32_t *__restrict__ ent, EntRec<TS> *__restrict__ went,
                                              TD *__restrict__ diag, double *__restrict__ dpart) {
    constexpr int kCap = 16 * 256;
    __shared__ int32_t rows[kCap];
    const long long N = g.N;
    const long long t0 = (long long)blockIdx.x * blockDim.x, t = t0 + threadIdx.x;
    const int p0 = pos[t0], p1 = pos[t0 + 256 < N ? t0 + 256 : N];
    const int c = t < N ? (int)cnt[t] : 0, p = t < N ? pos[t] : 0;  // requested with the staging
    const bool staged = p1 - p0 <= kCap;  // block-uniform
    if (staged) {  // all of a thread's loads first, then its LDS stores
        const int n = p1 - p0;
        int32_t v[kCap / 256];
#pragma unroll
        for (int it = 0; it < kCap / 256; ++it) {
            const int i = (int)threadIdx.x + 256 * it;
            v[it] = 0;
            if (256 * it < n) v[it] = ent[p0 + (i < n ? i : 0)];  // block-uniform test
        }
#pragma unroll
        for (int it = 0; it < kCap / 256; ++it) {
            const int i = (int)threadIdx.x + 256 * it;
            if (i < n) rows[i] = v[it];
        }
        __syncthreads();
    }
    const int cw = wave_max_i(c);  // all lanes
    double dmax = 0.0;
    if (t < N) {
        // two calls, so that the staged one addresses LDS directly (not
        // through flat addressing)
        const double d = staged ? sort_row_diag<DIM, WIDE, PER, TS, TA>(g, t, rows + (p - p0), c,
                                                                        cw, sb, w,
                                                                        went ? went + p : nullptr)
                                : sort_row_diag<DIM, WIDE, PER, TS, TA>(g, t, ent + p, c, cw, sb,
                                                                        w,
                                                                        went ? went + p : nullptr);
        diag[t] = (TD)d;
        dmax = d;
    }
    if (staged) {
        __syncthreads();
        for (int i = threadIdx.x; i < p1 - p0; i += blockDim.x) ent[p0 + i] = rows[i];
    }
    block_partial_max(dmax, dpart);
}

__global__ void k_copy_u32(const uint32_t *a, uint32_t *b, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}


// In-place exclusive scan of bsum[0 .. nb) by one block of 256 threads:
// 4096 values a round, 16 consecutive ones per thread (one round covers the
// chunk sums of a 2048^2 grid).
__global__ __launch_bounds__(256) void k_scan_top(int32_t *bsum, long long nb) {
    constexpr int V = 16;
    __shared__ int32_t lds[256];
    int32_t carry = 0;
    for (long long b0 = 0; b0 < nb; b0 += 256 * V) {
        const long long i0 = b0 + (long long)threadIdx.x * V;
        int32_t v[V], sum = 0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            v[k] = i0 + k < nb ? bsum[i0 + k] : 0;
            sum += v[k];
        }
        int32_t total;
        int32_t run = carry + block_excl_scan256(sum, lds, total);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (i0 + k < nb) bsum[i0 + k] = run;
            run += v[k];
        }
        carry += total;
    }
}

// dt_CFL = 1 / max_z A_zz from the per-block maxima.
__global__ __launch_bounds__(256) void k_cfl(const double *dpart, long long nb, double *maxdiag,
                                             double *dtcfl) {
    const double m = reduce_partials(dpart, nb, true);
    if (threadIdx.x != 0) return;
    *maxdiag = m;
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
// owns [lo, hi) relative to start.  pos holds every row's start and, at
// index N, the total entry count, so no scan is needed.
// Where the weight of an incoming edge is read: from the list of entry
// weights beside the entries (3D: a gather from the source's slot plane
// would touch another plane of the grid) or from the source's own weights
// (2D: those lines are in cache from the own part of nearby rows, and the
// gather costs less than streaming a second list).
template <int DIM> constexpr bool kInlineW = DIM == 3 && ADLBR_W3D_INLINE;

struct WaveLists {
    int start;
    unsigned total, lo, hi;
};

__device__ __forceinline__ WaveLists wave_lists(const int32_t *__restrict__ pos, long long z,
                                                long long N) {
    // All 64 lanes call this; the wave's rows are 64 consecutive points from
    // a multiple of 64.  A row's end is the next row's start (the next
    // lane's pos), so the counts are not read; the wave's end is one
    // scalar load.
    WaveLists L;
    const int lane = (int)(threadIdx.x & 63u);
    const int z0 = __builtin_amdgcn_readfirstlane((int)(z - lane));  // N < 2^28
    if ((long long)z0 >= N) {
        L.start = 0;
        L.total = L.lo = L.hi = 0u;
        return L;
    }
    const int zend = z0 + 64 < N ? z0 + 64 : (int)N;
    const int pz = z < N ? pos[z] : 0;
    const int pend = pos[zend];
    L.start = __builtin_amdgcn_readfirstlane(pz);
    const int pnext = __shfl_down(pz, 1, 64);
    const int phi = lane == 63 || z + 1 >= N ? pend : pnext;
    L.total = (unsigned)(pend - L.start);
    L.lo = z < N ? (unsigned)(pz - L.start) : 0u;
    L.hi = z < N ? (unsigned)(phi - L.start) : 0u;
    return L;
}

// Own part of row z: sum over slots o and signs s with z + s o in the grid
// of w_o(z) (u(z) - u(z + s o)).  Split in two so that a kernel can issue
// these loads before the dependent loads of the incoming part: issue()
// loads the weights and the neighbour values (u(z) where an edge is
// missing, so its term is exactly 0), sum() adds them up.
template <typename TS> struct W3 {
    TS v[3];
};
template <typename TS> struct W6 {
    TS v[6];
};

template <int DIM, bool WIDE, bool PER, typename TS, typename TA, typename TU> struct OwnPart {
    static constexpr int S = DIM == 2 ? 3 : 6;
    TA wq[S];
    TA un[2 * S];
    __device__ __forceinline__ void issue(const GridInfo &g, long long z, bool live, TA uz,
                                          const TU *__restrict__ u,
                                          const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                          const TS *__restrict__ w) {
        // Every load reads an address in the grid (point 0 for a dead lane,
        // the point itself for a missing edge) and the values that do not
        // count are dropped afterwards, so there is no per-lane branch around
        // a load and the wave issues them all before it waits.
        const int N = (int)g.N, zi = live ? (int)z : 0;  // N < 2^28, S N < 2^31
        Slots<DIM, WIDE> sl;
        sl.load(sb, zi);
        const Coord p = coords(zi, g);
        W3<TS> w3{};  // 2D: the three point-major weights in one load
        TS wr[S];
        if (S == 3) w3 = ((const W3<TS> *)w)[zi];
        W6<TS> w6{};  // 3D point-major: the six weights in one record
        if (S == 6 && !ADLBR_W3D_INLINE) w6 = ((const W6<TS> *)w)[zi];
#pragma unroll
        for (int q = 0; q < S; ++q)
            wr[q] = S == 3 ? w3.v[q < 3 ? q : 0]
                           : (!ADLBR_W3D_INLINE ? w6.v[q < 6 ? q : 0] : w[widx32<S>(q, zi, N)]);
        bool okq[2 * S];
        TU ur[2 * S];
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                int t = 0;
                okq[2 * q + k] = live && edge_target32<DIM, PER>(p, zi, sl.o[q], k ? 1 : -1, g, t);
                ur[2 * q + k] = u[(unsigned)(okq[2 * q + k] ? t : zi)];
            }
#pragma unroll
        for (int q = 0; q < S; ++q) {
            wq[q] = live ? Conv<TS, TA>::ld(wr[q]) : (TA)0;
#pragma unroll
            for (int k = 0; k < 2; ++k)
                un[2 * q + k] = okq[2 * q + k] ? Conv<TU, TA>::ld(ur[2 * q + k]) : uz;
        }
    }
    __device__ __forceinline__ TA sum(TA uz) const {
        TA acc = (TA)0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            TA part = (TA)0;
            part += uz - un[2 * q];
            part += uz - un[2 * q + 1];
            acc += wq[q] * part;
        }
        return acc;
    }
};

// Chunks of 64 entries whose loads a wave has in flight at once: 8 with
// 32-bit arithmetic; 4 with FP64, whose wider values would otherwise cost
// occupancy (109 instead of 81 registers in the 3D step).
template <typename TA> constexpr int kPreOf = sizeof(TA) == 8 ? 4 : 8;

// Chunk [e0, e0 + 64) of a wave's entries: this lane's edge value
// w_slot(y) (u(row) - u(y)), 0 past the end; the weight is wv (INLINE_W,
// loaded from the entry weights with the entry) or gathered from w.  Split in
// two so that a wave can issue the gathers of several chunks before it waits
// for any: issue() loads from addresses that are always in the grid (point
// z0 for lanes past the end, whose values are then dropped), with no per-lane
// branch around the loads; value() forms the product.  All 64 lanes must call
// issue().
template <bool INLINE_W, int S, typename TS, typename TA, typename TU> struct InEdge {
    TA ur;
    TS wy;
    TU uy;
    bool ok;
    __device__ __forceinline__ void issue(const WaveLists &L, long long z0, long long N, TA uz,
                                          int32_t v, TS wv, unsigned e0, const TU *__restrict__ u,
                                          const TS *__restrict__ w) {
        const int lane = (int)(threadIdx.x & 63u);
        ok = e0 + lane < L.total;
        ur = __shfl(uz, ok ? (v & 63) : 0, 64);  // all lanes take part
        wy = INLINE_W ? wv : TS{};
        uy = TU{};
        // a wave with entries left has z0 < N; N < 2^28 points, S N < 2^31
        const int y = ok ? (int)z0 + (v & 63) + (v >> 9) : (e0 < L.total ? (int)z0 : 0);
        if constexpr (kNarrow<TS> || kNarrow<TU>) {  // unconditional (see kNarrow)
            if (!INLINE_W) wy = w[widx32<S>(ok ? (v >> 6) & 7 : 0, y, (int)N)];
            uy = u[(unsigned)y];
        } else if (e0 < L.total) {  // wave-uniform: skip chunks past the lists
            if (!INLINE_W) wy = w[widx32<S>(ok ? (v >> 6) & 7 : 0, y, (int)N)];
            uy = u[(unsigned)y];
        }
    }
    __device__ __forceinline__ TA value() const {
        return ok ? Conv<TS, TA>::ld(wy) * (ur - Conv<TU, TA>::ld(uy)) : (TA)0;
    }
};

// Rows of one wave from a window of evaluated incoming edges: the values of
// the window's KPRE chunks (64 entries each, from entry eb on) go to the
// wave's slice of LDS, then every lane adds, in list order, the values of
// its own row that fall in the window.  Across the windows each row's
// incoming part is thus a plain sum in list order (deterministic).  LDS
// serves the wave's reads in order after its writes; the wave barriers keep
// the compiler from moving the accesses across them.  Needs blocks of kBS
// threads; all 64 lanes of the wave call it together.
template <typename TA, int KPRE>
__device__ __forceinline__ void add_window_rows(const WaveLists &L, unsigned eb,
                                                const TA (&val)[KPRE], TA &acc) {
    __shared__ TA win[kBS / 64][64 * KPRE];
    TA *sw = win[threadIdx.x >> 6];
    const unsigned lane = threadIdx.x & 63u;
#pragma unroll
    for (int j = 0; j < KPRE; ++j) sw[64 * j + lane] = val[j];
    __builtin_amdgcn_wave_barrier();
    const unsigned end = eb + 64u * KPRE;
    const unsigned lo = L.lo > eb ? L.lo : eb;
    const unsigned hi = L.hi < end ? L.hi : end;
    unsigned e = lo;
    for (; e + 4 <= hi; e += 4) {
        const TA a0 = sw[e - eb], a1 = sw[e + 1 - eb], a2 = sw[e + 2 - eb], a3 = sw[e + 3 - eb];
        acc += a0;
        acc += a1;
        acc += a2;
        acc += a3;
    }
    for (; e < hi; ++e) acc += sw[e - eb];
    __builtin_amdgcn_wave_barrier();
}

// Incoming part of the rows of one wavefront, computed cooperatively: the
// wave's entries are taken 64 at a time (coalesced loads, every lane busy),
// each lane evaluates one edge, and each row's values are then summed by
// its own lane (add_window_rows).  Up to kPre chunks are loaded before any
// is summed, so their memory latencies overlap.  All 64 lanes must call
// this.
template <bool INLINE_W, int S, typename TS, typename TA, typename TU>
__device__ __forceinline__ TA wave_incoming(const WaveLists &L, long long z, long long N, TA uz,
                                            const TU *__restrict__ u, const TS *__restrict__ w,
                                            const int32_t *__restrict__ ent,
                                            const EntRec<TS> *__restrict__ went) {
    constexpr int kPre = kPreOf<TA>;
    const int lane = (int)(threadIdx.x & 63u);
    const long long z0 = z & ~63ll;
    TA acc = (TA)0;
    for (unsigned eb = 0; eb < L.total; eb += 64 * kPre) {
        int32_t v[kPre];
        TS wv[kPre];
        TA val[kPre];
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            const unsigned e = eb + 64 * j + lane;
            if (INLINE_W) {
                load_rec<TS>(went, ent, L.start + e, e < L.total, v[j], wv[j]);
            } else {
                v[j] = e < L.total ? ent[L.start + e] : -1;
                wv[j] = TS{};
            }
        }
        InEdge<INLINE_W, S, TS, TA, TU> ie[kPre];
#pragma unroll
        for (int j = 0; j < kPre; ++j) ie[j].issue(L, z0, N, uz, v[j], wv[j], eb + 64 * j, u, w);
#pragma unroll
        for (int j = 0; j < kPre; ++j) val[j] = ie[j].value();
        add_window_rows<TA, kPre>(L, eb, val, acc);
    }
    return acc;
}


// One block of out = A u (STEP = false) or u - h A u (STEP = true): every
// wave takes kApplyPPT consecutive groups of 64 rows (a block kApplyPoints
// rows) and interleaves them -- all groups' own loads, then the entry loads
// and gathers of the same chunk in every group, then the reductions -- so
// several independent memory chains are in flight per wave.  blk is the
// block's index within its grid.  Shared by the single-operator and the
// batched kernels, so both give bit-identical results.  INLW: the weights
// of incoming edges come with their entries (went) instead of from the
// sources' weights (2D operators with records in a batch).
template <int DIM, bool WIDE, bool PER, bool STEP, typename TS, typename TA, bool INLW = kInlineW<DIM>>
__device__ __forceinline__ void apply_block(
    const GridInfo &g, long long blk, const TS *__restrict__ u, TS *__restrict__ out,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const TS *__restrict__ w,
    const uint8_t *__restrict__ cnt, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ ent, const EntRec<TS> *__restrict__ went, TA h) {
    constexpr int P = kApplyPPT, kPre = kPreOf<TA>;
    const long long N = g.N;
    const int lane = (int)(threadIdx.x & 63u);
    const long long zw = wave_group(g, blk, P);
    WaveLists L[P];
    TA uz[P], acc[P];
    OwnPart<DIM, WIDE, PER, TS, TA, TS> own[P];
    unsigned tmax = 0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const long long z = zw + 64 * k + lane;
        L[k] = wave_lists(pos, z, N);
        uz[k] = z < N ? Conv<TS, TA>::ld(u[z]) : (TA)0;
        acc[k] = (TA)0;
        tmax = L[k].total > tmax ? L[k].total : tmax;
    }
    int32_t v[P][kPre];
    TS wv[P][kPre];
    auto load_chunks = [&](unsigned eb) {
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int j = 0; j < kPre; ++j) {
                const unsigned e = eb + 64 * j + lane;
                if (INLW) {
                    load_rec<TS>(went, ent, L[k].start + e, e < L[k].total, v[k][j], wv[k][j]);
                } else {
                    v[k][j] = e < L[k].total ? ent[L[k].start + e] : -1;
                    wv[k][j] = TS{};
                }
            }
    };
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const long long z = zw + 64 * k + lane;
        own[k].issue(g, z, z < N, uz[k], u, sb, w);
    }
    for (unsigned eb = 0; eb < tmax; eb += 64 * kPre) {
        load_chunks(eb);
        TA val[P][kPre];
        InEdge<INLW, DIM == 2 ? 3 : 6, TS, TA, TS> ie[P][kPre];
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int j = 0; j < kPre; ++j)
                ie[k][j].issue(L[k], zw + 64 * k, N, uz[k], v[k][j], wv[k][j], eb + 64 * j, u, w);
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int j = 0; j < kPre; ++j) val[k][j] = ie[k][j].value();
#pragma unroll
        for (int k = 0; k < P; ++k) add_window_rows<TA, kPre>(L[k], eb, val[k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const long long z = zw + 64 * k + lane;
        if (z >= N) continue;
        const TA a = acc[k] + own[k].sum(uz[k]);
        out[z] = Conv<TS, TA>::st(STEP ? uz[k] - h * a : a);
    }
}

template <int DIM, bool WIDE, bool PER, bool STEP, typename TS, typename TA>
__global__ __launch_bounds__(kBS) void k_apply(
    GridInfo g, const TS *__restrict__ u, TS *__restrict__ out,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const TS *__restrict__ w,
    const uint8_t *__restrict__ cnt, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ ent, const EntRec<TS> *__restrict__ went, double dt,
    const double *__restrict__ dtcfl, int dt_mode) {
    const TA h = (TA)(dt_mode == ADLBR_DT_CFL ? dt * dtcfl[0] : dt);
    apply_block<DIM, WIDE, PER, STEP, TS, TA>(
        g, strip_block(xcd_block(blockIdx.x, gridDim.x), g, kApplyPoints), u, out, sb, w, cnt,
        pos, ent, went, h);
}


// Explicit step of a vector-valued image, ncomp <= kMaxComp components
// [c][N] stepped with one operator (the paper's extension to vector-valued
// images: each component independently, coupled only through the common
// tensor).  A wave loads its rows' slots, weights and incoming entries once
// and uses them for every component; each component's arithmetic is the
// single-component kernel's in the same order, so every component comes out
// bit-identical to stepping it alone.
constexpr int kMaxComp = 4;

template <int DIM, bool WIDE, bool PER, typename TS, typename TA>
__global__ __launch_bounds__(kBS) void k_step_multi(
    GridInfo g, int ncomp, const TS *__restrict__ u, TS *__restrict__ out,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const TS *__restrict__ w,
    const int32_t *__restrict__ pos, const int32_t *__restrict__ ent,
    const EntRec<TS> *__restrict__ went, double dt, const double *__restrict__ dtcfl,
    int dt_mode) {
    constexpr int kPre = kPreOf<TA>;
    constexpr int S = DIM == 2 ? 3 : 6;
    const TA h = (TA)(dt_mode == ADLBR_DT_CFL ? dt * dtcfl[0] : dt);
    const long long blk = strip_block(xcd_block(blockIdx.x, gridDim.x), g, kApplyPoints);
    const long long N = g.N;
    const int lane = (int)(threadIdx.x & 63u);
    const long long z0 = wave_group(g, blk, 1);
    const long long z = z0 + lane;
    const WaveLists L = wave_lists(pos, z, N);
    TA uz[kMaxComp], acc[kMaxComp], owns[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
        uz[c] = acc[c] = owns[c] = (TA)0;
        if (c < ncomp) {
            uz[c] = z < N ? Conv<TS, TA>::ld(u[c * N + z]) : (TA)0;
            OwnPart<DIM, WIDE, PER, TS, TA, TS> own;
            own.issue(g, z, z < N, uz[c], u + c * N, sb, w);
            owns[c] = own.sum(uz[c]);
        }
    }
    for (unsigned eb = 0; eb < L.total; eb += 64 * kPre) {
        int32_t v[kPre];
        TS wv[kPre];
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            const unsigned e = eb + 64 * j + lane;
            if (kInlineW<DIM>) {
                load_rec<TS>(went, ent, L.start + e, e < L.total, v[j], wv[j]);
            } else {
                v[j] = e < L.total ? ent[L.start + e] : -1;
                wv[j] = TS{};
            }
        }
#pragma unroll
        for (int c = 0; c < kMaxComp; ++c) {
            if (c >= ncomp) continue;
            InEdge<kInlineW<DIM>, S, TS, TA, TS> ie[kPre];
            TA val[kPre];
#pragma unroll
            for (int j = 0; j < kPre; ++j)
                ie[j].issue(L, z0, N, uz[c], v[j], wv[j], eb + 64 * j, u + c * N, w);
#pragma unroll
            for (int j = 0; j < kPre; ++j) val[j] = ie[j].value();
            add_window_rows<TA, kPre>(L, eb, val, acc[c]);
        }
    }
    if (z >= N) return;
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
        if (c < ncomp) {
            const TA a = acc[c] + owns[c];
            out[c * N + z] = Conv<TS, TA>::st(uz[c] - h * a);
        }
}

// The problem that block b belongs to (first_block ascending): the lanes of
// a wave test 64 descriptors at once and the highest lane whose first block
// is <= b wins, so the search costs one round of loads, not a chain of
// dependent ones.  Wave-uniform result.
__device__ __forceinline__ int find_prob(const BatchProb *__restrict__ probs, int nprob, long long b) {
    const int lane = (int)(threadIdx.x & 63u);
    int idx = 0;
    for (int base = 0; base < nprob; base += 64) {
        const int i = base + lane;
        const bool le = i < nprob && probs[i].first_block <= b;
        const unsigned long long m = __ballot(le);
        if (m) idx = base + 63 - __clzll((long long)m);
        if (m != ~0ull) break;  // the remaining descriptors start after b
    }
    return idx;
}

// Batched explicit step: one launch advances every problem of a class by one
// step.  Blocks are laid out problem after problem (first_block ascending);
// a block finds its problem (find_prob), then runs the single-operator block
// body.  XCD: remap block indices so that each XCD takes a contiguous range
// (neighbouring blocks share its L2).
template <int DIM, bool WIDE, bool PER, typename TS, typename TA, bool XCD, bool INLW = kInlineW<DIM>>
__global__ __launch_bounds__(kBS) void k_apply_batch(const BatchProb *__restrict__ probs, int nprob,
                                                     int parity) {
    const long long b = XCD ? xcd_block(blockIdx.x, gridDim.x) : (long long)blockIdx.x;
    const BatchProb &P = probs[find_prob(probs, nprob, b)];
    const GridInfo g = P.g;
    const TA h = (TA)(P.dt_mode == ADLBR_DT_CFL ? P.dt * P.dtcfl[0] : P.dt);
    apply_block<DIM, WIDE, PER, true, TS, TA, INLW>(
        g, strip_block(b - P.first_block, g, kApplyPoints), (const TS *)P.u[parity], (TS *)P.u[parity ^ 1],
        (const typename Slots<DIM, WIDE>::store_t *)P.sb, (const TS *)P.w, P.cnt, P.pos, P.ent,
        (const EntRec<TS> *)P.went, h);
}

// dst = src for every problem (u[1] -> u[0] after an odd number of steps).
template <typename TS>
__global__ __launch_bounds__(kBS) void k_copy_batch(const BatchProb *__restrict__ probs, int nprob) {
    const long long b = blockIdx.x;
    const BatchProb &P = probs[find_prob(probs, nprob, b)];
    for (int k = 0; k < P.block_points / kBS; ++k) {
        const long long z = (b - P.first_block) * P.block_points + k * kBS + threadIdx.x;
        if (z < P.g.N) ((TS *)P.u[0])[z] = ((const TS *)P.u[1])[z];
    }
}

// ----------------------------------------------------------- tiled apply --
// The explicit step with the u of a tile of targets and its halo staged in
// LDS (the tiled layout, ADLBR_OP_TILED).  Edges whose offset has all
// components within the halo h ("near" edges) never leave the staged
// region: a block finds every near edge that lands in its tile by visiting
// the sources of tile + halo, and sums them in LDS; only the "far" edges
// (some component beyond h) are listed by the assembly.  h is the
// operator's own reach, capped by the halo the LDS holds (2D 8, 3D 2), so a
// near-isotropic operator has no list at all.
//   own part       every edge of the target, in FP32 registers, neighbours
//                  from LDS (near) or from HBM (far), in slot order;
//   near incoming  scattered into a 64-bit fixed-point accumulator per
//                  target with LDS integer atomics: integer sums do not
//                  depend on the order of the additions, so the result is
//                  deterministic.  Scale 2^s per block from max A_zz and
//                  the range of u over the staged region: every term is at
//                  most M = max A_zz * range (a weight is at most its
//                  source's A_zz), s puts M below 2^50, and at most
//                  (2h+1)^d - 1 <= 288 terms reach a target, so the sum
//                  stays below 2^59; a term's rounding is at most
//                  2^-49 M;
//   far incoming   the target's list, in its sorted order, in FP32.
// A u = own + near + far, added in that order.
template <int DIM> struct TileCfg;
template <> struct TileCfg<2> {
    static constexpr int TX = 64, TY = 16, TZ = 1, HMAX = 8;
};
template <> struct TileCfg<3> {
    static constexpr int TX = 32, TY = 8, TZ = 8, HMAX = 2;
};
template <int DIM> struct Tile {
    using C = TileCfg<DIM>;
    static constexpr int TX = C::TX, TY = C::TY, TZ = C::TZ, HMAX = C::HMAX;
    static constexpr int T = TX * TY * TZ;                       // targets per block
    static constexpr int HX = TX + 2 * HMAX, HY = TY + 2 * HMAX;
    static constexpr int HZ = DIM == 3 ? TZ + 2 * HMAX : 1;
    static constexpr int H = HX * HY * HZ;                       // staged points at most
    static constexpr int PT = T / kBS;                           // targets per thread
    static_assert(T % kBS == 0, "whole targets per thread");
};

template <int DIM> __host__ __device__ inline long long tiles_of(const GridInfo &g) {
    using TL = Tile<DIM>;
    const long long ntx = (g.nx + TL::TX - 1) / TL::TX, nty = (g.ny + TL::TY - 1) / TL::TY;
    const long long ntz = DIM == 3 ? (g.nz + TL::TZ - 1) / TL::TZ : 1;
    return ntx * nty * ntz;
}

// Fixed point with 2^50 > |x * scale| (the magic constant 1.5 * 2^52 puts
// x * scale, rounded to nearest, in the low bits of a double).
__device__ __forceinline__ long long to_fixed(float x, double scale) {
    const double magic = 6755399441055744.0;
    return __double_as_longlong(fma((double)x, scale, magic)) - __double_as_longlong(magic);
}

// Scale 2^s and its inverse for terms of magnitude at most `bound` (see
// above); a zero bound has only zero terms, a non-finite one gives NaN
// results.
__device__ __forceinline__ void fixed_scale(double bound, double &scale, double &inv) {
    if (!(bound > 0.0)) {
        scale = inv = 1.0;
    } else if (!isfinite(bound)) {
        scale = 1.0;
        inv = __longlong_as_double(0x7ff8000000000000ll);
    } else {
        const int e = ilogb(bound) + 1;  // bound < 2^e
        scale = ldexp(1.0, 50 - e);
        inv = ldexp(1.0, e - 50);
    }
}

struct TileBox {
    int x0, y0, z0, tw, th, td;   // tile origin and extent (clipped to the grid)
    int hx0, hy0, hz0, sx, sy, sz; // staged region (tile + halo, clipped)
};

template <int DIM> __device__ __forceinline__ TileBox tile_box(const GridInfo &g, long long tile, int h) {
    using TL = Tile<DIM>;
    const int ntx = (g.nx + TL::TX - 1) / TL::TX, nty = (g.ny + TL::TY - 1) / TL::TY;
    TileBox b;
    const int t = (int)tile;
    b.x0 = (t % ntx) * TL::TX;
    b.y0 = ((t / ntx) % nty) * TL::TY;
    b.z0 = DIM == 3 ? (t / (ntx * nty)) * TL::TZ : 0;
    b.tw = min(TL::TX, g.nx - b.x0);
    b.th = min(TL::TY, g.ny - b.y0);
    b.td = DIM == 3 ? min(TL::TZ, g.nz - b.z0) : 1;
    b.hx0 = max(0, b.x0 - h);
    b.hy0 = max(0, b.y0 - h);
    b.hz0 = DIM == 3 ? max(0, b.z0 - h) : 0;
    b.sx = min(g.nx, b.x0 + b.tw + h) - b.hx0;
    b.sy = min(g.ny, b.y0 + b.th + h) - b.hy0;
    b.sz = DIM == 3 ? min(g.nz, b.z0 + b.td + h) - b.hz0 : 1;
    return b;
}

// LDS index of grid point (x, y, z) in the staged region.
template <int DIM> __device__ __forceinline__ int sidx(const TileBox &b, int x, int y, int z) {
    using TL = Tile<DIM>;
    return (x - b.hx0) + TL::HX * ((y - b.hy0) + (DIM == 3 ? TL::HY * (z - b.hz0) : 0));
}

template <int DIM> __device__ __forceinline__ bool in_tile(const TileBox &b, int x, int y, int z) {
    return (unsigned)(x - b.x0) < (unsigned)b.tw && (unsigned)(y - b.y0) < (unsigned)b.th &&
           (DIM == 2 || (unsigned)(z - b.z0) < (unsigned)b.td);
}
template <int DIM> __device__ __forceinline__ int tidx(const TileBox &b, int x, int y, int z) {
    using TL = Tile<DIM>;
    return (x - b.x0) + TL::TX * ((y - b.y0) + (DIM == 3 ? TL::TY * (z - b.z0) : 0));
}

// Weights of point z in the arithmetic type.
template <int DIM, typename TS, typename TA>
__device__ __forceinline__ void load_weights(const TS *__restrict__ w, int z, int N, TA *wq) {
    constexpr int S = DIM == 2 ? 3 : 6;
    if (S == 3) {
        const W3<TS> w3 = ((const W3<TS> *)w)[z];
#pragma unroll
        for (int q = 0; q < 3; ++q) wq[q] = Conv<TS, TA>::ld(w3.v[q < 3 ? q : 0]);
    } else {
#pragma unroll
        for (int q = 0; q < S; ++q) wq[q] = Conv<TS, TA>::ld(w[widx32<S>(q, z, N)]);
    }
}

__device__ __forceinline__ int max_abs3(const int *o, int dim) {
    int m = max(abs(o[0]), abs(o[1]));
    return dim == 3 ? max(m, abs(o[2])) : m;
}

// Block-wide min and max (blockDim.x == kBS), in every thread.
__device__ __forceinline__ void block_minmax(float &lo, float &hi, float *red) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, d, 64));
        hi = fmaxf(hi, __shfl_xor(hi, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = lo;
        red[4 + (threadIdx.x >> 6)] = hi;
    }
    __syncthreads();
    lo = fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
    hi = fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7]));
}

// Slots of a point from its packed store (unpacked where used, so that a
// thread can hold several points' packed slots with their loads in flight).
template <int DIM, bool WIDE>
__device__ __forceinline__ Slots<DIM, WIDE> unpack(const typename Slots<DIM, WIDE>::store_t &v) {
    Slots<DIM, WIDE> sl;
    sl.load(&v, 0);
    return sl;
}

// Coordinates of index k in a box of row length sx and plane size sx*sy
// (inv = 1/sx, inv2 = 1/(sx*sy) in FP32): floor((k + 1/2) * inv) is exact for
// k < 2^20, so no integer division is needed.
struct Unravel {
    int sx, sxy;
    float inv, inv2;
    __device__ __forceinline__ void at(int k, int &x, int &y, int &z) const {
        z = (int)(((float)k + 0.5f) * inv2);
        const int r = k - z * sxy;
        y = (int)(((float)r + 0.5f) * inv);
        x = r - y * sx;
    }
};

// One block of the tiled step (MODE 0: out = u - hstep A u; 1: out = A u)
// or of the diagonal pass (MODE 2: diag[z] += near incoming weights, and
// dpart[tile] = the tile's largest diagonal).  Shared by the single-operator
// and batched kernels, so both give bit-identical results.  The staged
// region's points are visited once, four per thread at a time (their slots
// and weights requested together): a point of the tile adds its own part
// (into ownv) and scatters its near edges that land in the tile, a halo
// point scatters its near edges that land in the tile.
template <int DIM, bool WIDE, int MODE, typename TS, typename TD>
__device__ __forceinline__ void tile_block(
    const GridInfo &g, long long tile, const TS *__restrict__ u, TS *__restrict__ out,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const TS *__restrict__ w,
    const int32_t *__restrict__ pos, const int32_t *__restrict__ ent,
    const EntRec<TS> *__restrict__ went, int h, double bound_scale, float hstep,
    TD *__restrict__ diag, double *__restrict__ dpart) {
    using TL = Tile<DIM>;
    typedef typename Slots<DIM, WIDE>::store_t store_t;
    constexpr int S = DIM == 2 ? 3 : 6;
    constexpr bool DIAG = MODE == 2;
    __shared__ float us[DIAG ? 1 : TL::H];
    __shared__ unsigned long long acc[TL::T];
    __shared__ float ownv[DIAG ? 1 : TL::T];
    __shared__ float red[8];
    const int N = (int)g.N;  // N < 2^28
    h = min(max(h, 0), TL::HMAX);  // the staged region must fit the LDS arrays
    const TileBox b = tile_box<DIM>(g, tile, h);
    const int nst = b.sx * b.sy * b.sz;
    const Unravel ur{b.sx, b.sx * b.sy, 1.0f / (float)b.sx, 1.0f / (float)(b.sx * b.sy)};
    // 1. stage u over tile + halo, with its range; clear the accumulators
    float lo = INFINITY, hi = -INFINITY;
    if (!DIAG) {
        constexpr int G = 8;
        for (int k0 = 0; k0 < nst; k0 += G * kBS) {  // block-uniform
            float v[G];
            int li[G];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int k = k0 + j * kBS + (int)threadIdx.x;
                int lx, ly, lz;
                ur.at(k < nst ? k : 0, lx, ly, lz);
                const int zg = (b.hx0 + lx) + g.nx * ((b.hy0 + ly) + g.ny * (b.hz0 + lz));
                v[j] = Conv<TS, float>::ld(u[zg]);
                li[j] = k < nst ? lx + TL::HX * (ly + TL::HY * lz) : -1;
            }
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (li[j] >= 0) {
                    us[li[j]] = v[j];
                    lo = fminf(lo, v[j]);
                    hi = fmaxf(hi, v[j]);
                }
        }
    }
    for (int k = threadIdx.x; k < TL::T; k += kBS) acc[k] = 0ull;
    if (!DIAG) block_minmax(lo, hi, red);  // contains a barrier
    __syncthreads();
    double scale, inv;
    fixed_scale(DIAG ? bound_scale : bound_scale * ((double)hi - (double)lo), scale, inv);
    // 2. every staged point as a source
    constexpr int G = 4;
    for (int k0 = 0; k0 < nst; k0 += G * kBS) {  // block-uniform
        store_t raw[G];
        TS wr[G][S];
        int xs[G], ys[G], zs[G];
        bool val[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int k = k0 + j * kBS + (int)threadIdx.x;
            val[j] = k < nst;
            int lx, ly, lz;
            ur.at(val[j] ? k : 0, lx, ly, lz);
            xs[j] = b.hx0 + lx;
            ys[j] = b.hy0 + ly;
            zs[j] = b.hz0 + lz;
            const int zi = xs[j] + g.nx * (ys[j] + g.ny * zs[j]);
            raw[j] = sb[zi];
            if (S == 3) {
                const W3<TS> w3 = ((const W3<TS> *)w)[zi];
#pragma unroll
                for (int q = 0; q < S; ++q) wr[j][q] = w3.v[q < 3 ? q : 0];
            } else {
#pragma unroll
                for (int q = 0; q < S; ++q) wr[j][q] = w[widx32<S>(q, zi, N)];
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (!val[j]) continue;
            const int x = xs[j], y = ys[j], zz = zs[j];
            const Slots<DIM, WIDE> sl = unpack<DIM, WIDE>(raw[j]);
            float wq[S];
#pragma unroll
            for (int q = 0; q < S; ++q) wq[q] = Conv<TS, float>::ld(wr[j][q]);
            const bool mine = !DIAG && in_tile<DIM>(b, x, y, zz);
            const float uy = DIAG ? 0.f : us[sidx<DIM>(b, x, y, zz)];
            // far neighbours of the own part (a wave-uniform test, then every
            // load from an in-grid address: the point itself where none is
            // needed)
            float uf[2 * S];
            bool anyfar = false;
            if (mine) {
#pragma unroll
                for (int q = 0; q < S; ++q) anyfar |= wq[q] > 0.f && max_abs3(sl.o[q], DIM) > h;
            }
            if (__any(anyfar)) {
                const int zi = x + g.nx * (y + g.ny * zz);
#pragma unroll
                for (int q = 0; q < S; ++q)
#pragma unroll
                    for (int sg = 0; sg < 2; ++sg) {
                        const int s1 = sg ? 1 : -1;
                        const int tx = x + s1 * sl.o[q][0], ty = y + s1 * sl.o[q][1];
                        const int tz = DIM == 3 ? zz + s1 * sl.o[q][2] : 0;
                        const bool ing = (unsigned)tx < (unsigned)g.nx && (unsigned)ty < (unsigned)g.ny &&
                                         (DIM == 2 || (unsigned)tz < (unsigned)g.nz);
                        const bool far = max_abs3(sl.o[q], DIM) > h;
                        const int ti = mine && ing && far && wq[q] > 0.f ? tx + g.nx * (ty + g.ny * tz) : zi;
                        uf[2 * q + sg] = Conv<TS, float>::ld(u[ti]);
                    }
            } else {
#pragma unroll
                for (int q = 0; q < 2 * S; ++q) uf[q] = 0.f;
            }
            float a = 0.f;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                if (!(wq[q] > 0.f)) continue;
                const bool near = max_abs3(sl.o[q], DIM) <= h;
                if (!mine && !near) continue;
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const int s1 = sg ? 1 : -1;
                    const int tx = x + s1 * sl.o[q][0], ty = y + s1 * sl.o[q][1];
                    const int tz = DIM == 3 ? zz + s1 * sl.o[q][2] : 0;
                    const bool lands = near && in_tile<DIM>(b, tx, ty, tz);
                    if (!mine) {
                        if (lands) {
                            const float v = DIAG ? wq[q] : wq[q] * (us[sidx<DIM>(b, tx, ty, tz)] - uy);
                            atomicAdd(&acc[tidx<DIM>(b, tx, ty, tz)],
                                      (unsigned long long)to_fixed(v, scale));
                        }
                        continue;
                    }
                    if (!((unsigned)tx < (unsigned)g.nx && (unsigned)ty < (unsigned)g.ny &&
                          (DIM == 2 || (unsigned)tz < (unsigned)g.nz)))
                        continue;  // Neumann truncation
                    const float ut = near ? us[sidx<DIM>(b, tx, ty, tz)] : uf[2 * q + sg];
                    const float term = wq[q] * (uy - ut);
                    a += term;
                    if (lands)
                        atomicAdd(&acc[tidx<DIM>(b, tx, ty, tz)],
                                  (unsigned long long)to_fixed(-term, scale));
                }
            }
            if (mine) ownv[tidx<DIM>(b, x, y, zz)] = a;
        }
    }
    __syncthreads();
    // 3. far incoming from the lists (row starts of all of the thread's
    // targets requested first), then the result
    double dmax = 0.0;
    int p0[TL::PT], p1[TL::PT];
#pragma unroll
    for (int j = 0; j < TL::PT; ++j) {
        const int k = (int)threadIdx.x + j * kBS;
        const int lx = k % TL::TX, ly = (k / TL::TX) % TL::TY, lz = k / (TL::TX * TL::TY);
        const bool live = !DIAG && lx < b.tw && ly < b.th && lz < b.td;
        const int zi = live ? (b.x0 + lx) + g.nx * ((b.y0 + ly) + g.ny * (b.z0 + lz)) : 0;
        p0[j] = live ? pos[zi] : 0;
        p1[j] = live ? pos[zi + 1] : 0;
    }
    for (int j = 0; j < TL::PT; ++j) {
        const int k = (int)threadIdx.x + j * kBS;
        const int lx = k % TL::TX, ly = (k / TL::TX) % TL::TY, lz = k / (TL::TX * TL::TY);
        if (lx >= b.tw || ly >= b.th || lz >= b.td) continue;
        const int x = b.x0 + lx, y = b.y0 + ly, zz = b.z0 + lz;
        const int zi = x + g.nx * (y + g.ny * zz);
        const double nearv = (double)(long long)acc[k] * inv;
        if (DIAG) {
            const double d = (double)diag[zi] + nearv;
            diag[zi] = (TD)d;
            dmax = fmax(dmax, d);
            continue;
        }
        const float uz = us[sidx<DIM>(b, x, y, zz)];
        float far = 0.f;
        for (int p = p0[j]; p < p1[j]; ++p) {
            int32_t v;
            TS wv;
            if (kInlineW<DIM>) {
                load_rec<TS>(went, ent, p, true, v, wv);
            } else {
                v = ent[p];
                wv = w[widx32<S>((v >> 6) & 7, zi + (v >> 9), N)];
            }
            far += Conv<TS, float>::ld(wv) * (uz - Conv<TS, float>::ld(u[zi + (v >> 9)]));
        }
        const float a = (ownv[k] + (float)nearv) + far;
        out[zi] = Conv<TS, float>::st(MODE == 0 ? uz - hstep * a : a);
    }
    if (DIAG) block_partial_max(dmax, dpart);
}

template <int DIM, bool WIDE, int MODE, typename TS>
__global__ __launch_bounds__(kBS) void k_apply_tiled(
    GridInfo g, const TS *__restrict__ u, TS *__restrict__ out,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const TS *__restrict__ w,
    const int32_t *__restrict__ pos, const int32_t *__restrict__ ent,
    const EntRec<TS> *__restrict__ went, const int32_t *__restrict__ hnear,
    const double *__restrict__ maxdiag, double dt, const double *__restrict__ dtcfl, int dt_mode) {
    const float hstep = (float)(dt_mode == ADLBR_DT_CFL ? dt * dtcfl[0] : dt);
    tile_block<DIM, WIDE, MODE, TS, float>(g, xcd_block(blockIdx.x, gridDim.x), u, out, sb, w,
                                           pos, ent, went, *hnear, *maxdiag, hstep, nullptr,
                                           nullptr);
}

// The diagonal's near incoming part (tiled layout): diag[z] += the weights
// of the near edges landing on z; dpart[tile] = the tile's largest A_zz.
template <int DIM, bool WIDE, typename TS, typename TD>
__global__ __launch_bounds__(kBS) void k_tile_diag(
    GridInfo g, const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const TS *__restrict__ w,
    const int32_t *__restrict__ hnear, const double *__restrict__ wmax, TD *__restrict__ diag,
    double *__restrict__ dpart) {
    tile_block<DIM, WIDE, 2, TS, TD>(g, blockIdx.x, (const TS *)nullptr, (TS *)nullptr, sb, w,
                                     nullptr, nullptr, nullptr, *hnear, *wmax, 0.f, diag, dpart);
}

// Batched tiled step: blocks laid out problem after problem, one tile each.
template <int DIM, bool WIDE, typename TS, bool XCD>
__global__ __launch_bounds__(kBS) void k_apply_tiled_batch(const BatchProb *__restrict__ probs,
                                                           int nprob, int parity) {
    const long long bb = XCD ? xcd_block(blockIdx.x, gridDim.x) : (long long)blockIdx.x;
    const BatchProb &P = probs[find_prob(probs, nprob, bb)];
    const GridInfo g = P.g;
    const float hstep = (float)(P.dt_mode == ADLBR_DT_CFL ? P.dt * P.dtcfl[0] : P.dt);
    tile_block<DIM, WIDE, 0, TS, float>(
        g, bb - P.first_block, (const TS *)P.u[parity], (TS *)P.u[parity ^ 1],
        (const typename Slots<DIM, WIDE>::store_t *)P.sb, (const TS *)P.w, P.pos, P.ent,
        (const EntRec<TS> *)P.went, *P.hnear, *P.maxdiag, hstep, (float *)nullptr, nullptr);
}

// Reach (largest offset component over the edges of positive weight) and
// largest weight of each block of points, for the tiled layout's halo and
// fixed-point scales; k_tile_params reduces them.
template <int DIM, bool WIDE, typename TS>
__global__ __launch_bounds__(256) void k_reach_wmax(GridInfo g,
                                                    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb,
                                                    const TS *__restrict__ w, double *__restrict__ rpart,
                                                    double *__restrict__ wpart) {
    constexpr int S = DIM == 2 ? 3 : 6;
    const long long z = (long long)blockIdx.x * 256 + threadIdx.x;
    double r = 0.0, wm = 0.0;
    if (z < g.N) {
        Slots<DIM, WIDE> sl;
        sl.load(sb, z);
        float wq[S];
        load_weights<DIM, TS, float>(w, (int)z, (int)g.N, wq);
        for (int q = 0; q < S; ++q)
            if (wq[q] > 0.f) {
                r = fmax(r, (double)max_abs3(sl.o[q], DIM));
                wm = fmax(wm, (double)wq[q]);
            }
    }
    block_partial_max(r, rpart);
    block_partial_max(wm, wpart);
}

// hnear = min(hmax, reach) (0 for the list layout: every edge is listed)
// and the largest weight.
__global__ __launch_bounds__(256) void k_tile_params(const double *rpart, const double *wpart,
                                                     long long nb, int hmax, int32_t *hnear,
                                                     double *wmax) {
    const double r = reduce_partials(rpart, nb, true);
    const double wm = reduce_partials(wpart, nb, true);
    if (threadIdx.x != 0) return;
    *hnear = hmax > 0 ? (int32_t)fmin((double)hmax, r) : 0;
    *wmax = wm;
}

// Conjugate-gradient direction with K = I + dt A (dt from the state):
//   q = K z + beta q,  p = z + beta p  (beta = 0 on the first iteration),
// so that q = K p without a second gather.  Each block writes its partial
// <p, q> in FP64 (partial[blk]); k_cg_alpha sums them in block order and
// sets alpha = <z, r> / <p, q>.
template <int DIM, bool WIDE, bool PER, typename T>
__global__ __launch_bounds__(kBS) void k_cg_direction(
    GridInfo g, const T *__restrict__ zv, T *__restrict__ q, T *__restrict__ p,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const T *__restrict__ w,
    const uint8_t *__restrict__ cnt, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ ent, const EntRec<T> *__restrict__ went, const CgState *st,
    double *partial, int first) {
    const long long N = g.N;
    // the apply's block order (XCD bands; 3D strips of planes)
    const long long blk = strip_block(xcd_block(blockIdx.x, gridDim.x), g, kApplyPoints);
    const long long z = wave_group(g, blk, 1) + (threadIdx.x & 63);
    const bool live = z < N;
    double pqz = 0.0;
    const bool skip = st->bad || st->done;
    const WaveLists L = wave_lists(pos, z, N);
    const T zz = live ? zv[z] : (T)0;
    OwnPart<DIM, WIDE, PER, T, T, T> own;
    own.issue(g, z, live && !skip, zz, zv, sb, w);
    T acc = skip ? (T)0 : wave_incoming<kInlineW<DIM>, DIM == 2 ? 3 : 6, T, T, T>(L, z, N, zz, zv, w, ent, went);
    if (live && !skip) {
        acc += own.sum(zz);
        const T dt = (T)st->dt;
        const T beta = first ? (T)0 : (T)st->beta;
        const T qn = zz + dt * acc + (first ? (T)0 : beta * q[z]);
        const T pn = zz + (first ? (T)0 : beta * p[z]);
        q[z] = qn;
        p[z] = pn;
        pqz = (double)pn * (double)qn;
    }
    __shared__ double red[kBS];
    red[threadIdx.x] = pqz;
    __syncthreads();
    for (int s = kBS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blk] = red[0];
}

// alpha = <z, r> / <p, q> from the partials (one block of kBS threads).
__global__ __launch_bounds__(kBS) void k_cg_alpha(CgState *st, const double *partial, long long nb) {
    const double pq = reduce_partials(partial, nb);
    if (threadIdx.x != 0 || st->bad || st->done) return;
    st->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) st->bad = 1;
    st->alpha = st->bad ? 0.0 : st->rz / pq;
}

// |b - (x + dt A x)|^2 with FP64 arithmetic (weights promoted); block
// partials, finished by k_sum_partials.
template <int DIM, bool WIDE, bool PER, typename T>
__global__ __launch_bounds__(kBS) void k_residual(
    GridInfo g, const T *__restrict__ b, const double *__restrict__ x,
    const typename Slots<DIM, WIDE>::store_t *__restrict__ sb, const T *__restrict__ w,
    const uint8_t *__restrict__ cnt, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ ent, const EntRec<T> *__restrict__ went, double dt, double *partial,
    T *__restrict__ rout) {
    const long long N = g.N;
    // the apply's block order (XCD bands; 3D strips of planes); the partial
    // stays at blockIdx.x
    const long long blk = strip_block(xcd_block(blockIdx.x, gridDim.x), g, kApplyPoints);
    const long long z = wave_group(g, blk, 1) + (threadIdx.x & 63);
    const bool live = z < N;
    double r2 = 0.0;
    const WaveLists L = wave_lists(pos, z, N);
    const double xz = live ? x[z] : 0.0;
    OwnPart<DIM, WIDE, PER, T, double, double> own;
    own.issue(g, z, live, xz, x, sb, w);
    double ax = wave_incoming<kInlineW<DIM>, DIM == 2 ? 3 : 6, T, double, double>(L, z, N, xz, x, w, ent, went);
    if (live) {
        ax += own.sum(xz);
        const double r = (double)b[z] - (xz + dt * ax);
        r2 = r * r;
        if (rout) rout[z] = (T)r;
    }
    block_partial_sum(r2, partial);
}

__global__ __launch_bounds__(kBS) void k_sum_partials(const double *partial, long long nb,
                                                      double *out) {
    const double t = reduce_partials(partial, nb);
    if (threadIdx.x == 0) *out = t;
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
    if (win_f64)
        hipLaunchKernelGGL((k_compact<DIM, WIDE, PER, double, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           off, (const double *)win, sb, w, op->mask, status);
    else
        hipLaunchKernelGGL((k_compact<DIM, WIDE, PER, float, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           off, (const float *)win, sb, w, op->mask, status);
    // the halo of the near edges (tiled layout) or 0 (every edge listed)
    constexpr bool kTiledOk = !PER && sizeof(TS) <= 4;
    bool tiled_params = false;
    if constexpr (kTiledOk) {
        if (op->tiled) {
            hipLaunchKernelGGL((k_reach_wmax<DIM, WIDE, TS>), dim3(nb), dim3(256), 0, s, g,
                               (const store_t *)sb, (const TS *)w, op->rpart, op->part);
            hipLaunchKernelGGL(k_tile_params, dim3(1), dim3(256), 0, s, (const double *)op->rpart,
                               (const double *)op->part, (long long)nb, Tile<DIM>::HMAX,
                               op->hnear, op->wmax);
            tiled_params = true;
        }
    }
    if (!tiled_params) hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, op->hnear, 1ll, 0);
    long long nparts;
    if (DIM == 2) {
        const int ntx = (g.nx + kTile - 1) / kTile, nty = (g.ny + kTile - 1) / kTile;
        const unsigned ntiles = (unsigned)(ntx * nty);
        const unsigned nchunk = (unsigned)nbins;  // 1024-point chunks
        hipLaunchKernelGGL((k_tile_rmax<WIDE>), dim3(ntiles), dim3(256), 0, s, g,
                           (const typename Slots<2, WIDE>::store_t *)op->sb,
                           (const uint8_t *)op->mask, op->trmax, op->brmax);
        hipLaunchKernelGGL(k_rmax_tiles, dim3(1), dim3(256), 0, s, (const int32_t *)op->trmax,
                           (long long)ntiles, op->rmax);
        hipLaunchKernelGGL((k_tile_count<WIDE, PER>), dim3(ntiles), dim3(256), 0, s, g,
                           (const typename Slots<2, WIDE>::store_t *)op->sb, (const uint8_t *)op->mask,
                           (const int32_t *)op->rmax, (const int32_t *)op->trmax,
                           (const int32_t *)op->brmax, (const int32_t *)op->hnear, op->cnt, op->rank,
                           status);
        hipLaunchKernelGGL(k_chunk_sum, dim3(nchunk), dim3(256), 0, s, (const uint8_t *)op->cnt, N,
                           (int32_t *)op->bincnt);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, (int32_t *)op->bincnt, nbins);
        hipLaunchKernelGGL(k_chunk_pos, dim3(nchunk), dim3(256), 0, s, (const uint8_t *)op->cnt, N,
                           (const int32_t *)op->bincnt, op->pos);
        hipLaunchKernelGGL((k_place2d<WIDE, PER>), dim3(nb), dim3(256), 0, s, g,
                           (const typename Slots<2, WIDE>::store_t *)op->sb,
                           (const uint8_t *)op->mask, (const uint8_t *)op->rank,
                           (const int32_t *)op->pos, (const int32_t *)op->hnear, op->ent);
        if (op->storage == ADLBR_F64)
            hipLaunchKernelGGL((k_rows<DIM, WIDE, PER, TS, TA, double>), dim3(nb), dim3(256), 0, s,
                               g, (const store_t *)op->sb, (const TS *)w, (const uint8_t *)op->cnt,
                               (const int32_t *)op->pos, op->ent, (EntRec<TS> *)op->went, (double *)op->diag,
                               op->part);
        else
            hipLaunchKernelGGL((k_rows<DIM, WIDE, PER, TS, TA, float>), dim3(nb), dim3(256), 0, s,
                               g, (const store_t *)op->sb, (const TS *)w, (const uint8_t *)op->cnt,
                               (const int32_t *)op->pos, op->ent, (EntRec<TS> *)op->went, (float *)op->diag,
                               op->part);
        nparts = nb;
    } else {
        hipLaunchKernelGGL(k_fill_i32, dim3(nbb), dim3(kBS), 0, s, (int32_t *)op->bincnt, nbins, 0);
        hipLaunchKernelGGL(k_fill_i32, dim3(nbb), dim3(kBS), 0, s, (int32_t *)op->bincur, nbins, 0);
        hipLaunchKernelGGL((k_bin_count<DIM, WIDE, PER>), dim3(nb), dim3(kBS), 0, s, g,
                           (const store_t *)sb, (const uint8_t *)op->mask, (const int32_t *)op->hnear,
                           op->bincnt);
        hipLaunchKernelGGL(k_copy_u32, dim3(nbb), dim3(kBS), 0, s, op->bincnt, op->binoff, nbins);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, (int32_t *)op->binoff, nbins);
        hipLaunchKernelGGL((k_bin_fill<DIM, WIDE, PER>), dim3(nb), dim3(kBS), 0, s, g,
                           (const store_t *)sb, (const uint8_t *)op->mask, (const int32_t *)op->hnear,
                           op->binoff, op->bincur, op->binbuf);
        if (op->storage == ADLBR_F64)
            hipLaunchKernelGGL((k_bin_build<DIM, WIDE, PER, TS, TA, double>), dim3((unsigned)nbins),
                               dim3(256), 0, s, g, op->bincnt, op->binoff, op->binbuf, sb, w,
                               op->pos, op->cnt, op->ent, (EntRec<TS> *)op->went, (double *)op->diag, op->part,
                               status);
        else
            hipLaunchKernelGGL((k_bin_build<DIM, WIDE, PER, TS, TA, float>), dim3((unsigned)nbins),
                               dim3(256), 0, s, g, op->bincnt, op->binoff, op->binbuf, sb, w,
                               op->pos, op->cnt, op->ent, (EntRec<TS> *)op->went, (float *)op->diag, op->part,
                               status);
        nparts = nbins;
    }
    if constexpr (kTiledOk) {
        if (op->tiled) {
            // the rows above hold the own part and the far incoming edges;
            // add the near incoming ones and take the largest A_zz per tile
            const long long nt = tiles_of<DIM>(g);
            hipLaunchKernelGGL((k_tile_diag<DIM, WIDE, TS, float>), dim3((unsigned)nt), dim3(kBS),
                               0, s, g, (const store_t *)sb, (const TS *)w,
                               (const int32_t *)op->hnear, (const double *)op->wmax,
                               (float *)op->diag, op->part);
            nparts = nt;
        }
    }
    hipLaunchKernelGGL(k_cfl, dim3(1), dim3(256), 0, s, (const double *)op->part, nparts,
                       op->maxdiag, op->dtcfl);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}

template <int DIM, bool WIDE, bool PER, typename TS, typename TA>
int apply_impl(const adlbr_operator *op, const void *u, void *out, bool step, double dt, int dt_mode,
               hipStream_t s) {
    typedef typename Slots<DIM, WIDE>::store_t store_t;
    const GridInfo g = op->gi;
    if constexpr (!PER && sizeof(TS) <= 4) {
        if (op->tiled) {
            const unsigned nt = (unsigned)tiles_of<DIM>(g);
            if (step)
                hipLaunchKernelGGL((k_apply_tiled<DIM, WIDE, 0, TS>), dim3(nt), dim3(kBS), 0, s, g,
                                   (const TS *)u, (TS *)out, (const store_t *)op->sb,
                                   (const TS *)op->w, op->pos, op->ent,
                                   (const EntRec<TS> *)op->went, (const int32_t *)op->hnear,
                                   (const double *)op->maxdiag, dt, op->dtcfl, dt_mode);
            else
                hipLaunchKernelGGL((k_apply_tiled<DIM, WIDE, 1, TS>), dim3(nt), dim3(kBS), 0, s, g,
                                   (const TS *)u, (TS *)out, (const store_t *)op->sb,
                                   (const TS *)op->w, op->pos, op->ent,
                                   (const EntRec<TS> *)op->went, (const int32_t *)op->hnear,
                                   (const double *)op->maxdiag, dt, op->dtcfl, dt_mode);
            return ADLBR_OK;
        }
    }
    const unsigned nb = (unsigned)((g.N + kApplyPoints - 1) / kApplyPoints);
    if (step)
        hipLaunchKernelGGL((k_apply<DIM, WIDE, PER, true, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           (const TS *)u, (TS *)out, (const store_t *)op->sb, (const TS *)op->w,
                           op->cnt, op->pos, op->ent, (const EntRec<TS> *)op->went, dt, op->dtcfl, dt_mode);
    else
        hipLaunchKernelGGL((k_apply<DIM, WIDE, PER, false, TS, TA>), dim3(nb), dim3(kBS), 0, s, g,
                           (const TS *)u, (TS *)out, (const store_t *)op->sb, (const TS *)op->w,
                           op->cnt, op->pos, op->ent, (const EntRec<TS> *)op->went, dt, op->dtcfl, dt_mode);
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

template <int DIM, bool WIDE, bool PER, typename TS, typename TA> struct BatchF {
    static int run(const adlbr_operator *rep, const BatchProb *probs, const BatchProb *hprobs,
                   int nprob, long long nblocks, int parity, int variant, int copy,
                   hipStream_t s) {
        typedef typename Slots<DIM, WIDE>::store_t store_t;
        if constexpr (!PER && sizeof(TS) <= 4) {
            if (rep->tiled && !copy) {
                if (variant & 4) {  // one launch per problem (same kernel as adlbr_step)
                    for (int i = 0; i < nprob; ++i) {
                        const BatchProb &P = hprobs[i];
                        hipLaunchKernelGGL((k_apply_tiled<DIM, WIDE, 0, TS>), dim3((unsigned)P.nblocks),
                                           dim3(kBS), 0, s, P.g, (const TS *)P.u[parity],
                                           (TS *)P.u[parity ^ 1], (const store_t *)P.sb,
                                           (const TS *)P.w, P.pos, P.ent, (const EntRec<TS> *)P.went,
                                           P.hnear, P.maxdiag, P.dt, P.dtcfl, P.dt_mode);
                    }
                } else if (variant & 1) {
                    hipLaunchKernelGGL((k_apply_tiled_batch<DIM, WIDE, TS, true>),
                                       dim3((unsigned)nblocks), dim3(kBS), 0, s, probs, nprob, parity);
                } else {
                    hipLaunchKernelGGL((k_apply_tiled_batch<DIM, WIDE, TS, false>),
                                       dim3((unsigned)nblocks), dim3(kBS), 0, s, probs, nprob, parity);
                }
                return ADLBR_OK;
            }
        }
        if (variant & 4) {  // one launch per problem (same kernel as adlbr_step)
            for (int i = 0; i < nprob; ++i) {
                const BatchProb &P = hprobs[i];
                if (copy) {
                    ADLBR_CHECK_HIP(hipMemcpyAsync(P.u[0], P.u[1], (size_t)P.g.N * sizeof(TS),
                                                   hipMemcpyDeviceToDevice, s));
                    continue;
                }
                const unsigned nb = (unsigned)((P.g.N + kApplyPoints - 1) / kApplyPoints);
                hipLaunchKernelGGL((k_apply<DIM, WIDE, PER, true, TS, TA>), dim3(nb), dim3(kBS), 0, s,
                                   P.g, (const TS *)P.u[parity], (TS *)P.u[parity ^ 1],
                                   (const store_t *)P.sb, (const TS *)P.w, P.cnt, P.pos, P.ent, (const EntRec<TS> *)P.went, P.dt,
                                   P.dtcfl, P.dt_mode);
            }
            return ADLBR_OK;
        }
        if (copy) {
            hipLaunchKernelGGL((k_copy_batch<TS>), dim3((unsigned)nblocks), dim3(kBS), 0, s, probs,
                               nprob);
        } else if (DIM == 2 && rep->went) {  // 2D records (the class has them all)
            if (variant & 1)
                hipLaunchKernelGGL((k_apply_batch<DIM, WIDE, PER, TS, TA, true, true>),
                                   dim3((unsigned)nblocks), dim3(kBS), 0, s, probs, nprob, parity);
            else
                hipLaunchKernelGGL((k_apply_batch<DIM, WIDE, PER, TS, TA, false, true>),
                                   dim3((unsigned)nblocks), dim3(kBS), 0, s, probs, nprob, parity);
        } else if (variant & 1) {
            hipLaunchKernelGGL((k_apply_batch<DIM, WIDE, PER, TS, TA, true>), dim3((unsigned)nblocks),
                               dim3(kBS), 0, s, probs, nprob, parity);
        } else {
            hipLaunchKernelGGL((k_apply_batch<DIM, WIDE, PER, TS, TA, false>),
                               dim3((unsigned)nblocks), dim3(kBS), 0, s, probs, nprob, parity);
        }
        return ADLBR_OK;
    }
};

template <int DIM, bool WIDE, bool PER, typename TS, typename TA> struct MultiF {
    static int run(const adlbr_operator *op, const void *u, void *out, int ncomp, double dt,
                   int mode, hipStream_t s) {
        typedef typename Slots<DIM, WIDE>::store_t store_t;
        const unsigned nb = (unsigned)((op->gi.N + kApplyPoints - 1) / kApplyPoints);
        hipLaunchKernelGGL((k_step_multi<DIM, WIDE, PER, TS, TA>), dim3(nb), dim3(kBS), 0, s,
                           op->gi, ncomp, (const TS *)u, (TS *)out, (const store_t *)op->sb,
                           (const TS *)op->w, op->pos, op->ent, (const EntRec<TS> *)op->went, dt,
                           op->dtcfl, mode);
        return ADLBR_OK;
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
                           (const TS *)op->w, op->cnt, op->pos, op->ent, (const EntRec<TS> *)op->went,
                           (const CgState *)st,
                           partial, first);
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kBS), 0, s, st, (const double *)partial,
                           (long long)nb);
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
                   double *out, double *partial, void *rout, hipStream_t s) {
        typedef typename Slots<DIM, WIDE>::store_t store_t;
        const GridInfo g = op->gi;
        const unsigned nb = (unsigned)((g.N + kBS - 1) / kBS);
        hipLaunchKernelGGL((k_residual<DIM, WIDE, PER, TS>), dim3(nb), dim3(kBS), 0, s, g,
                           (const TS *)b, x, (const store_t *)op->sb, (const TS *)op->w, op->cnt,
                           op->pos, op->ent, (const EntRec<TS> *)op->went, dt, partial, (TS *)rout);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBS), 0, s, (const double *)partial,
                           (long long)nb, out);
        return ADLBR_OK;
    }
};
template <int DIM, bool WIDE, bool PER> struct ResidualF<DIM, WIDE, PER, bf16, float> {
    static int run(const adlbr_operator *, double, const void *, const double *, double *,
                   double *, void *, hipStream_t) {
        return ADLBR_E_UNSUPPORTED;
    }
};
template <int DIM, bool WIDE, bool PER> struct ResidualF<DIM, WIDE, PER, _Float16, float> {
    static int run(const adlbr_operator *, double, const void *, const double *, double *,
                   double *, void *, hipStream_t) {
        return ADLBR_E_UNSUPPORTED;
    }
};

struct Layout {
    size_t sb, w, cnt, pos, ent, went, diag, scal, mask, part, rpart, trmax, brmax, rank, bincnt,
        bincur, binoff, binbuf, total;
};

// records: 2D operators keep each incoming entry with its weight as well
// (ADLBR_OP_RECORDS); 3D operators always do.
bool has_records(const GridInfo &g, int records) { return g.dim == 3 ? ADLBR_W3D_INLINE : records != 0; }

Layout layout(const GridInfo &g, int storage, int wide, int records) {
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
    L.went = o; o += has_records(g, records) ? align_up((dtype_size(storage) == 4 ? 8 : dtype_size(storage)) * (size_t)(2 * S) * N) : 0;
    L.diag = o; o += align_up((storage == ADLBR_F64 ? 8 : 4) * (size_t)N);
    L.scal = o; o += 256;
    L.mask = o; o += align_up((size_t)N + 64);
    // partials: one per 256-point block, per 3D bin or per tile of the
    // tiled layout
    const size_t ntiles = g.dim == 2 ? (size_t)((g.nx + kTile - 1) / kTile) * ((g.ny + kTile - 1) / kTile) : 0;
    const size_t nlt = (size_t)(g.dim == 2 ? tiles_of<2>(g) : tiles_of<3>(g));
    L.part = o; o += align_up(8 * (std::max(std::max((size_t)N / 256, nbins), nlt) + 64));
    L.rpart = o; o += align_up(8 * ((size_t)N / 256 + 64));
    L.trmax = o; o += ntiles ? align_up(4 * ntiles) : 0;
    const size_t nbricks = g.dim == 2 ? (size_t)((g.nx + kBrick - 1) / kBrick) * ((g.ny + kBrick - 1) / kBrick) : 0;
    L.brmax = o; o += nbricks ? align_up(4 * nbricks) : 0;
    L.rank = o; o += g.dim == 2 ? align_up(6 * (size_t)N) : 0;
    L.bincnt = o; o += align_up(4 * nbins + 4);
    const bool bins = g.dim == 3;  // the 2D tile assembly needs no bins
    L.bincur = o; o += bins ? align_up(4 * nbins + 4) : 0;
    L.binoff = o; o += bins ? align_up(4 * nbins + 4) : 0;
    L.binbuf = o; o += bins ? align_up(8 * (size_t)(2 * S) * N) : 0;
    L.total = o;
    return L;
}

}  // namespace

int batch_class(const adlbr_operator *op) {
    const int rec2d = op->gi.dim == 2 && op->went ? 1 : 0;  // 2D records: their own class
    return rec2d * 100000 + op->tiled * 10000 + op->gi.dim * 1000 + op->wide * 100 +
           op->gi.periodic * 10 + op->storage;
}

long long batch_blocks(const adlbr_operator *op, int *block_points) {
    if (op->tiled) {
        *block_points = op->gi.dim == 2 ? Tile<2>::T : Tile<3>::T;
        return op->gi.dim == 2 ? tiles_of<2>(op->gi) : tiles_of<3>(op->gi);
    }
    *block_points = kApplyPoints;
    return (op->gi.N + kApplyPoints - 1) / kApplyPoints;
}

void batch_describe(const adlbr_operator *op, BatchProb *d) {
    d->g = op->gi;
    d->sb = op->sb;
    d->w = op->w;
    d->cnt = op->cnt;
    d->pos = op->pos;
    d->ent = op->ent;
    d->went = op->went;
    d->dtcfl = op->dtcfl;
    d->hnear = op->hnear;
    d->maxdiag = op->maxdiag;
    int bp = 0;
    d->nblocks = batch_blocks(op, &bp);
    d->block_points = bp;
}

size_t batch_footprint(const adlbr_operator *op) {
    const size_t ts = dtype_size(op->storage);
    size_t sbs;
    if (op->gi.dim == 2) sbs = op->wide ? sizeof(Slots<2, true>::store_t) : sizeof(Slots<2, false>::store_t);
    else sbs = op->wide ? sizeof(Slots<3, true>::store_t) : sizeof(Slots<3, false>::store_t);
    // u and its successor, offsets, own weights, count, row start, and about
    // two incoming entries (each with its weight) per slot
    return (size_t)op->gi.N *
           (2 * ts + sbs + (size_t)op->slots * ts +
            2 * (size_t)op->slots * (op->went ? (ts <= 4 ? 8 : 4 + ts) : 4) +
            1 + 4);
}

int batch_launch(const adlbr_operator *rep, const BatchProb *probs, const BatchProb *hprobs,
                 int nprob, long long nblocks, int parity, int variant, int copy, hipStream_t s) {
    return dispatch<BatchF>(rep, probs, hprobs, nprob, nblocks, parity, variant, copy, s);
}

int cg_direction(const adlbr_operator *op, const void *z, void *q, void *p, CgState *st,
                 double *partial, int first, hipStream_t s) {
    if (op->tiled) return ADLBR_E_UNSUPPORTED;  // the solvers gather over full lists
    return dispatch<CgDirF>(op, z, q, p, st, partial, first, s);
}

// out = (I + dt A) u, written as one explicit step with step -dt.
int apply_K(const adlbr_operator *op, const void *u, void *out, double dt, hipStream_t s) {
    return dispatch<ApplyF>(op, u, out, true, -dt, (int)ADLBR_DT_ABS, s);
}

int true_residual(const adlbr_operator *op, double dt, const void *b, const double *x,
                  double *out, double *partial, void *rout, hipStream_t s) {
    if (op->tiled) return ADLBR_E_UNSUPPORTED;
    return dispatch<ResidualF>(op, dt, b, x, out, partial, rout, s);
}

const GridInfo &operator_grid(const adlbr_operator *op) { return op->gi; }
int operator_storage(const adlbr_operator *op) { return op->storage; }
const void *operator_diag(const adlbr_operator *op) { return op->diag; }
const void *operator_weights(const adlbr_operator *op) { return op->w; }
const void *operator_slots(const adlbr_operator *op) { return op->sb; }
int operator_wide(const adlbr_operator *op) { return op->wide; }
int operator_tiled(const adlbr_operator *op) { return op->tiled; }

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
    *bytes = layout(gi, storage, flags & ADLBR_OP_WIDE, flags & ADLBR_OP_RECORDS).total;
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
    if (flags & ~(ADLBR_OP_WIDE | ADLBR_OP_TILED | ADLBR_OP_RECORDS)) {
        set_error("adlbr_operator_create: unknown flags 0x%x", flags);
        return ADLBR_E_INVALID;
    }
    const int wide = flags & ADLBR_OP_WIDE ? 1 : 0;
    const int tiled = flags & ADLBR_OP_TILED ? 1 : 0;
    const int records = flags & ADLBR_OP_RECORDS ? 1 : 0;
    if (tiled && records) {
        set_error("adlbr_operator_create: ADLBR_OP_RECORDS needs the list layout");
        return ADLBR_E_UNSUPPORTED;
    }
    if (tiled && (gi.periodic || storage == ADLBR_F64)) {
        set_error("adlbr_operator_create: the tiled layout needs a Neumann grid and F32, BF16 or "
                  "F16 storage");
        return ADLBR_E_UNSUPPORTED;
    }
    if ((long long)(gi.dim == 2 ? 6 : 12) * gi.N >= (1ll << 31)) {
        set_error("adlbr_operator_create: too many edges for 32-bit list positions");
        return ADLBR_E_RANGE;
    }
    const Layout L = layout(gi, storage, wide, records);
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
    op->tiled = tiled;
    op->sb = b + L.sb;
    op->w = b + L.w;
    op->cnt = (uint8_t *)(b + L.cnt);
    op->pos = (int32_t *)(b + L.pos);
    op->ent = (int32_t *)(b + L.ent);
    op->went = has_records(gi, records) ? b + L.went : nullptr;
    op->diag = b + L.diag;
    op->maxdiag = (double *)(b + L.scal);
    op->dtcfl = (double *)(b + L.scal + 8);
    op->rmax = (int32_t *)(b + L.scal + 16);
    op->hnear = (int32_t *)(b + L.scal + 20);
    op->wmax = (double *)(b + L.scal + 24);
    op->rpart = (double *)(b + L.rpart);
    op->mask = (uint8_t *)(b + L.mask);
    op->part = (double *)(b + L.part);
    op->trmax = (int32_t *)(b + L.trmax);
    op->brmax = (int32_t *)(b + L.brmax);
    op->rank = (uint8_t *)(b + L.rank);
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

extern "C" int adlbr_operator_rebuild(adlbr_operator *op, const int16_t *offsets,
                                      const void *weights, int w_dtype, int32_t *status,
                                      void *stream) {
    clear_error();
    if (!op || !offsets || !weights || !status) {
        set_error("adlbr_operator_rebuild: null pointer argument");
        return ADLBR_E_INVALID;
    }
    if (w_dtype != ADLBR_F64 && w_dtype != ADLBR_F32) {
        set_error("adlbr_operator_rebuild: weights must be F64/F32");
        return ADLBR_E_INVALID;
    }
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, s, status);
    const int rc = dispatch<BuildF>(op, offsets, weights, (int)(w_dtype == ADLBR_F64), status, s);
    hipLaunchKernelGGL(k_status_final, dim3(1), dim3(1), 0, s, status);
    if (rc) return rc;
    ADLBR_LAUNCH_CHECK();
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

extern "C" int adlbr_step_multi(adlbr_operator *op, void *u, void *u_tmp, int ncomp, double dt,
                                int dt_mode, int64_t nsteps, void *stream) {
    clear_error();
    if (!op || !u || !u_tmp || u == u_tmp || nsteps < 0 || ncomp < 1 ||
        (dt_mode != ADLBR_DT_ABS && dt_mode != ADLBR_DT_CFL)) {
        set_error("adlbr_step_multi: bad argument");
        return ADLBR_E_INVALID;
    }
    if (op->tiled) {
        set_error("adlbr_step_multi: needs the list layout (create without ADLBR_OP_TILED)");
        return ADLBR_E_UNSUPPORTED;
    }
    hipStream_t s = as_stream(stream);
    const size_t plane = (size_t)op->gi.N * dtype_size(op->storage);
    // components in groups of kMaxComp, each group stepped nsteps times
    for (int c0 = 0; c0 < ncomp; c0 += kMaxComp) {
        const int nc = std::min(kMaxComp, ncomp - c0);
        char *ua = (char *)u + c0 * plane, *ub = (char *)u_tmp + c0 * plane;
        void *a = ua, *b = ub;
        for (int64_t k = 0; k < nsteps; ++k) {
            int rc = dispatch<MultiF>(op, (const void *)a, b, nc, dt, dt_mode, s);
            if (rc) return rc;
            std::swap(a, b);
        }
        ADLBR_LAUNCH_CHECK();
        if (a != ua)
            ADLBR_CHECK_HIP(hipMemcpyAsync(ua, a, nc * plane, hipMemcpyDeviceToDevice, s));
    }
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
