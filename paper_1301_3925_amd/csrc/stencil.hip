// AD-LBR stencil construction on the GPU: one thread per grid point.
//
// 2D (Section 2): Lagrange's reduction of Z^2 for the metric of D, sign fix
// of Corollary 2, superbase (e, f, -e-f), weights of Lemma 1.
// 3D (Section 2): greedy D-reduced basis (Definition 2), Proposition
// (MakeObtuse), Selling's decomposition.
//
// Every decision (rounding of a projection coefficient, a norm comparison,
// a sign test) is an FP64 operation on products of exact integer
// coefficients with the tensor entries, in a fixed order, and this file is
// compiled with -ffp-contract=off: the integer offsets are therefore a
// deterministic function of the FP64 tensor, reproducible on any IEEE
// machine that evaluates the same expressions.
//
// The 2D metric is Q = adj(D) = det(D) D^{-1}, a positive multiple of the
// paper's M = det(D)^{1/2} D^{-1} (eq. (DM)); reduced and obtuse bases do not
// change under positive scaling, and <e^perp, D f^perp> = <e, Q f> gives the
// Lemma 1 weights from the same products.
#include "common.h"

namespace adlbr {
namespace {

constexpr int kMaxIter = 200;

// Both reductions run first in 32-bit integers, whose products and
// coefficient sums are exact while every component stays within +-32767
// (2 * 32767^2 < 2^31); a point whose reduction leaves that range is
// reduced again, from the start, in 64-bit integers.  The coefficients are
// the same integers either way, hence so are the doubles and every
// decision taken from them.
constexpr int kSmall = 32767;

// ------------------------------------------------------------------- 2D --
struct Form2 {
    double xx, xy, yy;
};

template <typename I> struct V2T {
    I x, y;
};
typedef V2T<ll> V2;

template <typename I> __device__ __forceinline__ double form2(const Form2 &q, V2T<I> a, V2T<I> b) {
    const I cxx = a.x * b.x;
    const I cxy = a.x * b.y + a.y * b.x;
    const I cyy = a.y * b.y;
    return ((double)cxx * q.xx + (double)cxy * q.xy) + (double)cyy * q.yy;
}

// Lagrange: repeat (e, f) := (f, e - Round(<e,f>/<f,f>) f) while |e| > |f|.
// Iterations used, -1 past kMaxIter, -2 when 32-bit integers overflow.
template <typename I> __device__ int reduce_pair2(const Form2 &q, V2T<I> &e, V2T<I> &f) {
    for (int it = 1; it <= kMaxIter; ++it) {
        const double r = round(form2(q, e, f) / form2(q, f, f));
        const ll k = (ll)r;
        V2T<I> g;
        if constexpr (sizeof(I) == 4) {
            if (k < -kSmall || k > kSmall) return -2;
            const int ki = (int)k;
            g = V2T<I>{e.x - ki * f.x, e.y - ki * f.y};
            if (g.x < -kSmall || g.x > kSmall || g.y < -kSmall || g.y > kSmall) return -2;
        } else {
            g = V2T<I>{e.x - k * f.x, e.y - k * f.y};
        }
        e = f;
        f = g;
        if (!(form2(q, e, e) > form2(q, f, f))) return it;
    }
    return -1;
}

template <typename TD, typename TW>
__global__ void k_stencil2d(const TD *__restrict__ D, long long N, int16_t *__restrict__ off,
                            TW *__restrict__ w, int32_t *status) {
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= N) return;
    const double dxx = (double)D[z], dxy = (double)D[N + z], dyy = (double)D[2 * N + z];
    int st = 0;
    V2 s[3] = {{0, 0}, {0, 0}, {0, 0}};
    double g[3] = {0.0, 0.0, 0.0};
    const bool finite = isfinite(dxx) && isfinite(dxy) && isfinite(dyy);
    if (!finite || !(dxx > 0.0) || !(dyy > 0.0) || !(dxx * dyy - dxy * dxy > 0.0)) {
        st |= ADLBR_ST_NOT_SPD;
    } else {
        const Form2 q{dyy, -dxy, dxx};
        V2 e{1, 0}, f{0, 1};
        V2T<int> ei{1, 0}, fi{0, 1};
        int red = reduce_pair2<int>(q, ei, fi);
        if (red == -2) {
            red = reduce_pair2<ll>(q, e, f);  // left the 32-bit range: again in 64 bits
        } else {
            e = V2{ei.x, ei.y};
            f = V2{fi.x, fi.y};
        }
        if (red < 0) st |= ADLBR_ST_ITER;
        if (form2(q, e, f) > 0.0) f = V2{-f.x, -f.y};
        s[0] = e;
        s[1] = f;
        s[2] = V2{-e.x - f.x, -e.y - f.y};
        // gamma(+-s_i) = -1/2 <s_{i+1}, Q s_{i+2}>
        for (int i = 0; i < 3; ++i) {
            double v = -0.5 * form2(q, s[(i + 1) % 3], s[(i + 2) % 3]);
            if (v < 0.0) {
                st |= ADLBR_ST_CLAMPED;
                v = 0.0;
            }
            g[i] = v;
        }
        for (int i = 0; i < 3; ++i)
            if (s[i].x > 32767 || s[i].x < -32767 || s[i].y > 32767 || s[i].y < -32767)
                st |= ADLBR_ST_RANGE;
    }
    if (st & (ADLBR_ST_NOT_SPD | ADLBR_ST_RANGE | ADLBR_ST_ITER)) {
        for (int i = 0; i < 3; ++i) {
            s[i] = V2{0, 0};
            g[i] = 0.0;
        }
    }
    for (int i = 0; i < 3; ++i) {
        off[(2 * i) * N + z] = (int16_t)s[i].x;
        off[(2 * i + 1) * N + z] = (int16_t)s[i].y;
        w[i * N + z] = (TW)g[i];
    }
    report(status, z, st);
}

// ------------------------------------------------------------------- 3D --
struct Form3 {
    double xx, yy, zz, xy, xz, yz;
};

// Lattice vectors with integer components of type I (32-bit first, see
// kSmall).
template <typename I> struct V3T {
    I x, y, z;
};
typedef V3T<ll> V3;

template <typename I>
__device__ __forceinline__ double form3(const Form3 &q, const V3T<I> &a, const V3T<I> &b) {
    const I cxx = a.x * b.x, cyy = a.y * b.y, czz = a.z * b.z;
    const I cxy = a.x * b.y + a.y * b.x;
    const I cxz = a.x * b.z + a.z * b.x;
    const I cyz = a.y * b.z + a.z * b.y;
    return (((((double)cxx * q.xx + (double)cyy * q.yy) + (double)czz * q.zz) +
             (double)cxy * q.xy) + (double)cxz * q.xz) + (double)cyz * q.yz;
}

template <typename I> __device__ __forceinline__ bool small3(const V3T<I> &v) {
    return v.x >= -kSmall && v.x <= kSmall && v.y >= -kSmall && v.y <= kSmall &&
           v.z >= -kSmall && v.z <= kSmall;
}

// y - k x; with 32-bit integers false (and no result) when k or the result
// leaves +-32767.  The coefficient arrives as the 64-bit integer the 64-bit
// reduction uses, so the two agree even where a rounded coefficient is too
// large for a double to hold its neighbours exactly.
template <typename I>
__device__ __forceinline__ bool v3_axpy(ll k, const V3T<I> &x, const V3T<I> &y, V3T<I> &out) {
    if constexpr (sizeof(I) == 4) {
        if (k < -kSmall || k > kSmall) return false;
        const int ki = (int)k;
        out = V3T<I>{y.x - ki * x.x, y.y - ki * x.y, y.z - ki * x.z};
        return small3(out);
    } else {
        out = V3T<I>{y.x - k * x.x, y.y - k * x.y, y.z - k * x.z};
        return true;
    }
}

// Lagrange on the pair: iterations used, -1 past kMaxIter, -2 when 32-bit
// integers overflow.
template <typename I> __device__ int reduce_pair3(const Form3 &q, V3T<I> &e, V3T<I> &f) {
    for (int it = 1; it <= kMaxIter; ++it) {
        const double r = round(form3(q, e, f) / form3(q, f, f));
        V3T<I> g;
        if (!v3_axpy<I>((ll)r, f, e, g)) return -2;
        e = f;
        f = g;
        if (!(form3(q, e, e) > form3(q, f, f))) return it;
    }
    return -1;
}

// Greedy reduction: sort by norm (stable), reduce the first two with
// Lagrange, replace the third by its offset from the closest vector of the
// plane lattice of the first two (searched among round(y) + {-1,0,1}^2,
// first minimum in i-major order), until the third is not shorter than the
// second.  1: reduced; 0: past kMaxIter; -2: 32-bit overflow.
template <typename I> __device__ int greedy3(const Form3 &q, V3T<I> b[3]) {
    for (int it = 0; it < kMaxIter; ++it) {
        // stable insertion sort of three vectors by squared norm
        for (int i = 1; i < 3; ++i)
            for (int j = i; j > 0 && form3(q, b[j - 1], b[j - 1]) > form3(q, b[j], b[j]); --j) {
                const V3T<I> t = b[j];
                b[j] = b[j - 1];
                b[j - 1] = t;
            }
        const int rp = reduce_pair3<I>(q, b[0], b[1]);
        if (rp == -2) return -2;
        if (rp < 0) return 0;
        const double g11 = form3(q, b[0], b[0]), g12 = form3(q, b[0], b[1]);
        const double g22 = form3(q, b[1], b[1]);
        const double p1 = form3(q, b[0], b[2]), p2 = form3(q, b[1], b[2]);
        const double det = g11 * g22 - g12 * g12;
        const double y1 = (p1 * g22 - p2 * g12) / det;
        const double y2 = (p2 * g11 - p1 * g12) / det;
        const ll c1 = (ll)round(y1), c2 = (ll)round(y2);
        double best = INFINITY;
        V3T<I> bv = b[2];
        for (int i = -1; i <= 1; ++i)
            for (int j = -1; j <= 1; ++j) {
                V3T<I> t, v;
                if (!v3_axpy<I>(c1 + i, b[0], b[2], t) || !v3_axpy<I>(c2 + j, b[1], t, v)) return -2;
                const double n2 = form3(q, v, v);
                if (n2 < best) {
                    best = n2;
                    bv = v;
                }
            }
        b[2] = bv;
        if (form3(q, b[2], b[2]) >= form3(q, b[1], b[1])) return 1;
    }
    return 0;
}

__device__ __forceinline__ V3 cross3(const V3 &a, const V3 &b) {
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__device__ __forceinline__ V3 neg3(const V3 &a) { return V3{-a.x, -a.y, -a.z}; }

// Proposition (MakeObtuse): order the reduced basis so that
// |<b1,b2>| <= |<b1,b3>| <= |<b2,b3>| (first such permutation in
// lexicographic order), make <b1,b3>, <b2,b3> <= 0 by sign flips, and pick
// one of the two superbases of eq. (3DSuperBase).
__device__ void obtuse_superbase3(const Form3 &q, const V3 r[3], V3 e[4]) {
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int p = 0;
    for (int k = 0; k < 6; ++k) {
        const V3 &a = r[perms[k][0]], &b = r[perms[k][1]], &c = r[perms[k][2]];
        const double ab = fabs(form3(q, a, b)), ac = fabs(form3(q, a, c)), bc = fabs(form3(q, b, c));
        if (ab <= ac && ac <= bc) {
            p = k;
            break;
        }
    }
    V3 b1 = r[perms[p][0]], b2 = r[perms[p][1]];
    const V3 b3 = r[perms[p][2]];
    if (form3(q, b1, b3) > 0.0) b1 = neg3(b1);
    if (form3(q, b2, b3) > 0.0) b2 = neg3(b2);
    if (form3(q, b1, b2) <= 0.0) {
        e[0] = b1;
        e[1] = b2;
        e[2] = b3;
        e[3] = V3{-b1.x - b2.x - b3.x, -b1.y - b2.y - b3.y, -b1.z - b2.z - b3.z};
    } else {
        e[0] = neg3(b1);
        e[1] = b2;
        e[2] = V3{b1.x + b3.x, b1.y + b3.y, b1.z + b3.z};
        e[3] = V3{-b2.x - b3.x, -b2.y - b3.y, -b2.z - b3.z};
    }
}

template <typename TD, typename TW>
__global__ void k_stencil3d(const TD *__restrict__ D, long long N, int16_t *__restrict__ off,
                            TW *__restrict__ w, int32_t *status) {
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= N) return;
    // input planes xx, xy, xz, yy, yz, zz
    const double a = (double)D[z], xy = (double)D[N + z], xz = (double)D[2 * N + z];
    const double b = (double)D[3 * N + z], yz = (double)D[4 * N + z], c = (double)D[5 * N + z];
    int st = 0;
    V3 cs[6];
    double g[6];
    for (int k = 0; k < 6; ++k) {
        cs[k] = V3{0, 0, 0};
        g[k] = 0.0;
    }
    bool ok = isfinite(a) && isfinite(b) && isfinite(c) && isfinite(xy) && isfinite(xz) &&
              isfinite(yz);
    ok = ok && a > 0.0 && a * b - xy * xy > 0.0;
    ok = ok && (a * (b * c - yz * yz) - xy * (xy * c - yz * xz) + xz * (xy * yz - b * xz)) > 0.0;
    if (!ok) {
        st |= ADLBR_ST_NOT_SPD;
    } else {
        const Form3 q{a, b, c, xy, xz, yz};
        V3 r[3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        V3T<int> ri[3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        int red = greedy3<int>(q, ri);
        if (red == -2) {
            red = greedy3<ll>(q, r);  // left the 32-bit range: again in 64 bits
        } else {
            for (int k = 0; k < 3; ++k) r[k] = V3{ri[k].x, ri[k].y, ri[k].z};
        }
        if (red != 1) {
            st |= ADLBR_ST_ITER;
        } else {
            V3 e[4];
            obtuse_superbase3(q, r, e);
            // Selling: pair (i,j) -> slot e_k x e_l, weight -1/2 <e_i, D e_j>
            const int pairs[6][4] = {{0, 1, 2, 3}, {0, 2, 1, 3}, {0, 3, 1, 2},
                                     {1, 2, 0, 3}, {1, 3, 0, 2}, {2, 3, 0, 1}};
            for (int k = 0; k < 6; ++k) {
                cs[k] = cross3(e[pairs[k][2]], e[pairs[k][3]]);
                double v = -0.5 * form3(q, e[pairs[k][0]], e[pairs[k][1]]);
                if (v < 0.0) {
                    st |= ADLBR_ST_CLAMPED;
                    v = 0.0;
                }
                g[k] = v;
                const ll m = max(max(llabs(cs[k].x), llabs(cs[k].y)), llabs(cs[k].z));
                if (m > 32767) st |= ADLBR_ST_RANGE;
            }
        }
    }
    if (st & (ADLBR_ST_NOT_SPD | ADLBR_ST_RANGE | ADLBR_ST_ITER)) {
        for (int k = 0; k < 6; ++k) {
            cs[k] = V3{0, 0, 0};
            g[k] = 0.0;
        }
    }
    for (int k = 0; k < 6; ++k) {
        off[(3 * k) * N + z] = (int16_t)cs[k].x;
        off[(3 * k + 1) * N + z] = (int16_t)cs[k].y;
        off[(3 * k + 2) * N + z] = (int16_t)cs[k].z;
        w[k * N + z] = (TW)g[k];
    }
    report(status, z, st);
}

template <typename TD, typename TW>
void launch_stencil(int dim, const void *D, long long N, int16_t *off, void *w, int32_t *status,
                    hipStream_t s) {
    const int bs = dim == 2 ? 256 : 128;
    const unsigned nb = (unsigned)((N + bs - 1) / bs);
    if (dim == 2)
        hipLaunchKernelGGL((k_stencil2d<TD, TW>), dim3(nb), dim3(bs), 0, s, (const TD *)D, N, off,
                           (TW *)w, status);
    else
        hipLaunchKernelGGL((k_stencil3d<TD, TW>), dim3(nb), dim3(bs), 0, s, (const TD *)D, N, off,
                           (TW *)w, status);
}

}  // namespace
}  // namespace adlbr

using namespace adlbr;

extern "C" int adlbr_build_stencils(const adlbr_grid *g, const void *D, int D_dtype,
                                    int16_t *offsets, void *weights, int w_dtype,
                                    int32_t *status, void *stream) {
    clear_error();
    GridInfo gi;
    int rc = check_grid(g, &gi);
    if (rc) return rc;
    if (!D || !offsets || !weights || !status) {
        set_error("adlbr_build_stencils: null pointer argument");
        return ADLBR_E_INVALID;
    }
    if ((D_dtype != ADLBR_F64 && D_dtype != ADLBR_F32) ||
        (w_dtype != ADLBR_F64 && w_dtype != ADLBR_F32)) {
        set_error("adlbr_build_stencils: D and weights must be ADLBR_F64 or ADLBR_F32");
        return ADLBR_E_INVALID;
    }
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, s, status);
    if (D_dtype == ADLBR_F64 && w_dtype == ADLBR_F64)
        launch_stencil<double, double>(gi.dim, D, gi.N, offsets, weights, status, s);
    else if (D_dtype == ADLBR_F64)
        launch_stencil<double, float>(gi.dim, D, gi.N, offsets, weights, status, s);
    else if (w_dtype == ADLBR_F64)
        launch_stencil<float, double>(gi.dim, D, gi.N, offsets, weights, status, s);
    else
        launch_stencil<float, float>(gi.dim, D, gi.N, offsets, weights, status, s);
    hipLaunchKernelGGL(k_status_final, dim3(1), dim3(1), 0, s, status);
    ADLBR_LAUNCH_CHECK();
    return ADLBR_OK;
}
