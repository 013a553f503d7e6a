/*
 * AD-LBR reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of what the AD-LBR hot path
 * computes (Fehrenbach & Mirebeau, "Sparse non-negative stencils for
 * anisotropic diffusion").  It is used by the test-suite, the smoke check and
 * the benchmark's CPU baseline only; the product path never calls it.  It
 * shares no code with the HIP library.
 *
 * Compiled with gcc -O2 -ffp-contract=off (no FMA contraction), so every
 * floating-point decision is a plain IEEE double operation in the order
 * written here.
 *
 * Conventions (readings of the paper, each listed in the design doc):
 *  - 2D tensors are 3 planes (Dxx, Dxy, Dyy); 3D tensors are 6 planes
 *    (Dxx, Dxy, Dxz, Dyy, Dyz, Dzz); arrays are x-fastest.
 *  - The 2D reduction runs on Q = adj(D) = det(D) D^{-1}, a positive multiple
 *    of the paper's metric M = det(D)^{1/2} D^{-1} (Section 1, eq. (DM));
 *    reduced and obtuse bases do not depend on a positive scale.
 *  - Scalar products <e, Q f> of integer vectors are formed from the exact
 *    integer coefficients (c_xx, c_xy, c_yy) as ((c_xx Qxx + c_xy Qxy) +
 *    c_yy Qyy); in 3D as (((((c_xx Dxx + c_yy Dyy) + c_zz Dzz) + c_xy Dxy)
 *    + c_xz Dxz) + c_yz Dyz).  Both sides of a parity test must take the same
 *    decisions from the same doubles.
 *  - Round() is round-half-away-from-zero (C round()).
 *  - Weights use the paper's own formulas: in 2D the perpendicular form
 *    gamma(+-e_i) = -1/2 <e_{i+1}^perp, D e_{i+2}^perp> (Lemma 1, eq.
 *    (GammaZ)); in 3D Selling's -1/2 <e_i, D e_j> (Section 2, Lemma
 *    (Selling)); both clamped at 0 (they are >= 0 in exact arithmetic).
 *
 * Status codes per point (bit mask): 1 = not SPD / non-finite,
 * 2 = offset outside int16, 4 = iteration cap hit, 8 = a weight was clamped,
 * 16 = the 3x3 closest-vector search found a better candidate outside the
 * +-1 window (must never happen for a reduced pair).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXIT 200

/* ------------------------------------------------------------------ 2D -- */

/* <e, Q f> for integer vectors, Q = (Qxx, Qxy, Qyy). */
static double dot2q(const double Q[3], const int64_t e[2], const int64_t f[2])
{
    int64_t cxx = e[0] * f[0];
    int64_t cxy = e[0] * f[1] + e[1] * f[0];
    int64_t cyy = e[1] * f[1];
    return ((double)cxx * Q[0] + (double)cxy * Q[1]) + (double)cyy * Q[2];
}

/* <a, D b> for real 2-vectors, D = (Dxx, Dxy, Dyy), natural form. */
static double dot2d(const double D[3], const double a[2], const double b[2])
{
    double Db0 = D[0] * b[0] + D[1] * b[1];
    double Db1 = D[1] * b[0] + D[2] * b[1];
    return a[0] * Db0 + a[1] * Db1;
}

static int spd2(const double D[3])
{
    if (!isfinite(D[0]) || !isfinite(D[1]) || !isfinite(D[2])) return 0;
    if (!(D[0] > 0.0) || !(D[2] > 0.0)) return 0;
    return D[0] * D[2] - D[1] * D[1] > 0.0;
}

/* Lagrange's reduction (Section 2, eq. (GaussAlgo)) of the basis (e, f)
 * for the quadratic form Q:  do (e,f) := (f, e - Round(<e,Qf>/|f|^2) f)
 * while |e| > |f|.  Returns the number of iterations, or -1 at the cap. */
static int lagrange(const double Q[3], int64_t e[2], int64_t f[2],
                    double (*dot)(const double *, const int64_t *, const int64_t *))
{
    int it = 0;
    for (;;) {
        double r = round(dot(Q, e, f) / dot(Q, f, f));
        int64_t k = (int64_t)r;
        int64_t ne0 = f[0], ne1 = f[1];
        int64_t nf0 = e[0] - k * f[0], nf1 = e[1] - k * f[1];
        e[0] = ne0; e[1] = ne1; f[0] = nf0; f[1] = nf1;
        ++it;
        if (!(dot(Q, e, e) > dot(Q, f, f))) return it;
        if (it >= OR_MAXIT) return -1;
    }
}

/* Reduced basis (e, f) of Z^2 for the metric of D (before the sign fix). */
int or_reduce2d(const double *D, int64_t n, int64_t *basis /* [2][2][n] */,
                int32_t *iters)
{
    int bad = 0;
    for (int64_t z = 0; z < n; ++z) {
        double Dz[3] = {D[z], D[n + z], D[2 * n + z]};
        int64_t e[2] = {1, 0}, f[2] = {0, 1};
        int it = 0;
        if (spd2(Dz)) {
            double Q[3] = {Dz[2], -Dz[1], Dz[0]};
            it = lagrange(Q, e, f, dot2q);
        } else {
            it = -1;
            bad = 1;
        }
        basis[0 * n + z] = e[0]; basis[1 * n + z] = e[1];
        basis[2 * n + z] = f[0]; basis[3 * n + z] = f[1];
        if (iters) iters[z] = it;
    }
    return bad;
}

/* 2D AD-LBR stencil (Section 2: reduce, make obtuse, Lemma 1 weights).
 * off: [3][2][n] int16 slot offsets (e, f, g); the stencil is +-each slot.
 * w:   [3][n] weights gamma(+-slot).   status: [n] bit mask. */
int or_stencil2d(const double *D, int64_t n, int16_t *off, double *w,
                 int32_t *status)
{
    int any = 0;
    for (int64_t z = 0; z < n; ++z) {
        double Dz[3] = {D[z], D[n + z], D[2 * n + z]};
        int st = 0;
        int64_t s[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        double wz[3] = {0.0, 0.0, 0.0};
        if (!spd2(Dz)) {
            st |= 1;
        } else {
            double Q[3] = {Dz[2], -Dz[1], Dz[0]};
            int64_t e[2] = {1, 0}, f[2] = {0, 1};
            if (lagrange(Q, e, f, dot2q) < 0) st |= 4;
            /* Corollary 2: make <e, M f> <= 0 (strict test, no flip at 0). */
            if (dot2q(Q, e, f) > 0.0) { f[0] = -f[0]; f[1] = -f[1]; }
            s[0][0] = e[0]; s[0][1] = e[1];
            s[1][0] = f[0]; s[1][1] = f[1];
            s[2][0] = -e[0] - f[0]; s[2][1] = -e[1] - f[1];
            for (int i = 0; i < 3; ++i) {
                const int64_t *a = s[(i + 1) % 3], *b = s[(i + 2) % 3];
                double ap[2] = {(double)-a[1], (double)a[0]};
                double bp[2] = {(double)-b[1], (double)b[0]};
                double g = -0.5 * dot2d(Dz, ap, bp);
                if (g < 0.0) { st |= 8; g = 0.0; }
                wz[i] = g;
            }
            for (int i = 0; i < 3; ++i)
                for (int c = 0; c < 2; ++c)
                    if (s[i][c] > 32767 || s[i][c] < -32767) st |= 2;
        }
        if (st & 7) {
            memset(s, 0, sizeof s);
            wz[0] = wz[1] = wz[2] = 0.0;
        }
        for (int i = 0; i < 3; ++i) {
            off[(2 * i + 0) * n + z] = (int16_t)s[i][0];
            off[(2 * i + 1) * n + z] = (int16_t)s[i][1];
            w[i * n + z] = wz[i];
        }
        status[z] = st;
        any |= st;
    }
    return any;
}

/* ------------------------------------------------------------------ 3D -- */

/* D3 = (Dxx, Dyy, Dzz, Dxy, Dxz, Dyz) internally. */
static double dot3q(const double D3[6], const int64_t a[3], const int64_t b[3])
{
    int64_t cxx = a[0] * b[0], cyy = a[1] * b[1], czz = a[2] * b[2];
    int64_t cxy = a[0] * b[1] + a[1] * b[0];
    int64_t cxz = a[0] * b[2] + a[2] * b[0];
    int64_t cyz = a[1] * b[2] + a[2] * b[1];
    return ((((((double)cxx * D3[0] + (double)cyy * D3[1]) + (double)czz * D3[2])
              + (double)cxy * D3[3]) + (double)cxz * D3[4]) + (double)cyz * D3[5]);
}

/* natural <a, D b> for real 3-vectors, D3 as above */
static double dot3d(const double D3[6], const double a[3], const double b[3])
{
    double Db0 = D3[0] * b[0] + D3[3] * b[1] + D3[4] * b[2];
    double Db1 = D3[3] * b[0] + D3[1] * b[1] + D3[5] * b[2];
    double Db2 = D3[4] * b[0] + D3[5] * b[1] + D3[2] * b[2];
    return a[0] * Db0 + a[1] * Db1 + a[2] * Db2;
}

static int spd3(const double D3[6])
{
    for (int i = 0; i < 6; ++i) if (!isfinite(D3[i])) return 0;
    double a = D3[0], b = D3[1], c = D3[2], xy = D3[3], xz = D3[4], yz = D3[5];
    if (!(a > 0.0)) return 0;
    if (!(a * b - xy * xy > 0.0)) return 0;
    double det = a * (b * c - yz * yz) - xy * (xy * c - yz * xz) + xz * (xy * yz - b * xz);
    return det > 0.0;
}

/* 2D Lagrange loop for a pair of 3D vectors under the form D3. */
static int lagrange3(const double D3[6], int64_t e[3], int64_t f[3])
{
    int it = 0;
    for (;;) {
        double r = round(dot3q(D3, e, f) / dot3q(D3, f, f));
        int64_t k = (int64_t)r;
        int64_t ne[3] = {f[0], f[1], f[2]};
        int64_t nf[3] = {e[0] - k * f[0], e[1] - k * f[1], e[2] - k * f[2]};
        memcpy(e, ne, sizeof ne);
        memcpy(f, nf, sizeof nf);
        ++it;
        if (!(dot3q(D3, e, e) > dot3q(D3, f, f))) return it;
        if (it >= OR_MAXIT) return -1;
    }
}

/* Greedy reduction of a basis of Z^3 (the recursive greedy algorithm of
 * Semaev / Nguyen-Stehle cited in Section 2, which the paper uses but does
 * not print): sort by norm, Lagrange-reduce the first two vectors, replace
 * the third by its distance to the closest vector of the plane lattice they
 * span, repeat until the third is not shorter than the second.  The output
 * is a D-reduced (Minkowski) basis, Definition 2. */
static int greedy3(const double D3[6], int64_t b[3][3], int *flags)
{
    int it = 0;
    for (;;) {
        /* stable insertion sort by squared norm */
        for (int i = 1; i < 3; ++i) {
            int j = i;
            while (j > 0 && dot3q(D3, b[j - 1], b[j - 1]) > dot3q(D3, b[j], b[j])) {
                int64_t t[3];
                memcpy(t, b[j], sizeof t);
                memcpy(b[j], b[j - 1], sizeof t);
                memcpy(b[j - 1], t, sizeof t);
                --j;
            }
        }
        if (lagrange3(D3, b[0], b[1]) < 0) { *flags |= 4; return -1; }
        /* real coordinates of the projection of b2 on span(b0, b1) */
        double g11 = dot3q(D3, b[0], b[0]), g12 = dot3q(D3, b[0], b[1]);
        double g22 = dot3q(D3, b[1], b[1]);
        double p1 = dot3q(D3, b[0], b[2]), p2 = dot3q(D3, b[1], b[2]);
        double det = g11 * g22 - g12 * g12;
        double y1 = (p1 * g22 - p2 * g12) / det;
        double y2 = (p2 * g11 - p1 * g12) / det;
        int64_t c1 = (int64_t)round(y1), c2 = (int64_t)round(y2);
        /* closest vector among round(y) + {-1,0,1}^2 (i-major, first min) */
        double best = INFINITY;
        int64_t bv[3] = {0, 0, 0};
        for (int i = -1; i <= 1; ++i)
            for (int j = -1; j <= 1; ++j) {
                int64_t x1 = c1 + i, x2 = c2 + j;
                int64_t v[3];
                for (int c = 0; c < 3; ++c) v[c] = b[2][c] - x1 * b[0][c] - x2 * b[1][c];
                double q = dot3q(D3, v, v);
                if (q < best) { best = q; memcpy(bv, v, sizeof bv); }
            }
        /* check: no candidate in the +-2 window is strictly better */
        for (int i = -2; i <= 2; ++i)
            for (int j = -2; j <= 2; ++j) {
                if (i >= -1 && i <= 1 && j >= -1 && j <= 1) continue;
                int64_t v[3];
                for (int c = 0; c < 3; ++c)
                    v[c] = b[2][c] - (c1 + i) * b[0][c] - (c2 + j) * b[1][c];
                if (dot3q(D3, v, v) < best) *flags |= 16;
            }
        memcpy(b[2], bv, sizeof bv);
        ++it;
        if (dot3q(D3, b[2], b[2]) >= dot3q(D3, b[1], b[1])) return it;
        if (it >= OR_MAXIT) { *flags |= 4; return -1; }
    }
}

static void load3(const double *D, int64_t n, int64_t z, double D3[6])
{
    /* input planes: xx, xy, xz, yy, yz, zz */
    D3[0] = D[0 * n + z];
    D3[3] = D[1 * n + z];
    D3[4] = D[2 * n + z];
    D3[1] = D[3 * n + z];
    D3[5] = D[4 * n + z];
    D3[2] = D[5 * n + z];
}

int or_reduce3d(const double *D, int64_t n, int64_t *basis /* [3][3][n] */,
                int32_t *status)
{
    int any = 0;
    for (int64_t z = 0; z < n; ++z) {
        double D3[6];
        load3(D, n, z, D3);
        int64_t b[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        int fl = 0;
        if (!spd3(D3)) fl |= 1; else greedy3(D3, b, &fl);
        for (int i = 0; i < 3; ++i)
            for (int c = 0; c < 3; ++c) basis[(3 * i + c) * n + z] = b[i][c];
        if (status) status[z] = fl;
        any |= fl;
    }
    return any;
}

static void cross3(const int64_t a[3], const int64_t b[3], int64_t c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Proposition (MakeObtuse): from a D-reduced basis build a D-obtuse
 * superbase (e0, e1, e2, e3). */
static void make_obtuse(const double D3[6], int64_t r[3][3], int64_t sb[4][3])
{
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                   {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int p = 0;
    for (int k = 0; k < 6; ++k) {
        const int64_t *a = r[perm[k][0]], *b = r[perm[k][1]], *c = r[perm[k][2]];
        double ab = fabs(dot3q(D3, a, b)), ac = fabs(dot3q(D3, a, c));
        double bc = fabs(dot3q(D3, b, c));
        if (ab <= ac && ac <= bc) { p = k; break; }
    }
    int64_t b1[3], b2[3], b3[3];
    memcpy(b1, r[perm[p][0]], sizeof b1);
    memcpy(b2, r[perm[p][1]], sizeof b2);
    memcpy(b3, r[perm[p][2]], sizeof b3);
    if (dot3q(D3, b1, b3) > 0.0) for (int c = 0; c < 3; ++c) b1[c] = -b1[c];
    if (dot3q(D3, b2, b3) > 0.0) for (int c = 0; c < 3; ++c) b2[c] = -b2[c];
    if (dot3q(D3, b1, b2) <= 0.0) {
        for (int c = 0; c < 3; ++c) {
            sb[0][c] = b1[c]; sb[1][c] = b2[c]; sb[2][c] = b3[c];
            sb[3][c] = -b1[c] - b2[c] - b3[c];
        }
    } else {
        for (int c = 0; c < 3; ++c) {
            sb[0][c] = -b1[c]; sb[1][c] = b2[c]; sb[2][c] = b1[c] + b3[c];
            sb[3][c] = -b2[c] - b3[c];
        }
    }
}

int or_superbase3d(const double *D, int64_t n, int64_t *sbo /* [4][3][n] */,
                   int32_t *status)
{
    int any = 0;
    for (int64_t z = 0; z < n; ++z) {
        double D3[6];
        load3(D, n, z, D3);
        int64_t b[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        int64_t sb[4][3] = {{0}};
        int fl = 0;
        if (!spd3(D3)) fl |= 1;
        else if (greedy3(D3, b, &fl) >= 0) make_obtuse(D3, b, sb);
        for (int i = 0; i < 4; ++i)
            for (int c = 0; c < 3; ++c) sbo[(3 * i + c) * n + z] = sb[i][c];
        if (status) status[z] = fl;
        any |= fl;
    }
    return any;
}

/* 3D AD-LBR stencil: superbase + Selling's decomposition.
 * Pairs (i,j) in order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3); offset
 * c_ij = e_k x e_l with {k<l} the complement; weight -1/2 <e_i, D e_j>.
 * off: [6][3][n] int16, w: [6][n]. */
int or_stencil3d(const double *D, int64_t n, int16_t *off, double *w,
                 int32_t *status)
{
    static const int pr[6][4] = {{0, 1, 2, 3}, {0, 2, 1, 3}, {0, 3, 1, 2},
                                 {1, 2, 0, 3}, {1, 3, 0, 2}, {2, 3, 0, 1}};
    int any = 0;
    for (int64_t z = 0; z < n; ++z) {
        double D3[6];
        load3(D, n, z, D3);
        int64_t b[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        int64_t sb[4][3];
        int64_t c6[6][3];
        double w6[6];
        int fl = 0;
        memset(c6, 0, sizeof c6);
        memset(w6, 0, sizeof w6);
        if (!spd3(D3)) {
            fl |= 1;
        } else if (greedy3(D3, b, &fl) >= 0) {
            make_obtuse(D3, b, sb);
            for (int q = 0; q < 6; ++q) {
                int i = pr[q][0], j = pr[q][1], k = pr[q][2], l = pr[q][3];
                cross3(sb[k], sb[l], c6[q]);
                double ei[3] = {(double)sb[i][0], (double)sb[i][1], (double)sb[i][2]};
                double ej[3] = {(double)sb[j][0], (double)sb[j][1], (double)sb[j][2]};
                double g = -0.5 * dot3d(D3, ei, ej);
                if (g < 0.0) { fl |= 8; g = 0.0; }
                w6[q] = g;
                for (int c = 0; c < 3; ++c)
                    if (c6[q][c] > 32767 || c6[q][c] < -32767) fl |= 2;
            }
        }
        if (fl & 7) { memset(c6, 0, sizeof c6); memset(w6, 0, sizeof w6); }
        for (int q = 0; q < 6; ++q) {
            for (int c = 0; c < 3; ++c) off[(3 * q + c) * n + z] = (int16_t)c6[q][c];
            w[q * n + z] = w6[q];
        }
        status[z] = fl;
        any |= fl;
    }
    return any;
}

/* ----------------------------------------------------------- operator -- */

static int64_t mirror(int64_t i, int64_t n);

/* Scatter form of A = 1/2 grad E_h (eq. (def:E*)) with h = 1: every
 * directed edge (y, y + s*o_i(y)) whose target lies in the grid adds
 * w_i(y) (delta_y - delta_t)(delta_y - delta_t)^T.  Emits COO triplets
 * (4 per edge) that the caller sums into a sparse matrix.
 * dims: n[0..dim-1]; mode 0 drops an edge whose target leaves the grid
 * (Neumann truncation V(z;h), Section 1), mode 1 wraps it (periodic),
 * mode 2 reflects it back (half-sample mirror: the even extension of u,
 * the reflecting boundary of the restoration test, Section 4).  Returns
 * the number of triplets. */
int64_t or_operator_coo(int dim, const int64_t *nd, int mode,
                        const int16_t *off, const double *w,
                        int64_t *ri, int64_t *ci, double *v)
{
    int64_t nx = nd[0], ny = nd[1], nz = dim == 3 ? nd[2] : 1;
    int64_t n = nx * ny * nz;
    int K = dim == 2 ? 3 : 6;
    int64_t t = 0;
    for (int64_t y = 0; y < n; ++y) {
        int64_t p[3] = {y % nx, (y / nx) % ny, y / (nx * ny)};
        for (int i = 0; i < K; ++i) {
            double wy = w[i * n + y];
            if (wy == 0.0) continue;
            for (int s = -1; s <= 1; s += 2) {
                int64_t q[3] = {p[0], p[1], p[2]};
                int inside = 1;
                for (int c = 0; c < dim; ++c) {
                    int64_t len = nd[c];
                    q[c] = p[c] + s * (int64_t)off[(dim * i + c) * n + y];
                    if (mode == 1) {
                        q[c] %= len;
                        if (q[c] < 0) q[c] += len;
                    } else if (mode == 2) {
                        q[c] = mirror(q[c], len);
                    } else if (q[c] < 0 || q[c] >= len) {
                        inside = 0;
                    }
                }
                if (!inside) continue;
                int64_t tz = q[0] + nx * (q[1] + ny * q[2]);
                ri[t] = y;  ci[t] = y;  v[t] = wy;  ++t;
                ri[t] = y;  ci[t] = tz; v[t] = -wy; ++t;
                ri[t] = tz; ci[t] = tz; v[t] = wy;  ++t;
                ri[t] = tz; ci[t] = y;  v[t] = -wy; ++t;
            }
        }
    }
    return t;
}

static int64_t mirror(int64_t i, int64_t n)
{
    /* half-sample symmetric extension: -1 -> 0, n -> n-1, period 2n */
    int64_t p = 2 * n;
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - 1 - i;
}

/* ---------------------------------------------------------------- CED -- */

static int64_t reflect(int64_t i, int64_t n)
{
    /* half-sample symmetric extension: -1 -> 0, n -> n-1, period 2n */
    int64_t p = 2 * n;
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - 1 - i;
}

static double *gauss_taps(double s, int *r_out)
{
    int r = (int)ceil(3.0 * s);
    if (r < 1) r = 1;
    double *g = (double *)malloc(sizeof(double) * (2 * r + 1));
    double sum = 0.0;
    for (int k = -r; k <= r; ++k) {
        g[k + r] = exp(-(double)(k * k) / (2.0 * s * s));
        sum += g[k + r];
    }
    for (int k = 0; k < 2 * r + 1; ++k) g[k] /= sum;
    *r_out = r;
    return g;
}

/* separable Gaussian blur along axis `ax` of a field with dims nd */
static void blur_axis(const double *in, double *out, int dim, const int64_t *nd,
                      int ax, const double *g, int r)
{
    int64_t nx = nd[0], ny = nd[1], nz = dim == 3 ? nd[2] : 1;
    int64_t n = nx * ny * nz;
    int64_t stride = ax == 0 ? 1 : (ax == 1 ? nx : nx * ny);
    int64_t len = nd[ax];
    for (int64_t z = 0; z < n; ++z) {
        int64_t p = ax == 0 ? z % nx : (ax == 1 ? (z / nx) % ny : z / (nx * ny));
        double acc = 0.0;
        for (int k = -r; k <= r; ++k)
            acc += g[k + r] * in[z + (reflect(p + k, len) - p) * stride];
        out[z] = acc;
    }
}

static void blur(const double *in, double *out, double *tmp, int dim,
                 const int64_t *nd, double s)
{
    int r;
    double *g = gauss_taps(s, &r);
    int64_t n = nd[0] * nd[1] * (dim == 3 ? nd[2] : 1);
    if (dim == 2) {
        blur_axis(in, tmp, dim, nd, 0, g, r);
        blur_axis(tmp, out, dim, nd, 1, g, r);
    } else {
        blur_axis(in, out, dim, nd, 0, g, r);
        blur_axis(out, tmp, dim, nd, 1, g, r);
        blur_axis(tmp, out, dim, nd, 2, g, r);
    }
    (void)n;
    free(g);
}

/* Eigen-decomposition of a symmetric 2x2 matrix by one Jacobi rotation:
 * mu[0] >= mu[1], v[0] the eigenvector of mu[0]. */
static void eig2(double a, double b, double c, double mu[2], double v[2][2])
{
    double th = 0.5 * atan2(2.0 * b, a - c);
    double cs = cos(th), sn = sin(th);
    double m1 = a * cs * cs + 2.0 * b * cs * sn + c * sn * sn;
    double m2 = a * sn * sn - 2.0 * b * cs * sn + c * cs * cs;
    if (m1 >= m2) {
        mu[0] = m1; mu[1] = m2;
        v[0][0] = cs; v[0][1] = sn; v[1][0] = -sn; v[1][1] = cs;
    } else {
        mu[0] = m2; mu[1] = m1;
        v[0][0] = -sn; v[0][1] = cs; v[1][0] = cs; v[1][1] = sn;
    }
}

/* Cyclic Jacobi for a symmetric 3x3 matrix A (overwritten): eigenvalues on
 * the diagonal, eigenvectors in the columns of V.  Sorted descending. */
static void eig3(double A[3][3], double mu[3], double V[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off <= 1e-15 * scale || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                double th = 0.5 * atan2(2.0 * A[p][q], A[q][q] - A[p][p]);
                double c = cos(th), s = sin(th);
                /* A := J^T A J with J the rotation in the (p,q) plane */
                for (int k = 0; k < 3; ++k) {
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int idx[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (A[idx[j]][idx[j]] > A[idx[i]][idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
    double W[3][3];
    for (int k = 0; k < 3; ++k) {
        mu[k] = A[idx[k]][idx[k]];
        for (int i = 0; i < 3; ++i) W[i][k] = V[i][idx[k]];
    }
    memcpy(V, W, sizeof W);
}

static double coherence(double C, double dmu)
{
    /* exp(-C / dmu^2), with exp(-C/0) := 0 */
    if (dmu == 0.0) return 0.0;
    return exp(-C / (dmu * dmu));
}

/* Structure-tensor diffusion tensor (Section 4: coherence-enhancing
 * diffusion in 2D and 3D; edge-enhancing variant for 3D):
 * u_sigma = K_sigma * u, J = K_rho * (grad u_sigma grad u_sigma^T),
 * for a vector-valued image (ncomp planes of n values) the sum of the
 * components' products grad u_c,sigma grad u_c,sigma^T before the K_rho
 * blur (the common tensor; the Conclusion leaves the coupling to it),
 * D = sum lambda_k v_k v_k^T with the eigenvalue map `map`:
 *   map 0 (CED): lambda_1 = alpha, lambda_k = alpha + (1-alpha) exp(-C/(mu_1-mu_k)^2)
 *   map 1 (EED): lambda_k = 1 - exp(-C/mu_k^2) for k < d, lambda_d = 1
 * sigma, rho are standard deviations; kernels truncated at ceil(3 s) and
 * normalized; mirror boundary; central differences. */
int or_structure_tensor_d(int dim, const int64_t *nd, const double *u, int ncomp,
                          double sigma, double rho, double alpha, double C,
                          int map, double *Dout)
{
    int64_t n = nd[0] * nd[1] * (dim == 3 ? nd[2] : 1);
    int nj = dim == 2 ? 3 : 6;
    double *us = (double *)malloc(sizeof(double) * n);
    double *tmp = (double *)malloc(sizeof(double) * n);
    double *J = (double *)calloc((size_t)(n * nj), sizeof(double));
    double *Js = (double *)malloc(sizeof(double) * n);
    int64_t nx = nd[0], ny = nd[1];
    for (int comp = 0; comp < ncomp; ++comp) {
        blur(u + comp * n, us, tmp, dim, nd, sigma);
        for (int64_t z = 0; z < n; ++z) {
            int64_t p[3] = {z % nx, (z / nx) % ny, z / (nx * ny)};
            int64_t st[3] = {1, nx, nx * ny};
            double g[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < dim; ++c) {
                int64_t ip = reflect(p[c] + 1, nd[c]), im = reflect(p[c] - 1, nd[c]);
                g[c] = 0.5 * (us[z + (ip - p[c]) * st[c]] - us[z + (im - p[c]) * st[c]]);
            }
            /* upper triangle of g g^T, row by row */
            int q = 0;
            for (int a = 0; a < dim; ++a)
                for (int b = a; b < dim; ++b, ++q)
                    J[q * n + z] += g[a] * g[b];
        }
    }
    for (int k = 0; k < nj; ++k) {
        blur(J + k * n, Js, tmp, dim, nd, rho);
        memcpy(J + k * n, Js, sizeof(double) * n);
    }
    for (int64_t z = 0; z < n; ++z) {
        if (dim == 2) {
            double mu[2], v[2][2], lam[2];
            eig2(J[z], J[n + z], J[2 * n + z], mu, v);
            if (map == 0) {
                lam[0] = alpha;
                lam[1] = alpha + (1.0 - alpha) * coherence(C, mu[0] - mu[1]);
            } else {
                lam[0] = mu[0] == 0.0 ? 1.0 : 1.0 - exp(-C / (mu[0] * mu[0]));
                lam[1] = 1.0;
            }
            double dxx = 0, dxy = 0, dyy = 0;
            for (int k = 0; k < 2; ++k) {
                dxx += lam[k] * v[k][0] * v[k][0];
                dxy += lam[k] * v[k][0] * v[k][1];
                dyy += lam[k] * v[k][1] * v[k][1];
            }
            Dout[z] = dxx; Dout[n + z] = dxy; Dout[2 * n + z] = dyy;
        } else {
            double A[3][3] = {{J[z], J[n + z], J[2 * n + z]},
                              {J[n + z], J[3 * n + z], J[4 * n + z]},
                              {J[2 * n + z], J[4 * n + z], J[5 * n + z]}};
            double mu[3], V[3][3], lam[3];
            eig3(A, mu, V);
            if (map == 0) {
                lam[0] = alpha;
                lam[1] = alpha + (1.0 - alpha) * coherence(C, mu[0] - mu[1]);
                lam[2] = alpha + (1.0 - alpha) * coherence(C, mu[0] - mu[2]);
            } else {
                lam[0] = mu[0] == 0.0 ? 1.0 : 1.0 - exp(-C / (mu[0] * mu[0]));
                lam[1] = mu[1] == 0.0 ? 1.0 : 1.0 - exp(-C / (mu[1] * mu[1]));
                lam[2] = 1.0;
            }
            static const int pq[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
            for (int q = 0; q < 6; ++q) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    acc += lam[k] * V[pq[q][0]][k] * V[pq[q][1]][k];
                Dout[q * n + z] = acc;
            }
        }
    }
    free(us); free(tmp); free(J); free(Js);
    return 0;
}
