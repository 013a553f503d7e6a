"""Pins of the oracle operator A = 1/2 grad E_h and explicit Euler.

The operator is checked against the energy's definition by brute force
(polarization on tiny grids), against the closed form for quadratic u with
constant D, and against the structural properties the paper states:
symmetric, non-positive off-diagonal, annihilates constants, conserves mass,
and the maximum principle for dt <= 1 / max A_zz.
"""
import numpy as np

import oracle
from oracle import brute
from paper_1301_3925_amd import synth


def _case2d(n=(9, 7), kappa=10.0, seed=5):
    D = synth.tensor2d_field(seed, n[0], n[1], kappa)
    off, w, _ = oracle.stencil2d(D)
    return n, off, w


def _case3d(n=(5, 4, 4), kappa=8.0, seed=6):
    D = synth.tensor3d_field(seed, n, kappa)
    off, w, _ = oracle.stencil3d(D)
    return n, off, w


def test_dense_operator_equals_energy_polarization():
    """u^T A u = E_h(u) for all u (A = 1/2 grad E_h, eq. (def:E*)): the
    dense matrix read off the energy by polarization equals the scattered
    CSR operator entry by entry (2D Neumann, 2D periodic, 3D Neumann)."""
    for dims, off, w, per in [(*_case2d(), False), (*_case2d((6, 6), 5.0, 9), True),
                              (*_case3d(), False)]:
        n = int(np.prod(dims))
        A = oracle.operator_matrix(dims, off, w, periodic=per).toarray()
        Ad = brute.dense_operator_from_energy(
            lambda u: oracle.energy(dims, off, w, u, periodic=per), n)
        assert np.max(np.abs(A - Ad)) <= 1e-12 * np.max(np.abs(A))


def test_structure_symmetric_nonneg_constants():
    """Non-negativity paragraph of Section 1: A symmetric semi-definite,
    off-diagonal <= 0, diagonal > 0; A 1 = 0 (so mass is conserved).
    Reading: under Neumann truncation a boundary point whose offsets all
    leave the grid and that no stencil reaches is isolated (zero row), so
    the diagonal is >= 0 everywhere and > 0 at interior points."""
    for dims, off, w in [_case2d((40, 33), 50.0), _case3d((10, 9, 8), 30.0)]:
        A = oracle.operator_matrix(dims, off, w)
        assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
        Ao = A.tocoo()
        offd = Ao.data[Ao.row != Ao.col]
        assert np.all(offd <= 0.0)
        assert np.all(A.diagonal() >= 0.0)
        # a point with one positive-weight offset that stays in the grid
        # has a positive diagonal
        X = np.indices(dims[::-1]).reshape(len(dims), -1)[::-1]
        linked = np.zeros(A.shape[0], bool)
        for i in range(w.shape[0]):
            for sg in (-1, 1):
                q = X + sg * off[i].astype(np.int64)
                ok = np.all([(q[c] >= 0) & (q[c] < dims[c]) for c in range(len(dims))], axis=0)
                linked |= ok & (w[i] > 0)
        assert linked.mean() > 0.9 and np.all(A.diagonal()[linked] > 0.0)
        one = np.ones(A.shape[0])
        assert np.max(np.abs(A @ one)) <= 1e-13 * A.diagonal().max()
        u = synth.uniform(3, A.shape[0])
        assert u @ (A @ u) >= -1e-12


def test_quadratic_u_constant_d_closed_form():
    """Constant D and u = 1/2 x^T S x: at interior points (A u)(z) = -tr(D S),
    since the linear terms cancel over the symmetric stencil and
    sum gamma e e^T = D (eq. (DSum))."""
    rng = np.random.default_rng(0)
    for dim in (2, 3):
        n = (24, 24) if dim == 2 else (14, 14, 14)
        N = int(np.prod(n))
        if dim == 2:
            D = synth.tensor2d_const(0.7, 4.0, N)
            off, w, _ = oracle.stencil2d(D)
            Dm = np.array([[D[0, 0], D[1, 0]], [D[1, 0], D[2, 0]]])
        else:
            D = np.repeat(synth.random_spd3(4, 1, 3.0), N, axis=1)
            off, w, _ = oracle.stencil3d(D)
            Dm = np.array([[D[0, 0], D[1, 0], D[2, 0]], [D[1, 0], D[3, 0], D[4, 0]],
                           [D[2, 0], D[4, 0], D[5, 0]]])
        S = rng.normal(size=(dim, dim))
        S = S + S.T
        X = np.indices(n[::-1]).reshape(dim, -1)[::-1].astype(np.float64)
        u = 0.5 * np.einsum("in,ij,jn->n", X, S, X)
        A = oracle.operator_matrix(n, off, w)
        Au = A @ u
        r = int(np.abs(off).max())
        inner = np.all([(X[c] >= r) & (X[c] < n[c] - r) for c in range(dim)], axis=0)
        assert inner.sum() > 10
        assert np.allclose(Au[inner], -np.trace(Dm @ S), rtol=1e-9, atol=1e-9)


def test_affine_energy_density():
    """Consistency identity (eq. (approxEnergy)): for affine u with gradient
    g, each interior point's energy sum_{e in V(z)} gamma_z(e) <g, e>^2 equals
    <g, D(z) g> exactly (up to rounding)."""
    n = (30, 30)
    D = synth.tensor2d_field(77, n[0], n[1], 20.0)
    off, w, _ = oracle.stencil2d(D)
    g = np.array([0.3, -1.7])
    dens = sum(2 * w[i] * (off[i, 0] * g[0] + off[i, 1] * g[1]) ** 2 for i in range(3))
    want = D[0] * g[0] ** 2 + 2 * D[1] * g[0] * g[1] + D[2] * g[1] ** 2
    assert np.allclose(dens, want, rtol=1e-12, atol=0)


def test_explicit_euler_mass_max_principle_energy():
    """Explicit Euler with dt = 0.9 / max A_zz: mass sum(u) conserved,
    min u0 <= u^n <= max u0 (the discrete maximum principle that the
    non-negative scheme guarantees), and E_h(u^n) non-increasing."""
    for dims, off, w in [_case2d((64, 64), 10.0, 1301), _case3d((12, 12, 12), 50.0, 8)]:
        A = oracle.operator_matrix(dims, off, w)
        dt = 0.9 * oracle.cfl(A)
        u = synth.uniform(11, A.shape[0])
        lo, hi, m0 = u.min(), u.max(), u.sum()
        e_prev = u @ (A @ u)
        for _ in range(20):
            u = oracle.explicit_steps(A, u, dt, 1)
            e = u @ (A @ u)
            assert e <= e_prev * (1 + 1e-12)
            e_prev = e
        assert lo - 1e-12 <= u.min() and u.max() <= hi + 1e-12
        assert abs(u.sum() - m0) <= 1e-10 * abs(m0)


def test_overflow_field_reaches_centre_more_than_255_times():
    """The crafted field of the operator's incoming-list limit test: the
    oracle's stencils of synth.overflow_field3d() put more than 255
    positive-weight edges on the centre (each needle stencil holds the
    primitive vector towards it, Section 2: the stencil of a near
    rank-one tensor contains the lattice direction it is aligned with)."""
    dims, D, c = synth.overflow_field3d()
    off, w, st = oracle.stencil3d(D)
    A = oracle.operator_matrix(dims, off, w)
    assert (A.getrow(c).toarray() != 0).sum() - 1 > 255


# ----------------------------------------------------------------------------
# The reflecting boundary (the restoration test's, Section 4): an edge whose
# target leaves the grid is mirrored back (half-sample mirror, the even
# extension of u).

def test_reflect_operator_is_the_gradient_of_its_energy():
    """A = 1/2 grad E_h with the mirrored targets, read off the energy by
    polarization on tiny grids with offsets longer than the grid is from
    its border (kappa 30 in 2D, 20 in 3D), equals the scattered operator."""
    from oracle import brute
    for dims, D in [((7, 6), synth.tensor2d_field(5, 7, 6, 30.0)),
                    ((5, 4, 4), synth.tensor3d_field(6, (5, 4, 4), 20.0))]:
        off, w, _ = oracle.stencil(D)
        assert np.abs(off).max() >= 3
        n = D.shape[1]
        A = oracle.operator_matrix(dims, off, w, reflect=True).toarray()
        Ad = brute.dense_operator_from_energy(
            lambda v: oracle.energy(dims, off, w, v, reflect=True), n)
        assert np.abs(A - Ad).max() <= 1e-12 * np.abs(Ad).max()
        assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
        assert np.abs(A.sum(1)).max() <= 1e-12 * np.abs(A).max()


def _mirror_field(D, dims):
    """The tensor field on the doubled grid (2 n per axis) that the even
    extension of u sees: D at the mirror image of each point, with the
    off-diagonal entries of every mirrored axis negated (D -> M D M, M the
    reflection)."""
    d = len(dims)
    big = tuple(2 * n for n in dims)
    idx = np.indices(big[::-1]).reshape(d, -1)[::-1]  # x, y[, z]
    src = np.zeros(idx.shape[1], np.int64)
    sgn = np.ones((d, idx.shape[1]))
    stride = 1
    for c in range(d):
        m = idx[c]
        flip = m >= dims[c]
        src += np.where(flip, 2 * dims[c] - 1 - m, m) * stride
        sgn[c] = np.where(flip, -1.0, 1.0)
        stride *= dims[c]
    pairs = [(0, 0), (0, 1), (1, 1)] if d == 2 else \
        [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    return np.stack([D[k][src] * sgn[a] * sgn[b] for k, (a, b) in enumerate(pairs)]), big, src


def test_reflect_operator_equals_periodic_operator_on_the_even_extension():
    """On the doubled grid with the mirrored tensor field and periodic
    wrap, the even extension of u is mapped by the AD-LBR operator to the
    even extension of A_reflect u (the weight function is unique, Lemma 5,
    so the mirrored tensor's stencil is the mirrored stencil).  This ties
    the reflecting mode to the periodic one, which the spectral tests pin."""
    for dims, D in [((12, 10), synth.tensor2d_field(21, 12, 10, 30.0)),
                    ((6, 5, 4), synth.tensor3d_field(22, (6, 5, 4), 20.0))]:
        off, w, _ = oracle.stencil(D)
        A = oracle.operator_matrix(dims, off, w, reflect=True)
        Db, big, src = _mirror_field(D, dims)
        ob, wb, _ = oracle.stencil(Db)
        Ap = oracle.operator_matrix(big, ob, wb, periodic=True)
        u = synth.uniform(3, D.shape[1])
        ub = u[src]
        # the base block of the doubled grid: every coordinate below n
        base = np.ones(src.size, bool)
        idx = np.indices(big[::-1]).reshape(len(dims), -1)[::-1]
        for c in range(len(dims)):
            base &= idx[c] < dims[c]
        got = (Ap @ ub)[base]
        ref = A @ u
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
