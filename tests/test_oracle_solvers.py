"""Pins of the solver and CNN oracle (oracle/solvers.py).

The paper solves its linear systems by conjugate gradients (Section 4,
restoration test); the flexible CG and the learned preconditioner are not in
the paper, so they are pinned by dense solves, textbook identities, a
library convolution and finite differences.
"""
import numpy as np
import pytest

import oracle
from oracle import solvers
from paper_1301_3925_amd import synth


def _system(dims=(16, 12), kappa=20.0, seed=3, mult=50.0):
    D = synth.tensor2d_field(seed, *dims, kappa)
    off, w, _ = oracle.stencil2d(D)
    A = oracle.operator_matrix(dims, off, w)
    dt = mult * oracle.cfl(A)
    return A, dt, solvers.system_matrix(A, dt), off, w


def test_pcg_matches_dense_cholesky():
    """Jacobi-PCG reaches the dense solution of (I + dt A) x = b."""
    import scipy.linalg as sl
    A, dt, K, _, _ = _system()
    b = synth.uniform(1, K.shape[0])
    x, it, rel = solvers.jacobi_pcg(K, b, tol=1e-10)
    xd = sl.cho_solve(sl.cho_factor(K.toarray()), b)
    assert rel <= 1e-10
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_cg_identity_preconditioner_is_textbook_cg():
    """With P = I the iterates are those of plain CG, which on a matrix
    with m distinct eigenvalues terminates in m steps (here m = 3)."""
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    lam = np.repeat([1.0, 4.0, 9.0], 10)
    import scipy.sparse as sp
    K = sp.csr_matrix(Q @ np.diag(lam) @ Q.T)
    b = rng.normal(size=30)
    x, it, rel = solvers.jacobi_pcg(K, b, tol=1e-10, precond=False)
    assert it <= 4 and rel <= 1e-10


def test_fcg_with_fixed_linear_preconditioner_equals_pcg():
    """Flexible CG with the fixed SPD preconditioner diag(K)^-1 produces the
    PCG iterates (same residual history to rounding)."""
    A, dt, K, _, _ = _system()
    b = synth.uniform(2, K.shape[0])
    inv = 1.0 / K.diagonal()
    _, it1, _, h1 = solvers.jacobi_pcg(K, b, tol=1e-8, history=True)
    _, it2, _, fb, h2 = solvers.fcg(K, b, lambda r: inv * r, tol=1e-8, history=True)
    assert not fb and it1 == it2
    assert np.allclose(h1, h2, rtol=1e-6, atol=1e-14)


def test_pcg_iterations_within_condition_bound():
    """CG error bound: iterations <= ceil(sqrt(cond)/2 ln(2/tol)) for the
    Jacobi-preconditioned system."""
    A, dt, K, _, _ = _system((24, 24), 50.0, 4)
    b = synth.uniform(3, K.shape[0])
    d = 1.0 / np.sqrt(K.diagonal())
    M = (K.toarray() * d[:, None]) * d[None, :]
    ev = np.linalg.eigvalsh(M)
    cond = ev[-1] / ev[0]
    bound = np.ceil(np.sqrt(cond) / 2 * np.log(2 / 1e-6)) + 5
    _, it, rel = solvers.jacobi_pcg(K, b, tol=1e-6)
    assert rel <= 1e-6 and it <= bound


def test_fcg_falls_back_on_bad_preconditioner():
    """A preconditioner that returns -r (not a descent direction) makes FCG
    restart with Jacobi-PCG, which still converges."""
    A, dt, K, _, _ = _system()
    b = synth.uniform(4, K.shape[0])
    x, it, rel, fb = solvers.fcg(K, b, lambda r: -r, tol=1e-6)
    assert fb and rel <= 1e-6


def test_fcg_falls_back_on_stall():
    """A preconditioner that is SPD but nearly ignores all but eight unknowns
    (<z, r> > 0 throughout, next to no progress) trips the stall rule;
    Jacobi-PCG then converges from where FCG stopped."""
    A, dt, K, _, _ = _system()
    n = K.shape[0]
    b = synth.uniform(5, n)
    m = np.full(n, 1e-9)
    m[:: n // 8][:8] = 1.0

    x, it, rel, fb, h = solvers.fcg(K, b, lambda r: m * r, tol=1e-6, history=True)
    assert fb and rel <= 1e-6
    assert len(h) == 21  # the stall is detected after exactly 20 iterations
    assert min(h[1:]) > 0.99 * h[0]
    _, itj, _ = solvers.jacobi_pcg(K, b, tol=1e-6)
    assert it >= 20 + itj - 5


@pytest.mark.parametrize("dim", [2, 3])
def test_conv_matches_library_correlation(dim):
    """A single-channel layer equals scipy's zero-padded correlation."""
    from scipy.ndimage import correlate
    rng = np.random.default_rng(dim)
    shp = (9, 7) if dim == 2 else (6, 5, 4)
    x = rng.normal(size=(1,) + shp)
    W = rng.normal(size=(1, 1) + (3,) * dim)
    out = solvers.conv(x, W, np.array([0.25]))[0]
    ref = correlate(x[0], W[0, 0], mode="constant", cval=0.0) + 0.25
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13)


def _net_case(dim):
    dims = (16, 12) if dim == 2 else (8, 7, 6)
    D = synth.tensor2d_field(5, *dims, 30.0) if dim == 2 else synth.tensor3d_field(6, dims, 20.0)
    off, w, _ = oracle.stencil(D)
    A = oracle.operator_matrix(dims, off, w)
    dt = 50 * oracle.cfl(A)
    F = solvers.net_features(dims, off, w, A.diagonal(), dt)
    width = 16 if dim == 2 else 4
    P = solvers.net_init(3, dim, width=width, hidden=8)
    return dims, A, dt, F, P, width


@pytest.mark.parametrize("dim", [2, 3])
def test_net_backward_matches_finite_differences(dim):
    """Chain-rule gradients of sum(gz * z) w.r.t. every parameter (r path,
    gates, gate net) equal central differences (eps = 1e-6)."""
    dims, A, dt, F, P, width = _net_case(dim)
    rng = np.random.default_rng(11)
    n = int(np.prod(dims))
    r = rng.normal(size=n)
    gz = rng.normal(size=n)
    kd = 1 + dt * A.diagonal()
    grads = solvers.net_backward(P, F, r, gz)

    def f(Q):
        return float(gz @ solvers.net_precondition(Q, solvers.net_gates(Q, F), r, kd))

    for name, _ in solvers.net_shapes(dim, width, 8):
        Wt = P[name]
        for _ in range(3):
            idx = tuple(int(rng.integers(0, k)) for k in Wt.shape)
            h = 1e-6 * max(1.0, abs(Wt[idx]))
            Qp = {k: v.copy() for k, v in P.items()}
            Qm = {k: v.copy() for k, v in P.items()}
            Qp[name][idx] += h
            Qm[name][idx] -= h
            fd = (f(Qp) - f(Qm)) / (2 * h)
            assert abs(fd - grads[name][idx]) <= 1e-5 * max(1.0, abs(fd)), (name, idx)


def test_net_is_linear_in_r_and_reduces_to_jacobi():
    """N is linear in r (gates do not depend on r); with W1 = 0 the
    preconditioner is Jacobi and flexible CG reproduces Jacobi-PCG."""
    dims, A, dt, F, P, _ = _net_case(2)
    rng = np.random.default_rng(2)
    n = int(np.prod(dims))
    kd = 1 + dt * A.diagonal()
    G = solvers.net_gates(P, F)
    r1, r2 = rng.normal(size=n), rng.normal(size=n)
    z = lambda r: solvers.net_precondition(P, G, r, kd)
    assert np.allclose(z(2 * r1 - 3 * r2), 2 * z(r1) - 3 * z(r2), rtol=1e-10, atol=1e-12)
    P0 = dict(P)
    P0["W1"] = np.zeros_like(P["W1"])
    G0 = solvers.net_gates(P0, F)
    assert np.allclose(solvers.net_precondition(P0, G0, r1, kd), r1 / kd, rtol=0, atol=0)
    K = solvers.system_matrix(A, dt)
    b = synth.uniform(4, n)
    _, it1, _ = solvers.jacobi_pcg(K, b, tol=1e-8)
    _, it2, _, fb = solvers.fcg(K, b, lambda r: solvers.net_precondition(P0, G0, r, kd), tol=1e-8)
    assert not fb and it1 == it2


@pytest.mark.parametrize("dim", [2, 3])
def test_conv_adjoint_identity(dim):
    """<conv(x, W), y> = <x, conv_adjoint(y, W)> for random multi-channel
    x, y, W (zero padding on both sides)."""
    rng = np.random.default_rng(20 + dim)
    shp = (7, 6) if dim == 2 else (5, 4, 6)
    x = rng.normal(size=(3,) + shp)
    y = rng.normal(size=(4,) + shp)
    W = rng.normal(size=(4, 3) + (3,) * dim)
    lhs = float(np.sum(solvers.conv(x, W, np.zeros(4)) * y))
    rhs = float(np.sum(x * solvers.conv_adjoint(y, W)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("dim", [2, 3])
def test_net_preconditioner_is_spd(dim):
    """The dense matrix of r -> N(r) (columns from unit vectors) is
    symmetric and positive semi-definite, so diag(K)^-1 + N is SPD and
    <z, r> >= <r / diag K, r> for every r."""
    dims, A, dt, F, P, _ = _net_case(dim)
    n = int(np.prod(dims))
    G = solvers.net_gates(P, F)
    shp = G.shape[1:]
    M = np.stack([solvers.net_apply(P, G, e, shp).reshape(-1) for e in np.eye(n)], axis=1)
    scale = np.abs(M).max()
    assert scale > 0
    assert np.abs(M - M.T).max() <= 1e-12 * scale
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() >= -1e-12 * scale
    kd = 1 + dt * A.diagonal()
    r = np.random.default_rng(3).normal(size=n)
    assert solvers.net_precondition(P, G, r, kd) @ r >= (r / kd) @ r


def test_net_pack_roundtrip():
    P = solvers.net_init(1, 3, width=16, hidden=16)
    flat = solvers.net_pack(P, 3)
    Q = solvers.net_unpack(flat, 3)
    assert all(np.array_equal(P[k], Q[k]) for k in P)
    T = 27
    assert flat.size == 16 * 13 * T + 16 + 32 * 16 + 32 + 16 * T + 16 * 16 * T


def test_energy_loss_minimum_and_gradient():
    """The energy loss is minimal at z = K^-1 r, with gradient (Kz - r)/r.r."""
    A, dt, K, _, _ = _system((10, 9))
    r = synth.uniform(5, K.shape[0]) - 0.5
    zs = np.linalg.solve(K.toarray(), r)
    l0, g0 = solvers.energy_loss(K, zs, r)
    assert np.linalg.norm(g0) <= 1e-12
    rng = np.random.default_rng(1)
    for _ in range(3):
        dz = 1e-3 * rng.normal(size=r.size)
        assert solvers.energy_loss(K, zs + dz, r)[0] > l0
    z = rng.normal(size=r.size)
    l, g = solvers.energy_loss(K, z, r)
    e = rng.normal(size=r.size)
    h = 1e-6
    fd = (solvers.energy_loss(K, z + h * e, r)[0] - solvers.energy_loss(K, z - h * e, r)[0]) / (2 * h)
    assert abs(fd - g @ e) <= 1e-6 * max(1.0, abs(fd))
