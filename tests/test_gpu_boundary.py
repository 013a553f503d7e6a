"""Boundary modes on the GPU against the FP64 oracle, and the spectral
correctness of the GPU operator.

- ADLBR_REFLECT (targets mirrored back into the grid, the reflecting
  boundary of the restoration test, Section 4): apply, diagonal and CFL
  bound against the oracle's reflecting operator (FP64 1e-12, FP32 1e-5) on
  grids whose offsets reach several points past the border, 2D and 3D;
  explicit steps; batches (bit-identical to single steps); the restoration
  test itself with this boundary.
- Spectral correctness (Section 1, and the figure on the seven smallest
  eigenvalues): the seven smallest eigenvalues of h^-2 A for the tensor
  [[19/2, 6], [6, 4]] on the periodic unit square, computed from the GPU
  operator alone (shift-invert Lanczos whose every product is a GPU solve
  with K = I + dt A), equal the oracle's and converge to 4 pi^2 <k, D k>.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1301_3925_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_1301_3925_amd as adlbr
    assert torch.cuda.is_available()
    return adlbr


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


REFLECT_CASES = [
    ("2d-reach", (97, 61), lambda: synth.tensor2d_field(11, 97, 61, 50.0)),
    ("2d-thin", (3, 500), lambda: synth.tensor2d_field(17, 3, 500, 20.0)),
    ("3d", (20, 17, 13), lambda: synth.tensor3d_field(13, (20, 17, 13), 50.0)),
    ("3d-strips", (32, 16, 13), lambda: synth.tensor3d_field(15, (32, 16, 13), 50.0)),
]


@pytest.mark.parametrize("name,dims,mk", REFLECT_CASES, ids=[c[0] for c in REFLECT_CASES])
def test_reflect_apply(lib, name, dims, mk):
    import torch
    D = mk()
    off, w, st = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    on, wn = off.cpu().numpy(), w.cpu().numpy()
    A = oracle.operator_matrix(dims, on, wn, reflect=True)
    An = oracle.operator_matrix(dims, on, wn)
    assert abs(A - An).max() > 0  # the border differs from the truncation
    op = lib.Operator(dims, off, w, storage=torch.float64, reflect=True)
    u = synth.uniform(5, op.N)
    assert _rel(op.apply(torch.from_numpy(u).cuda()).cpu().numpy(), A @ u) <= 1e-12
    assert np.allclose(op.diagonal().cpu().numpy(), A.diagonal(), rtol=1e-13, atol=1e-15)
    assert abs(op.dt_cfl() - oracle.cfl(A)) <= 1e-14 * oracle.cfl(A)
    op32 = lib.Operator(dims, off, w, storage=torch.float32, reflect=True)
    ug = torch.from_numpy(u).float().cuda()
    assert _rel(op32.apply(ug).double().cpu().numpy(), A @ ug.double().cpu().numpy()) <= 1e-5


def test_reflect_steps_and_batch(lib):
    """50 FP64 steps against the oracle; a batch of reflecting, Neumann and
    periodic problems is bit-identical to stepping each alone."""
    import torch
    dims = (64, 48)
    D = synth.tensor2d_field(1301, *dims, 10.0)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy(), reflect=True)
    op = lib.Operator(dims, off, w, storage=torch.float64, reflect=True)
    u0 = synth.uniform(9, op.N)
    u = torch.from_numpy(u0).cuda()
    op.step(u, 0.9, 50, cfl_fraction=True)
    assert _rel(u.cpu().numpy(), oracle.explicit_steps(A, u0, 0.9 * oracle.cfl(A), 50)) <= 1e-12
    ops = [op, lib.Operator(dims, off, w, storage=torch.float64),
           lib.Operator(dims, off, w, storage=torch.float64, periodic=True)]
    D3 = synth.tensor3d_field(4, (12, 11, 9), 20.0)
    o3, w3, _ = lib.build_stencils(torch.from_numpy(D3).cuda(), (12, 11, 9))
    ops.append(lib.Operator((12, 11, 9), o3, w3, storage=torch.float64, reflect=True))
    us = [torch.from_numpy(synth.uniform(20 + k, o.N)).cuda() for k, o in enumerate(ops)]
    ref = [x.clone() for x in us]
    for o, x in zip(ops, ref):
        o.step(x, 0.9, 5, cfl_fraction=True)
    b = lib.Batch(ops, us, dt=0.9, dt_mode="cfl")
    b.run(5)
    torch.cuda.synchronize()
    for k, (x, r) in enumerate(zip(us, ref)):
        assert torch.equal(x, r), k


def test_restoration_with_reflecting_boundary(lib):
    """The restoration test as the paper ran it, with reflecting boundary
    conditions: the GPU solution equals the oracle's at N = 100 and the
    error against the closed form falls at least at first order."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    import torch
    lam, kappa = 1e-3, 5.0
    errs, sizes = [], (100, 200, 400, 800)
    for n in sizes:
        D, v = synth.restoration_problem(n, kappa)
        off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), (n, n))
        op = lib.Operator((n, n), off, w, storage=torch.float64, reflect=True)
        x, rep = op.solve(torch.from_numpy(v).cuda(), lam * n * n, tol=1e-10, max_iter=20000)
        assert rep["converged"] == 1
        uh = x.cpu().numpy()
        if n == 100:
            A = oracle.operator_matrix((n, n), off.cpu().numpy(), w.cpu().numpy(), reflect=True)
            uo = spla.spsolve((sp.identity(n * n) + lam * n * n * A).tocsc(), v)
            assert np.linalg.norm(uh - uo) <= 1e-8 * np.linalg.norm(uo)
        errs.append(oracle.restoration_errors(uh, oracle.restoration_exact(n, kappa, lam), n))
    e = np.array(errs)
    slope = np.polyfit(np.log(sizes), np.log(e[:, 0]), 1)[0]
    print("reflect restoration L2", e[:, 0], "H1", e[:, 1], "slope", slope)
    assert slope <= -1.0


def _gpu_smallest_eigenvalues(lib, n, k=7):
    """The k smallest eigenvalues of h^-2 A (h = 1/n, periodic) from the GPU
    operator: the largest eigenvalues mu of K^-1, K = I + dt A, by Lanczos
    (scipy's eigsh: host arithmetic on vectors only) with every product
    K^-1 v a GPU Jacobi-PCG solve; lambda = (1/mu - 1) / dt * n^2."""
    import torch
    from scipy.sparse.linalg import LinearOperator, eigsh
    D = np.repeat(np.array([[9.5], [6.0], [4.0]]), n * n, axis=1)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), (n, n), periodic=True)
    op = lib.Operator((n, n), off, w, storage=torch.float64, periodic=True)
    dt = n * n / (4 * math.pi ** 2 * 2.0)

    def mv(v):
        b = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64).reshape(-1)).cuda()
        x, rep = op.solve(b, dt, tol=1e-13, max_iter=50000)
        assert rep["converged"] == 1
        return x.cpu().numpy()

    Kinv = LinearOperator((n * n, n * n), matvec=mv, dtype=np.float64)
    mu = eigsh(Kinv, k=k + 1, which="LA", tol=1e-12, ncv=40,
               v0=synth.uniform(3, n * n), return_eigenvectors=False)
    lam = np.sort((1.0 / mu - 1.0) / dt * n * n)[:k]
    return lam, off.cpu().numpy(), w.cpu().numpy()


def test_spectral_convergence_on_the_gpu(lib):
    D0 = np.array([[9.5, 6.0], [6.0, 4.0]])
    ks = [(a, b) for a in range(-4, 5) for b in range(-4, 5)]
    cont = np.sort([4 * math.pi ** 2 * np.array(k) @ D0 @ np.array(k) for k in ks])[:7]
    errs = []
    for n in (16, 32, 64, 128):
        ev, off, w = _gpu_smallest_eigenvalues(lib, n)
        if n <= 32:
            A = oracle.operator_matrix((n, n), off, w, periodic=True).toarray() * n * n
            ref = np.sort(np.linalg.eigvalsh(A))[:7]
            assert np.max(np.abs(ev - ref) / np.maximum(ref, 1.0)) <= 1e-8
        errs.append(np.max(np.abs(ev - cont) / np.maximum(cont, 1.0)))
    print("spectral errors n = 16, 32, 64, 128:", errs)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.01
