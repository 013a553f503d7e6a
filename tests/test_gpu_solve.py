"""GPU parity of the implicit solvers against the FP64 oracle.

Jacobi-PCG on K = I + dt A (dt = 50 / max A_zz): with FP64 storage the
residual history follows the oracle's to rounding; with FP32 storage the
solution matches the oracle's to the FP32 tolerance and the iteration count
to within 2.
"""
import numpy as np
import pytest

import oracle
from oracle import solvers
from paper_1301_3925_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_1301_3925_amd as adlbr
    assert torch.cuda.is_available()
    return adlbr


def _problem(lib, dims, kappa, seed, storage):
    import torch
    D = synth.tensor2d_field(seed, *dims, kappa) if len(dims) == 2 else \
        synth.tensor3d_field(seed, dims, kappa)
    off, w, st = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=storage)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy())
    dt = 50.0 * oracle.cfl(A)
    return op, A, dt


@pytest.mark.parametrize("dims,kappa", [((96, 80), 200.0), ((20, 18, 16), 50.0)])
def test_jacobi_pcg_fp64_matches_oracle(lib, dims, kappa):
    import torch
    op, A, dt = _problem(lib, dims, kappa, 1305, torch.float64)
    K = solvers.system_matrix(A, dt)
    b = synth.uniform(7, op.N)
    xr, itr, relr = solvers.jacobi_pcg(K, b, tol=1e-6)
    x, rep = op.solve(torch.from_numpy(b).cuda(), dt, tol=1e-6, check_every=7)
    assert rep["converged"] == 1 and rep["rel_res"] <= 1e-6, rep
    assert abs(rep["iters"] - itr) <= 1, (rep, itr)
    xs = np.linalg.solve(K.toarray(), b) if op.N <= 8000 else xr
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-5 * np.linalg.norm(xs)


def test_jacobi_pcg_fp32(lib):
    import torch
    dims = (128, 96)
    op, A, dt = _problem(lib, dims, 200.0, 11, torch.float32)
    K = solvers.system_matrix(A, dt)
    b = synth.uniform(8, op.N)
    xr, itr, _ = solvers.jacobi_pcg(K, b, tol=1e-7)
    x, rep = op.solve(torch.from_numpy(b).float().cuda(), dt, tol=1e-6)
    assert rep["converged"] == 1 and rep["rel_res"] <= 1e-6
    _, it6, _ = solvers.jacobi_pcg(K, b, tol=1e-6)
    assert abs(rep["iters"] - it6) <= 2
    assert np.linalg.norm(x.double().cpu().numpy() - xr) <= 3e-6 * np.linalg.norm(xr)


def test_initial_guess_and_not_converged(lib):
    import torch
    dims = (64, 64)
    op, A, dt = _problem(lib, dims, 50.0, 12, torch.float64)
    K = solvers.system_matrix(A, dt)
    b = synth.uniform(9, op.N)
    x, rep = op.solve(torch.from_numpy(b).cuda(), dt, tol=1e-6, max_iter=2, check_every=1)
    assert rep["converged"] == 0 and rep["iters"] == 2 and rep["rel_res"] > 1e-6
    # continue from that iterate: the initial guess is used
    x2, rep2 = op.solve(torch.from_numpy(b).cuda(), dt, tol=1e-6, x=x.clone())
    assert rep2["converged"] == 1
    xr = solvers.jacobi_pcg(K, b, tol=1e-9)[0]
    assert np.linalg.norm(x2.cpu().numpy() - xr) <= 1e-5 * np.linalg.norm(xr)


def test_solve_deterministic(lib):
    import torch
    dims = (200, 150)
    op, A, dt = _problem(lib, dims, 100.0, 13, torch.float32)
    b = torch.from_numpy(synth.uniform(10, op.N)).float().cuda()
    x1, r1 = op.solve(b, dt)
    x2, r2 = op.solve(b, dt)
    assert torch.equal(x1, x2) and r1["iters"] == r2["iters"]
