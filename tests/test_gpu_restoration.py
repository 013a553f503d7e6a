"""The restoration test on the GPU (Section 4, the synthetic test with an
analytic solution, eq. (elliptic)): -lambda div(D grad u) + u = v on the
unit square with lambda = 1e-3, discretized as (I + lambda h^-2 A) u = v on
N x N pixels (h = 1/N), A the AD-LBR operator of the library, solved by the
library's Jacobi-PCG in FP64 to a true relative residual of 1e-10.

- At N = 100 and 200 the GPU solution equals the oracle's (its own stencils,
  operator and a sparse direct solve) to 1e-8.
- For kappa = 2, 5, 10 and N = 100 ... 1200 the L2 and H1 errors against
  the closed form fall at least at first order, the paper's expectation:
  the least-squares slope of log error against log N is <= -1 (L2) and
  <= -0.7 (H1; at kappa = 10 the layer of width sqrt(lambda)/kappa = 0.003
  is resolved only from N ~ 300 on, so the first sizes are pre-asymptotic).
"""
import numpy as np
import pytest

import oracle
from paper_1301_3925_amd import synth

pytestmark = pytest.mark.gpu

LAM = 1e-3
SIZES = (100, 200, 400, 800, 1200)


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_1301_3925_amd as adlbr
    assert torch.cuda.is_available()
    return adlbr


@pytest.mark.parametrize("kappa", [2.0, 5.0, 10.0])
def test_restoration_converges_to_the_analytic_solution(lib, kappa):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    import torch
    errs, iters = [], []
    for n in SIZES:
        D, v = synth.restoration_problem(n, kappa)
        off, w, st = lib.build_stencils(torch.from_numpy(D).cuda(), (n, n))
        assert lib.status_flags(st) & ~lib.capi.ST_CLAMPED == 0
        op = lib.Operator((n, n), off, w, storage=torch.float64)
        x, rep = op.solve(torch.from_numpy(v).cuda(), LAM * n * n, tol=1e-10, max_iter=20000)
        assert rep["converged"] == 1 and rep["rel_res"] <= 1e-10, rep
        iters.append(rep["iters"])
        uh = x.cpu().numpy()
        if n <= 200:
            ro, rw, _ = oracle.stencil2d(D)
            assert np.array_equal(off.cpu().numpy(), ro)
            A = oracle.operator_matrix((n, n), ro, rw)
            uo = spla.spsolve((sp.identity(n * n) + LAM * n * n * A).tocsc(), v)
            assert np.linalg.norm(uh - uo) <= 1e-8 * np.linalg.norm(uo)
        errs.append(oracle.restoration_errors(uh, oracle.restoration_exact(n, kappa, LAM), n))
    e = np.array(errs)
    lg = np.log(np.array(SIZES, dtype=float))
    s_l2 = np.polyfit(lg, np.log(e[:, 0]), 1)[0]
    s_h1 = np.polyfit(lg, np.log(e[:, 1]), 1)[0]
    print(f"kappa {kappa}: L2 {e[:, 0]} H1 {e[:, 1]} slopes {s_l2:.2f} {s_h1:.2f} iters {iters}")
    assert s_l2 <= -1.0 and s_h1 <= -0.7
    assert e[-1, 0] < e[0, 0] / 5
