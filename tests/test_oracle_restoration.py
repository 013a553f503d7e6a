"""Pins of the restoration test's exact solution and of the discrete
problem the GPU solves for it (Section 4, the synthetic restoration test,
eq. (elliptic)).

- The closed form u = u0 o f solves -lambda div(D grad u) + u = v at every
  point off the stripe's edge: the residual, evaluated by nested central
  differences of the closed form, vanishes to the differences' accuracy.
- The oracle's operator on the n x n grid of spacing h = 1/n, in the system
  (I + lambda h^-2 A) u = v (v averaged over each pixel), has a solution
  that converges to the closed form at least at first order (the paper's
  schemes are first order): halving h divides the L2 error by 1.8 or more.  A wrong scale of A (a factor 2 in
  A = 1/2 grad E_h, or h^-1 instead of h^-2) would converge to the solution
  of another equation and the error would stall.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1301_3925_amd import synth

LAM = 1e-3


@pytest.mark.parametrize("kappa", [2.0, 5.0, 10.0])
def test_closed_form_solves_the_elliptic_equation(kappa):
    alpha = 1.0 / 3.0
    rng = np.random.default_rng(int(kappa))
    x = rng.uniform(0.05, 0.95, 4000)
    y = rng.uniform(0.05, 0.95, 4000)
    t = y + alpha * np.cos(2 * math.pi * x)
    d = 1e-4
    keep = np.abs(t - 0.5) > 4 * d * (1 + 2 * math.pi * alpha)
    x, y = x[keep], y[keep]
    u = lambda a, b: oracle.restoration_exact_at(a, b, kappa, LAM, alpha)
    s = lambda a: 2 * math.pi * alpha * np.sin(2 * math.pi * a)

    def flux(a, b):
        ux = (u(a + d, b) - u(a - d, b)) / (2 * d)
        uy = (u(a, b + d) - u(a, b - d)) / (2 * d)
        return ux + s(a) * uy, s(a) * ux + (s(a) ** 2 + kappa ** -2) * uy

    div = ((flux(x + d, y)[0] - flux(x - d, y)[0]) / (2 * d)
           + (flux(x, y + d)[1] - flux(x, y - d)[1]) / (2 * d))
    v = (y + alpha * np.cos(2 * math.pi * x) < 0.5).astype(float)
    res = -LAM * div + u(x, y) - v
    assert np.abs(res).max() <= 2e-3


def test_oracle_discrete_solution_converges_first_order():
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    kappa = 2.0
    errs = []
    for n in (40, 80, 160):
        D, v = synth.restoration_problem(n, kappa)
        off, w, _ = oracle.stencil2d(D)
        A = oracle.operator_matrix((n, n), off, w)
        K = (sp.identity(n * n) + LAM * n * n * A).tocsc()
        uh = spla.spsolve(K, v)
        errs.append(oracle.restoration_errors(uh, oracle.restoration_exact(n, kappa, LAM), n))
    l2 = [e[0] for e in errs]
    print(errs)
    assert l2[0] / l2[1] > 1.8 and l2[1] / l2[2] > 1.8
    assert l2[2] < 0.002
