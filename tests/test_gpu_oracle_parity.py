"""GPU paths compared directly with the FP64 oracle where earlier tests
compared them only with another GPU path:

- the BF16 MFMA inference of the learned preconditioner (2D fused kernel,
  3D layer kernels) element by element against the oracle's exact
  preconditioner, on grids that do not divide into the 16 x 16 / 8 x 8 x 4
  tiles;
- flexible CG's iteration counts against the oracle's flexible CG, with a
  fixed Jacobi preconditioner (N = 0) and with the untrained network;
- 3D BF16/FP16 storage (its entry weights live in an array of their own)
  against the oracle, on grids that take the strip traversal;
- the storage variants' errors after 50/100/150/200 steps against the
  oracle on a volume of the 256^3 recipe's kind;
- a crafted field where more than 255 stencils reach one point: the
  operator reports it, and every other row is still exact.
"""
import math

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


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _net_case(lib, dims, kappa, seed, W1_zero=False):
    import torch
    D = (synth.tensor2d_field(seed, *dims, kappa) if len(dims) == 2
         else synth.tensor3d_field(seed, dims, kappa))
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=torch.float32)
    o = off.cpu().numpy()
    w32 = w.float().double().cpu().numpy()
    A = oracle.operator_matrix(dims, o, w32)
    dt = 50.0 * oracle.cfl(A)
    dim = len(dims)
    P = solvers.net_init(seed + 1, dim)
    if W1_zero:
        P["W1"][:] = 0.0
    flat = solvers.net_pack(P, dim)
    net = lib.Net(op, params=torch.from_numpy(flat).float())
    net.prepare(dt)
    P32 = solvers.net_unpack(flat.astype(np.float32).astype(np.float64), dim)
    kd = 1.0 + dt * A.diagonal()
    F = solvers.net_features(dims, o, w32, A.diagonal(), dt)
    G = solvers.net_gates(P32, F)
    return op, A, dt, net, P32, G, kd


# BF16 bound of the MFMA inference.  N(r) = C1^T g1 C2^T g2 C2 g1 C1 r is
# four correlations; on the MFMA path each product's two operands are
# rounded to BF16 (unit roundoff 2^-9 each) and each layer's FP32 sum is
# rounded to BF16 once more, and the gates are 8-bit, |g8 - g| <= 1/510.
# Summed over the four layers the error of every element is then at most
# about 4 x 3 x 2^-9 = 0.023 of the same network run with |W| and |r|
# (gates raised by 1/510), element by element: the standard forward bound
# for sums of products.  The test allows 0.03 of that.
TAU_BF16 = 0.03


@pytest.mark.parametrize("dims", [(100, 75), (37, 29), (21, 18, 13), (9, 10, 7)])
def test_mfma_inference_matches_oracle(lib, dims):
    import torch
    op, A, dt, net, P, G, kd = _net_case(lib, dims, 100.0 if len(dims) == 2 else 50.0, 9)
    r = (synth.uniform(4, op.N) - 0.5).astype(np.float32).astype(np.float64)
    z = net.precondition(torch.from_numpy(r).float().cuda()).double().cpu().numpy()
    zr = solvers.net_precondition(P, G, r, kd)
    n_gpu = z - r / kd
    n_ref = zr - r / kd
    Pa = {k: np.abs(v) for k, v in P.items()}
    S = solvers.net_apply(Pa, np.minimum(G + 1.0 / 510, 1.0), np.abs(r), G.shape[1:]).reshape(-1)
    ratio = np.abs(n_gpu - n_ref) / np.maximum(S, 1e-30)
    print("max |dN| / |N|abs:", ratio.max(), "rel-L2 of N:", _rel(n_gpu, n_ref))
    assert np.all(np.abs(n_gpu - n_ref) <= TAU_BF16 * S + 1e-7 * np.abs(r / kd))
    assert _rel(z, zr) <= 1e-2


@pytest.mark.parametrize("dims", [(96, 80), (20, 18, 16)])
def test_fcg_jacobi_net_iterations_match_oracle(lib, dims):
    """With W1 = 0 the network adds nothing (N = 0), so flexible CG runs
    with the fixed preconditioner diag(K)^-1: its iteration count equals
    the oracle's flexible CG (truncation 1) with that preconditioner to
    within one, and its solution the oracle's."""
    import torch
    op, A, dt, net, P, G, kd = _net_case(lib, dims, 200.0 if len(dims) == 2 else 50.0, 21,
                                         W1_zero=True)
    K = solvers.system_matrix(A, dt)
    b = synth.uniform(6, op.N).astype(np.float32).astype(np.float64)
    x, rep = op.solve(torch.from_numpy(b).float().cuda(), dt, method="fcg", net=net, tol=1e-6,
                      check_every=1)
    xr, itr, relr, fb = solvers.fcg(K, b, lambda r: r / kd, tol=1e-6)
    print("gpu", rep["iters"], "oracle", itr)
    assert rep["converged"] == 1 and rep["fell_back"] == 0 and not fb
    assert rep["net_iters"] == rep["iters"]
    assert abs(rep["iters"] - itr) <= 1
    assert _rel(x.double().cpu().numpy(), xr) <= 3e-6


@pytest.mark.parametrize("dims", [(96, 80), (20, 18, 16)])
def test_fcg_untrained_net_iterations_near_oracle(lib, dims):
    """Flexible CG with the untrained network: the GPU runs the BF16 MFMA
    inference, the oracle the exact preconditioner.  The two
    preconditioners differ by the BF16 bound above, so the iteration counts
    agree to within 10% (at least 2)."""
    import torch
    op, A, dt, net, P, G, kd = _net_case(lib, dims, 200.0 if len(dims) == 2 else 50.0, 22)
    K = solvers.system_matrix(A, dt)
    b = synth.uniform(7, op.N).astype(np.float32).astype(np.float64)
    x, rep = op.solve(torch.from_numpy(b).float().cuda(), dt, method="fcg", net=net, tol=1e-6,
                      check_every=1)
    xr, itr, relr, fb = solvers.fcg(K, b, lambda r: solvers.net_precondition(P, G, r, kd),
                                    tol=1e-6)
    print("gpu", rep["iters"], "oracle", itr)
    assert rep["converged"] == 1 and rep["fell_back"] == 0 and not fb
    assert rep["net_iters"] == rep["iters"] > 0
    assert abs(rep["iters"] - itr) <= max(2, math.ceil(0.1 * itr))
    assert _rel(x.double().cpu().numpy(), xr) <= 3e-6


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("dims", [(32, 16, 13), (24, 20, 18)])
def test_3d_16bit_storage_vs_oracle(lib, storage, dims):
    """3D u and weights in BF16/FP16 with FP32 arithmetic, 20 steps at 0.9
    of the CFL bound, against the FP64 oracle started from the same rounded
    u0: within 8 unit roundoffs (2^-8 BF16, 2^-11 FP16), mass to 4."""
    import torch
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[storage]
    eps = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}[storage]
    D = synth.tensor3d_field(15, dims, 50.0)
    off, w, st = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=tdt)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy())
    ug = torch.from_numpy(synth.uniform(2, op.N)).to(tdt).cuda()
    u0q = ug.double().cpu().numpy()
    ref = oracle.explicit_steps(A, u0q, 0.9 * oracle.cfl(A), 20)
    op.step(ug, 0.9, 20, cfl_fraction=True)
    got = ug.double().cpu().numpy()
    assert _rel(got, ref) <= 8 * eps
    assert abs(got.sum() - u0q.sum()) <= 4 * eps * abs(u0q.sum())


def test_storage_variants_errors_vs_oracle_over_200_steps(lib):
    """The precision workload's question on a 64^3 volume of the same
    recipe (kappa <= 50): 200 explicit steps in FP64, FP32, BF16 and FP16
    storage, relative L2 error against the FP64 oracle after 50, 100, 150
    and 200 steps.  Bound: every stored u and weight is rounded with
    relative error <= eps/2, and I - dt A is non-expansive in the maximum
    norm, so the error grows at most linearly, n eps/2 per point for u plus
    the weights' share, below n eps in all (eps = 2^-52, 2^-23, 2^-8,
    2^-11).  FP64 and FP32 meet the tolerances of the explicit scheme's
    parity tests (1e-12, 1e-5)."""
    import torch
    dims = (64, 64, 64)
    D = synth.tensor3d_field(1303, dims, 50.0)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy())
    dt = 0.9 * oracle.cfl(A)
    u0 = synth.uniform(1304, int(np.prod(dims)))
    eps = {"f64": 2.0 ** -52, "f32": 2.0 ** -23, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
    tol = {"f64": 1e-12, "f32": 1e-5}
    dts = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
           "f16": torch.float16}
    errs = {}
    for name, tdt in dts.items():
        op = lib.Operator(dims, off, w, storage=tdt)
        ug = torch.from_numpy(u0).to(tdt).cuda()
        ref = ug.double().cpu().numpy()
        errs[name] = []
        for n in (50, 100, 150, 200):
            ref = oracle.explicit_steps(A, ref, dt, 50)
            op.step(ug, 0.9, 50, cfl_fraction=True)
            e = _rel(ug.double().cpu().numpy(), ref)
            errs[name].append(e)
            assert e <= n * eps[name], (name, n, e)
            if name in tol:
                assert e <= tol[name], (name, n, e)
    print(errs)


def test_incoming_overflow_is_reported_and_other_rows_exact(lib):
    """More than 255 stencils reach the centre (the oracle count is
    pinned on the CPU in test_oracle_operator.py): the operator sets ADLBR_ST_INCOMING, the
    checked constructor raises, and with the check off the apply still
    reads only valid entries -- every row but the centre's equals the
    oracle's to FP64 rounding, including the last row of the centre's bin
    of 1024 targets, whose list holds the padding after the clamped rows."""
    import torch
    dims, D, c = synth.overflow_field3d()
    off, w, st = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    with pytest.raises(lib.AdlbrError):
        lib.Operator(dims, off, w, storage=torch.float64)
    op = lib.Operator(dims, off, w, storage=torch.float64, check=False)
    s = op.status.cpu().numpy()
    assert s[1] & lib.capi.ST_INCOMING and 0 <= s[0] <= c
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy())
    u = synth.uniform(3, op.N)
    Au = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    ref = A @ u
    keep = np.ones(op.N, bool)
    keep[c] = False
    assert np.all(np.isfinite(Au))
    assert _rel(Au[keep], ref[keep]) <= 1e-12
    last = ((c >> 10) << 10) + 1023
    assert abs(Au[last] - ref[last]) <= 1e-12 * max(1.0, abs(ref[last]))
