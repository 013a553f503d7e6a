"""GPU parity of the learned preconditioner's kernels against the FP64 oracle.

The GPU runs N = B^T diag(g2) B as an expanded four-layer stack with tied
weights; the oracle applies B and its adjoint directly, so agreement checks
the expansion and the gradient folding as well.

Forward, gates and features at FP32 tolerance (1e-5 relative L2); backward
(all parameter gradients through the r path, the gates and the gate net) at
1e-4; Adam against torch.optim.Adam on the CPU.
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


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _case(lib, dim, dims=None):
    import torch
    dims = dims or ((40, 32) if dim == 2 else (10, 9, 8))
    D = synth.tensor2d_field(3, *dims, 50.0) if dim == 2 else synth.tensor3d_field(4, dims, 20.0)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=torch.float32)
    w32 = w.float().double().cpu().numpy()
    o = off.cpu().numpy()
    A = oracle.operator_matrix(dims, o, w32)
    dt = 50.0 * oracle.cfl(A)
    P = solvers.net_init(5, dim)
    flat = solvers.net_pack(P, dim)
    net = lib.Net(op, params=torch.from_numpy(flat).float())
    net.prepare(dt)
    diag = op.diagonal().cpu().numpy()
    P32 = solvers.net_unpack(flat.astype(np.float32).astype(np.float64), dim)
    F = solvers.net_features(dims, o, w32, diag, dt)
    return dims, op, A, dt, net, P32, F, diag


@pytest.mark.parametrize("dim", [2, 3])
def test_features_gates_forward(lib, dim):
    import torch
    dims, op, A, dt, net, P, F, diag = _case(lib, dim)
    assert _rel(net.features.cpu().numpy(), F.reshape(F.shape[0], -1)) <= 1e-6
    G = solvers.net_gates(P, F)
    gx = net.gates.cpu().numpy()
    assert _rel(gx[:32], G.reshape(G.shape[0], -1)) <= 1e-5
    # the four-layer stack's gates are [g1, g2, g1, 1]
    assert np.array_equal(gx[32:48], gx[:16]) and np.all(gx[48] == 1.0)
    r = synth.uniform(3, op.N) - 0.5
    z = net.forward(torch.from_numpy(r).float().cuda()).double().cpu().numpy()
    kd = 1.0 + dt * diag
    zr = solvers.net_precondition(P, G, r.astype(np.float32).astype(np.float64), kd)
    assert _rel(z, zr) <= 1e-5


@pytest.mark.parametrize("dim,dims", [(2, None), (3, None), (3, (19, 17, 9))],
                         ids=["2d", "3d", "3d-tiles"])
def test_backward_all_parameters(lib, dim, dims):
    """Every parameter's gradient against the oracle's chain rule; the 3D
    grids span several 8 x 8 x 4 tiles of the matrix-core weight gradient,
    ragged in every direction."""
    import torch
    dims, op, A, dt, net, P, F, diag = _case(lib, dim, dims)
    rng = np.random.default_rng(7)
    r = rng.normal(size=op.N).astype(np.float32).astype(np.float64)
    gz = rng.normal(size=op.N).astype(np.float32).astype(np.float64)
    rg = torch.from_numpy(r).float().cuda()
    saved = torch.empty((49, op.N), dtype=torch.float32, device="cuda")
    net.forward(rg, saved=saved)
    gp = torch.zeros(net.nparams, dtype=torch.float32, device="cuda")
    gg = torch.zeros((49, op.N), dtype=torch.float32, device="cuda")
    net.backward(rg, torch.from_numpy(gz).float().cuda(), saved, gp, gg)
    net.gates_backward(gg, gp)
    ref = solvers.net_backward(P, F, r, gz)
    got = solvers.net_unpack(gp.double().cpu().numpy(), dim)
    for name, _ in solvers.net_shapes(dim):
        assert _rel(got[name], ref[name]) <= 1e-4, name


def test_loss_grad(lib):
    import torch
    dims, op, A, dt, net, P, F, diag = _case(lib, 2)
    K = solvers.system_matrix(A, dt)
    rng = np.random.default_rng(8)
    r = rng.normal(size=op.N).astype(np.float32).astype(np.float64)
    z = rng.normal(size=op.N).astype(np.float32).astype(np.float64)
    gz = torch.empty(op.N, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.loss_grad(dt, torch.from_numpy(r).float().cuda(), torch.from_numpy(z).float().cuda(), gz, loss)
    lr, gr = solvers.energy_loss(K, z, r)
    assert abs(loss.item() - lr) <= 1e-5 * abs(lr)
    assert _rel(gz.double().cpu().numpy(), gr) <= 1e-5


def test_adam_matches_torch(lib):
    import torch
    n = 1000
    p0 = torch.randn(n, generator=torch.Generator().manual_seed(0))
    p_ref = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([p_ref], lr=1e-2)
    p = p0.clone().cuda()
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    for step in range(1, 6):
        g = torch.randn(n, generator=torch.Generator().manual_seed(step))
        opt.zero_grad()
        p_ref.grad = 0.25 * g  # the library averages a batch of 4 summed gradients
        opt.step()
        lib.adam(p, g.cuda(), m, v, step, 1e-2, grad_scale=0.25)
    assert torch.allclose(p.cpu(), p_ref.detach(), rtol=1e-5, atol=1e-6)


def test_residual(lib):
    import torch
    dims, op, A, dt, net, P, F, diag = _case(lib, 2)
    K = solvers.system_matrix(A, dt)
    b = synth.uniform(1, op.N).astype(np.float32).astype(np.float64)
    x = synth.uniform(2, op.N).astype(np.float32).astype(np.float64)
    r = lib.residual(op, torch.from_numpy(b).float().cuda(), torch.from_numpy(x).float().cuda(), dt)
    assert _rel(r.double().cpu().numpy(), b - K @ x) <= 1e-5


@pytest.mark.parametrize("dims", [(100, 75), (21, 18, 13)])
def test_mfma_inference_matches_fp32_forward(lib, dims):
    """The MFMA inference (2D: the fused kernel; 3D: the layer kernels)
    agrees with the FP32 forward to BF16 accuracy on a ragged grid (tiles
    cut by every edge)."""
    import torch
    D = (synth.tensor2d_field(9, *dims, 100.0) if len(dims) == 2
         else synth.tensor3d_field(9, dims, 50.0))
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=torch.float32)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy())
    net = lib.Net(op, seed=3)
    net.prepare(50.0 * oracle.cfl(A))
    r = torch.from_numpy(synth.uniform(4, op.N) - 0.5).float().cuda()
    z32 = net.forward(r)
    z16 = net.precondition(r)
    n32 = (z32 - r * net.features[0])
    n16 = (z16 - r * net.features[0])
    assert float((n16 - n32).norm() / n32.norm()) <= 3e-2
    assert float((z16 - z32).norm() / z32.norm()) <= 1e-2


@pytest.mark.parametrize("dim", [2, 3])
def test_fcg_untrained_net_converges(lib, dim):
    """Flexible CG with the (untrained) network reaches 1e-6 true residual
    on the network itself, with no fallback to Jacobi-PCG, through the MFMA
    inference in both dimensions (2D: the fused kernel; 3D: the 1 -> 16
    and 16 -> 1 layers in FP32, the two 16 -> 16 layers on MFMA)."""
    import torch
    dims = (96, 80) if dim == 2 else (20, 18, 16)
    D = synth.tensor2d_field(21, *dims, 200.0) if dim == 2 else synth.tensor3d_field(22, dims, 50.0)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=torch.float32)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy())
    dt = 50.0 * oracle.cfl(A)
    net = lib.Net(op, seed=5)
    net.prepare(dt)
    b = torch.from_numpy(synth.uniform(6, op.N)).float().cuda()
    x, rep = op.solve(b, dt, method="fcg", net=net, tol=1e-6)
    assert rep["converged"] == 1 and rep["rel_res"] <= 1e-6, rep
    assert rep["fell_back"] == 0 and rep["net_iters"] == rep["iters"] > 0, rep
    K = solvers.system_matrix(A, dt)
    xr = solvers.jacobi_pcg(K, b.double().cpu().numpy(), tol=1e-9)[0]
    assert _rel(x.double().cpu().numpy(), xr) <= 3e-6


def test_fcg_falls_back_on_nan_weights(lib):
    """A network with NaN weights makes FCG restart with Jacobi-PCG."""
    import torch
    dims = (64, 64)
    D = synth.tensor2d_field(23, *dims, 50.0)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=torch.float32)
    dt = 50.0 * op.dt_cfl()
    p = lib.Net.init_params(2, 1)
    p[-10:] = float("nan")
    net = lib.Net(op, params=p)
    net.prepare(dt)
    b = torch.from_numpy(synth.uniform(7, op.N)).float().cuda()
    x, rep = op.solve(b, dt, method="fcg", net=net, tol=1e-6)
    assert rep["fell_back"] == 1 and rep["converged"] == 1 and rep["rel_res"] <= 1e-6, rep


def test_training_gains_over_untrained_and_jacobi(lib):
    """The 'gain' test: a network trained on solver-generated residuals
    (seeds distinct from the test right-hand side) needs fewer FCG
    iterations than the untrained network and than Jacobi-PCG."""
    import torch
    dims = (128, 128)
    D = synth.tensor2d_field(1305, *dims, 200.0)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=torch.float32)
    dt = 50.0 * op.dt_cfl()
    b = torch.from_numpy(synth.uniform(1305, op.N)).float().cuda()
    _, rj = op.solve(b, dt, tol=1e-6, check_every=1)
    untrained = lib.Net(op, seed=0)
    untrained.prepare(dt)
    _, ru = op.solve(b, dt, method="fcg", net=untrained, tol=1e-6, check_every=1)
    net, hist = lib.train_net(op, dt, rhs_seeds=range(2001, 2005), steps=150, batch=4, lr=3e-3,
                              seed=0, log_every=50)
    _, rt = op.solve(b, dt, method="fcg", net=net, tol=1e-6, check_every=1)
    print("jacobi", rj["iters"], "untrained", ru["iters"], "trained", rt["iters"], hist)
    assert rt["converged"] == 1 and rt["fell_back"] == 0
    assert rt["iters"] < ru["iters"] and rt["iters"] < rj["iters"]
