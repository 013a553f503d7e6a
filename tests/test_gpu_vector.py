"""Vector-valued images on the GPU (the Conclusion: AD-LBR runs on each
component with one common tensor; the coupling lies in the tensor).

- adlbr_step_multi: every component bit-identical to adlbr_step on that
  component alone, for 1..9 components (groups of four and a tail), 2D and
  3D, FP64, FP32 and BF16 storage; and equal to the oracle's explicit steps
  (FP64 1e-12, FP32 1e-5) with Neumann, periodic and reflecting boundaries.
- adlbr_structure_tensor_vec: the summed tensor against the oracle's (FP64
  1e-12, FP32 1e-5), through the LDS-tiled 2D FP32 kernels and the
  streaming passes; one component is bit-identical to
  adlbr_structure_tensor.
- A colour CED run end to end: tensor from three channels, one operator,
  fused steps, against the oracle.
"""
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


def _field(dims, seed, kappa):
    return (synth.tensor2d_field(seed, *dims, kappa) if len(dims) == 2
            else synth.tensor3d_field(seed, dims, kappa))


@pytest.mark.parametrize("dims,kappa", [((97, 61), 30.0), ((20, 17, 13), 20.0)])
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("ncomp", [1, 3, 4, 5, 9])
def test_step_multi_bitwise_per_component(lib, dims, kappa, storage, ncomp):
    import torch
    td = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[storage]
    off, w, _ = lib.build_stencils(torch.from_numpy(_field(dims, 3, kappa)).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=td)
    u = torch.stack([torch.from_numpy(synth.uniform(40 + c, op.N)) for c in range(ncomp)])
    u = u.to(td).cuda().contiguous()
    ref = u.clone()
    for c in range(ncomp):
        x = ref[c].clone()
        op.step(x, 0.9, 7, cfl_fraction=True)
        ref[c] = x
    op.step_multi(u, 0.9, 7, cfl_fraction=True)
    torch.cuda.synchronize()
    for c in range(ncomp):
        assert torch.equal(u[c], ref[c]), c


@pytest.mark.parametrize("mode", ["neumann", "periodic", "reflect"])
@pytest.mark.parametrize("dims", [(64, 48), (12, 11, 9)])
def test_step_multi_vs_oracle(lib, mode, dims):
    import torch
    per, refl = mode == "periodic", mode == "reflect"
    off, w, _ = lib.build_stencils(torch.from_numpy(_field(dims, 8, 10.0)).cuda(), dims,
                                   periodic=per)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy(), periodic=per,
                               reflect=refl)
    h = 0.9 * oracle.cfl(A)
    u0 = np.stack([synth.uniform(60 + c, A.shape[0]) for c in range(3)])
    for td, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
        op = lib.Operator(dims, off, w, storage=td, periodic=per, reflect=refl)
        u = torch.from_numpy(u0).to(td).cuda().contiguous()
        op.step_multi(u, 0.9, 25, cfl_fraction=True)
        got = u.double().cpu().numpy()
        for c in range(3):
            uq = torch.from_numpy(u0[c]).to(td).double().numpy()
            ref = oracle.explicit_steps(A, uq, h, 25)
            assert _rel(got[c], ref) <= tol, (td, c)


def test_step_multi_rejects(lib):
    import torch
    dims = (40, 30)
    off, w, _ = lib.build_stencils(torch.from_numpy(_field(dims, 2, 5.0)).cuda(), dims)
    op = lib.Operator(dims, off, w, storage=torch.float32, tiled=True)
    u = torch.zeros((2, op.N), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.AdlbrError) as ei:
        op.step_multi(u, 0.9, 1, cfl_fraction=True)
    assert ei.value.code == lib.capi.E_UNSUPPORTED
    opl = lib.Operator(dims, off, w, storage=torch.float32)
    with pytest.raises(ValueError):
        opl.step_multi(torch.zeros((2, op.N + 1), dtype=torch.float32, device="cuda"), 0.9, 1)
    # zero steps leave u alone
    x = torch.rand((2, op.N), dtype=torch.float32, device="cuda")
    y = x.clone()
    opl.step_multi(x, 0.9, 0, cfl_fraction=True)
    assert torch.equal(x, y)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("dims", [(160, 120), (7, 5), (20, 18, 16)])
def test_structure_tensor_vec_vs_oracle(lib, dtype, dims):
    """FP32 2D takes the LDS-tiled kernels, the rest the streaming passes."""
    import torch
    td = {"f32": torch.float32, "f64": torch.float64}[dtype]
    n = int(np.prod(dims))
    if len(dims) == 2 and n > 100:
        u = np.stack([synth.ced_image2d(90 + c, *dims).reshape(-1) for c in range(3)])
    else:
        u = np.stack([synth.uniform(90 + c, n) for c in range(3)])
    ug = torch.from_numpy(u).to(td).cuda().contiguous()
    ref_in = ug.double().cpu().numpy()
    tol = 1e-5 if dtype == "f32" else 1e-12
    for eig_map in (("ced", "eed") if len(dims) == 3 else ("ced",)):
        D = lib.structure_tensor(ug, dims, 1.0, 4.0, 1e-2, 1e-6, eig_map=eig_map)
        ref = oracle.structure_tensor_d(ref_in, dims, 1.0, 4.0, 1e-2, 1e-6,
                                        oracle.CED if eig_map == "ced" else oracle.EED)
        assert _rel(D.double().cpu().numpy(), ref) <= tol, eig_map
    # one component: the same bits as the scalar entry point
    D1 = lib.structure_tensor(ug[:1].contiguous(), dims, 1.0, 4.0, 1e-2, 1e-6)
    D0 = lib.structure_tensor(ug[0].contiguous(), dims, 1.0, 4.0, 1e-2, 1e-6)
    assert torch.equal(D1, D0)


def test_colour_ced_end_to_end(lib):
    """Three channels: the common CED tensor, its stencils, 10 fused FP32
    steps; every channel against the oracle's run on the same tensor."""
    import torch
    dims = (96, 80)
    u0 = np.stack([synth.ced_image2d(110 + c, *dims).reshape(-1) for c in range(3)])
    ug = torch.from_numpy(u0).float().cuda().contiguous()
    D = lib.structure_tensor(ug, dims, 1.0, 4.0, 1e-2, 1e-6)
    Dr = oracle.structure_tensor_d(ug.double().cpu().numpy(), dims, 1.0, 4.0, 1e-2, 1e-6)
    assert _rel(D.double().cpu().numpy(), Dr) <= 1e-5
    off, w, st = lib.build_stencils(D, dims)
    assert st.cpu().numpy()[0] == -1
    op = lib.Operator(dims, off, w, storage=torch.float32)
    A = oracle.operator_matrix(dims, off.cpu().numpy(), w.cpu().numpy())
    x = ug.clone()
    op.step_multi(x, 0.9, 10, cfl_fraction=True)
    got = x.double().cpu().numpy()
    for c in range(3):
        ref = oracle.explicit_steps(A, ug[c].double().cpu().numpy(), 0.9 * oracle.cfl(A), 10)
        assert _rel(got[c], ref) <= 1e-5, c
