"""The allocation-free structure tensor (adlbr_structure_tensor_noalloc),
through the C ABI, against the workspace entry point adlbr_structure_tensor
and the FP64 oracle: two calls in a row, the second on a smaller grid (the
static scratch keeps the first call's contents), then a grid whose scratch
would exceed the static array, which is refused before any launch."""
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


def test_noalloc_tensor_matches_workspace_entry_point_twice(lib):
    import torch
    # first call: a 2D FP32 image (scratch 2 x 3 x N x 4 bytes = 18.9 MB)
    dims = (1024, 768)
    u = torch.from_numpy(synth.ced_image2d(21, *dims, ndiscs=5)).float().cuda()
    got = lib.structure_tensor_noalloc(u, dims, 1.0, 4.0, 1e-4, 1e-5)
    ref = lib.structure_tensor(u, dims, 1.0, 4.0, 1e-4, 1e-5)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    Dr = oracle.structure_tensor_d(u.double().cpu().numpy(), dims, 1.0, 4.0, 1e-4, 1e-5)
    assert _rel(got.double().cpu().numpy(), Dr) <= 1e-5
    # second call, smaller: a 3D FP64 volume (scratch 4.1 MB), edge-enhancing map
    dims3 = (40, 36, 30)
    u3 = torch.from_numpy(synth.ced_image3d(22, 40)[: int(np.prod(dims3))]).cuda()
    got3 = lib.structure_tensor_noalloc(u3, dims3, 0.5, 2.0, 1e-2, 1e-3, eig_map="eed")
    ref3 = lib.structure_tensor(u3, dims3, 0.5, 2.0, 1e-2, 1e-3, eig_map="eed")
    torch.cuda.synchronize()
    assert torch.equal(got3, ref3)
    Dr3 = oracle.structure_tensor_d(u3.cpu().numpy(), dims3, 0.5, 2.0, 1e-2, 1e-3, oracle.EED)
    assert _rel(got3.cpu().numpy(), Dr3) <= 1e-12


def test_noalloc_tensor_refuses_grids_beyond_its_scratch(lib):
    import torch
    dims = (2400, 2400)  # 2 x 3 x 5.76e6 x 4 bytes = 138 MB > 128 MiB
    u = torch.zeros(dims[0] * dims[1], dtype=torch.float32, device="cuda")
    out = torch.empty((3, u.numel()), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.AdlbrError) as ei:
        lib.structure_tensor_noalloc(u, dims, 1.0, 4.0, 1e-4, 1e-5, out=out)
    assert ei.value.code == lib.capi.E_NOMEM
