"""GPU parity of the stencil builder against the FP64 oracle.

Offsets are integers decided in FP64: they must match bit for bit.  Weights
are FP64 values computed by different formulas on the two sides (oracle: the
paper's perpendicular form; GPU: the adjugate form), each a difference of
products of size |D| r^2 for stencil radius r, so the bound is
|w_gpu - w_oracle| <= 1e-14 |D|_max max(1, r^2) per point.  In 3D a weight
-1/2 <e_i, D e_j> is a sum of products of size |D| |e_i|_1 |e_j|_1 over the
superbase vectors, which can be far longer than the offsets e_k x e_l once
the anisotropy is extreme; there the bound takes max(1, r^2, max_i |e_i|_1^2).
FP32 weights must equal the FP32 rounding of the oracle's value to 1e-6
relative.
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


def _gpu(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _check(lib, D, dims, D_dtype="f64", w_dtype="f64"):
    import torch
    td = {"f64": torch.float64, "f32": torch.float32}
    Dg = _gpu(D, td[D_dtype])
    off, w, st = lib.build_stencils(Dg, dims, w_dtype=td[w_dtype])
    Dref = Dg.double().cpu().numpy()  # the oracle sees exactly the GPU's input
    ro, rw, rst = oracle.stencil(Dref)
    off, w, st = off.cpu().numpy(), w.cpu().numpy(), st.cpu().numpy()
    bad = np.where(rst & 7)[0]
    assert st[0] == (bad[0] if bad.size else -1)
    assert np.array_equal(off, ro), "offsets differ"
    if w_dtype == "f64":
        r2 = (ro.astype(np.float64) ** 2).sum(1).max(0)
        if len(dims) == 3:
            sb = oracle.superbase3d(Dref)[0].astype(np.float64)
            r2 = np.maximum(r2, np.abs(sb).sum(1).max(0) ** 2)
        scale = np.nan_to_num(np.abs(Dref), nan=0.0, posinf=0.0).max(0) * np.maximum(1.0, r2)
        assert np.all(np.abs(w - rw) <= 1e-14 * scale)
    else:
        assert np.allclose(w, rw.astype(np.float32).astype(np.float64), rtol=1e-6, atol=0)
    return off, w


def test_c1_field_2d(lib):
    """64x64, kappa = 10 smooth orientation field (the 64^2 FP64 workload)."""
    D = synth.tensor2d_field(1301, 64, 64, 10.0)
    _check(lib, D, (64, 64))


@pytest.mark.parametrize("kmax", [3.0, 10.0, 200.0, 5000.0])
def test_random_tensors_2d(lib, kmax):
    D = synth.random_spd2(100 + int(kmax), 20000, kmax)
    _check(lib, D, (200, 100))


@pytest.mark.parametrize("kmax", [1e5, 1e7])
def test_extreme_anisotropy_2d(lib, kmax):
    """Reduced bases with components in the thousands and, at kappa = 1e7,
    beyond +-32767: there the 32-bit reduction overflows and the point is
    reduced again in 64-bit integers (and its offsets leave int16: status
    RANGE); offsets, weights and status still match the oracle."""
    D = synth.random_spd2(100 + int(kmax), 20000, kmax)
    off, _ = _check(lib, D, (200, 100))
    assert np.abs(off).max() > 3000
    if kmax >= 1e7:
        b, _ = oracle.reduce2d(D)
        assert (np.abs(b).max((0, 1)) > 32767).sum() >= 1  # the 64-bit path ran


def test_rational_and_tie_tensors_2d(lib):
    """Exact rationals and exact ties (D = Id, axis-aligned, the
    spectral-figure tensor, 2 mu = lambda_1^2 ties): identical decisions."""
    cols = [(1, 0, 1), (9.5, 6, 4), (2, 1, 2), (1, 0.5, 1), (1, -0.5, 1), (4, 2, 2),
            (3, 0, 0.25), (1, 1, 2), (2, 1, 1), (5, 3, 2), (0.5, 0.25, 0.5), (1, 0, 4)]
    D = np.array(cols, dtype=np.float64).T
    D = np.tile(D, (1, 40))
    _check(lib, D, (D.shape[1], 1))


def test_fp32_tensor_input_2d(lib):
    D = synth.tensor2d_field(7, 300, 200, 100.0)
    _check(lib, D, (300, 200), D_dtype="f32", w_dtype="f32")


def test_invalid_tensor_status_2d(lib):
    D = synth.random_spd2(3, 1000, 10.0)
    D[:, 417] = [1.0, 2.0, 1.0]      # indefinite
    D[:, 900] = [np.nan, 0.0, 1.0]   # not finite
    off, w = _check(lib, D, (1000, 1))
    assert np.all(off[:, :, [417, 900]] == 0) and np.all(w[:, [417, 900]] == 0)


def test_c3_recipe_3d(lib):
    """The 3D mixed needle/plate/isotropic recipe with kappa <= 50."""
    D = synth.tensor3d_field(1303, (24, 20, 16), 50.0)
    _check(lib, D, (24, 20, 16))


@pytest.mark.parametrize("kmax", [2.0, 10.0, 50.0, 200.0])
def test_random_tensors_3d(lib, kmax):
    D = synth.random_spd3(200 + int(kmax), 6000, kmax)
    _check(lib, D, (30, 20, 10))


@pytest.mark.parametrize("kmax", [1e6, 1e7])
def test_extreme_anisotropy_3d(lib, kmax):
    """Reduced bases with components in the tens of thousands and beyond the
    16-bit offset range: the 32-bit reduction overflows and the point is
    reduced again in 64-bit integers; offsets, weights and status still
    match the oracle.  (Past kappa ~ 1e8 the FP64 greedy reduction itself
    runs out of 64-bit integers on both sides, so no parity is claimed
    there.)"""
    D = synth.random_spd3(7, 4000, kmax)
    off, _ = _check(lib, D, (40, 10, 10))
    assert np.abs(off).max() > 10000
    if kmax >= 1e7:
        b, _ = oracle.reduce3d(D)
        assert (np.abs(b).max((0, 1)) > 32767).sum() >= 1  # the 64-bit path ran


def test_identity_and_ties_3d(lib):
    D = np.zeros((6, 8))
    D[0], D[3], D[5] = 1.0, 1.0, 1.0
    D[1, 1] = 0.5
    D[2, 2] = -0.5
    D[4, 3] = 0.25
    D[:, 4] = [2, 1, 1, 2, 1, 2]
    D[:, 5] = [1, 0, 0, 2, 0, 3]
    D[:, 6] = [3, -1, -1, 3, -1, 3]
    D[:, 7] = [1, 0.5, 0.5, 1, 0.5, 1]
    _check(lib, D, (8, 1, 1))


def test_invalid_tensor_status_3d(lib):
    D = synth.random_spd3(9, 500, 10.0)
    D[:, 123] = [1, 2, 0, 1, 0, 1]
    off, w = _check(lib, D, (500, 1, 1))
    assert np.all(w[:, 123] == 0)
