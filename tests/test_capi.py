"""The C-ABI library loads and exports every symbol include/adlbr.h declares.

No compute call is made here (there may be no GPU): only host-side argument
validation, which returns before any HIP call.
"""
import ctypes
import os

import pytest

from paper_1301_3925_amd import capi


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(capi.LIB_PATH):
        from paper_1301_3925_amd import build
        build.build()
    return capi.load()


def test_every_declared_symbol_is_exported(lib):
    names = capi.declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(capi.SIGNATURES), "binding and header disagree"


def test_version_and_error_string(lib):
    assert lib.adlbr_version() >= 100
    assert isinstance(lib.adlbr_last_error(), bytes)


def test_workspace_query_and_validation(lib):
    g = capi.Grid()
    g.dim, g.boundary = 2, capi.NEUMANN
    g.n[0], g.n[1], g.n[2] = 2048, 2048, 1
    nb = ctypes.c_size_t()
    assert lib.adlbr_operator_workspace(ctypes.byref(g), capi.F32, 0, ctypes.byref(nb)) == 0
    N = 2048 * 2048
    # slots 4 + weights 12 + cnt 1 + pos 4 + entries 24 + diag 4 + mask 1
    # + edge ranks 6 (+ per-block partials, chunk sums, and the 4 x 4 brick
    # and 64 x 64 tile reaches of the tile assembly: 1/4 + 1/1024 bytes a point)
    assert 56 * N <= nb.value <= 56 * N + N // 4 + N // 16 + 128 * 1024
    g.dim = 4
    assert lib.adlbr_operator_workspace(ctypes.byref(g), capi.F32, 0, ctypes.byref(nb)) == capi.E_INVALID
    assert b"dim" in lib.adlbr_last_error()
    g.dim = 3
    g.n[0] = g.n[1] = g.n[2] = 1024  # 2^30 points: too many
    assert lib.adlbr_operator_workspace(ctypes.byref(g), capi.F32, 0, ctypes.byref(nb)) == capi.E_RANGE
    g.n[0] = g.n[1] = g.n[2] = 16
    assert lib.adlbr_operator_workspace(ctypes.byref(g), 9, 0, ctypes.byref(nb)) == capi.E_INVALID
    assert lib.adlbr_tensor_workspace(ctypes.byref(g), capi.F32, ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 6 * 4 * 16 ** 3


def test_null_arguments_rejected_before_any_launch(lib):
    g = capi.Grid()
    g.dim, g.boundary = 2, capi.NEUMANN
    g.n[0], g.n[1], g.n[2] = 8, 8, 1
    rc = lib.adlbr_build_stencils(ctypes.byref(g), None, capi.F64, None, None, capi.F64, None, None)
    assert rc == capi.E_INVALID
    rc = lib.adlbr_apply(None, None, None, None)
    assert rc == capi.E_INVALID
    rc = lib.adlbr_step(None, None, None, 0.1, capi.DT_ABS, 1, None)
    assert rc == capi.E_INVALID
    h = ctypes.c_void_p()
    rc = lib.adlbr_operator_create(ctypes.byref(g), None, None, capi.F64, capi.F32, 0, None, 0,
                                   None, None, ctypes.byref(h))
    assert rc == capi.E_INVALID
