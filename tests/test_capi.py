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


def test_tuner_cache_file_round_trip(lib, tmp_path):
    """The batch tuner's JSON cache: load merges a file's entries (keyed by
    class, floor(log2 points) and problem count), save writes them back in
    the same format, a malformed file changes nothing.  Host code only."""
    import json
    import paper_1301_3925_amd as adlbr
    adlbr.tune_cache_clear()
    src = tmp_path / "tune.json"
    src.write_text(json.dumps({"format": "adlbr-batch-tune", "version": 1, "entries": [
        {"class": 2001, "log2_points": 25, "problems": 64, "variant": 1, "chunk_bytes": 234881024},
        {"class": 3001, "log2_points": 24, "problems": 8, "variant": 6, "chunk_bytes": 0}]}))
    adlbr.tune_cache_load(src)
    # any point count in [2^25, 2^26) falls in the first entry's bucket
    assert adlbr.tune_cache_lookup(2001, 56455727, 64) == (1, 234881024)
    assert adlbr.tune_cache_lookup(2001, 1 << 25, 64) == (1, 234881024)
    assert adlbr.tune_cache_lookup(2001, 1 << 26, 64) is None
    assert adlbr.tune_cache_lookup(3001, 23505948, 8) == (6, 0)
    assert adlbr.tune_cache_lookup(3001, 23505948, 9) is None
    out = tmp_path / "saved.json"
    adlbr.tune_cache_save(out)
    saved = json.loads(out.read_text())
    assert saved["format"] == "adlbr-batch-tune"
    got = sorted((e["class"], e["log2_points"], e["problems"], e["variant"], e["chunk_bytes"])
                 for e in saved["entries"])
    assert got == [(2001, 25, 64, 1, 234881024), (3001, 24, 8, 6, 0)]
    adlbr.tune_cache_clear()
    assert adlbr.tune_cache_lookup(2001, 56455727, 64) is None
    adlbr.tune_cache_load(out)
    assert adlbr.tune_cache_lookup(3001, 23505948, 8) == (6, 0)
    # malformed files: refused, the cache unchanged
    for bad in ({"format": "something-else", "entries": []},
                {"format": "adlbr-batch-tune", "entries": [{"class": 1, "log2_points": 3,
                                                            "problems": 2, "variant": 16,
                                                            "chunk_bytes": 0}]},
                {"format": "adlbr-batch-tune", "entries": [{"class": 1, "problems": 2,
                                                            "variant": 0, "chunk_bytes": 0}]}):
        f = tmp_path / "bad.json"
        f.write_text(json.dumps(bad))
        with pytest.raises(adlbr.AdlbrError) as ei:
            adlbr.tune_cache_load(f)
        assert ei.value.code == capi.E_INVALID
    with pytest.raises(adlbr.AdlbrError):
        adlbr.tune_cache_load(tmp_path / "missing.json")
    assert adlbr.tune_cache_lookup(3001, 23505948, 8) == (6, 0)
    assert adlbr.tune_cache_lookup(1, 8, 2) is None
    adlbr.tune_cache_clear()
