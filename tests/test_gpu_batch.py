"""Batched explicit stepping (adlbr_batch_*) against single-operator steps.

The grouped kernel runs the same per-block body as adlbr_step, so every
problem of a batch must come out bit-identical to stepping it alone, for
any launch variant, with and without the captured graph, for even and odd
step counts and for replays of the graph, with and without the 2D
records (ADLBR_OP_RECORDS).  One 2D problem is also checked against the
FP64 oracle.
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


def _problems(lib, dtype, periodic=False, records=False):
    import torch
    specs = [((70, 45), 10.0), ((33, 90), 30.0), ((128, 64), 5.0), ((12, 11, 9), 8.0),
             ((20, 17, 15), 20.0), ((5, 3), 2.0)]
    ops, us = [], []
    for k, (dims, kappa) in enumerate(specs):
        D = (synth.tensor2d_field(100 + k, *dims, kappa) if len(dims) == 2
             else synth.tensor3d_field(100 + k, dims, kappa))
        off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
        ops.append(lib.Operator(dims, off, w, storage=dtype, periodic=periodic, records=records))
        us.append(torch.from_numpy(synth.uniform(200 + k, int(np.prod(dims)))).to(dtype).cuda())
    return ops, us


@pytest.mark.parametrize("nsteps", [1, 6, 7])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_single_steps_bitwise(lib, nsteps, graph):
    import torch
    ops, us = _problems(lib, torch.float32)
    ref = [u.clone() for u in us]
    for op, u in zip(ops, ref):
        op.step(u, 0.9, nsteps, cfl_fraction=True)
    b = lib.Batch(ops, us, dt=0.9, dt_mode="cfl")
    b.run(nsteps, graph=graph)
    torch.cuda.synchronize()
    for k, (u, r) in enumerate(zip(us, ref)):
        assert torch.equal(u, r), k


def test_batch_every_variant_and_graph_replay(lib):
    """The tuner's variants reorder blocks only; replays continue the state."""
    import torch
    ops, us = _problems(lib, torch.float64, periodic=True)
    ref = [u.clone() for u in us]
    for op, u in zip(ops, ref):
        op.step(u, 0.5, 8, cfl_fraction=True)
    b = lib.Batch(ops, us, dt=0.5, dt_mode="cfl")
    vs = b.tune(steps=2, use_cache=False)
    assert len(vs) == 2 and sum(v["problems"] for v in vs) == len(ops)
    assert all(0 <= v["variant"] < 8 for v in vs)
    b.run(4)
    b.run(4)  # replay of the captured graph
    torch.cuda.synchronize()
    for k, (u, r) in enumerate(zip(us, ref)):
        assert torch.equal(u, r), k


@pytest.mark.parametrize("chunk_bytes", [0, 1, 300_000])
@pytest.mark.parametrize("variant", range(16))
def test_batch_forced_variant_bitwise(lib, variant, chunk_bytes):
    """Grouped or per-problem launches, in any block order, whole or cut into
    chunks (1 byte: one problem per chunk), one chunk at a time or two in
    flight on two streams, give the same bits."""
    import torch
    ops, us = _problems(lib, torch.float32)
    ref = [u.clone() for u in us]
    for op, u in zip(ops, ref):
        op.step(u, 0.9, 5, cfl_fraction=True)
    b = lib.Batch(ops, us, dt=0.9, dt_mode="cfl")
    for cls in range(len(b.variants())):
        b.set_variant(cls, variant, chunk_bytes)
    vs = b.variants()
    assert all(v["variant"] == variant and v["chunk_bytes"] == chunk_bytes for v in vs)
    if chunk_bytes == 1:
        assert [v["chunks"] for v in vs] == [v["problems"] for v in vs]
    if chunk_bytes == 0:
        assert all(v["chunks"] == 1 for v in vs)
    b.run(2)
    b.run(3)  # odd count: the final copy runs through the same variant
    torch.cuda.synchronize()
    for k, (u, r) in enumerate(zip(us, ref)):
        assert torch.equal(u, r), k
    with pytest.raises(Exception):
        b.set_variant(0, 16)


def test_batch_absolute_dt_and_oracle(lib):
    import torch
    ops, us = _problems(lib, torch.float64)
    dts = [0.5 * op.dt_cfl() for op in ops]
    u0 = us[0].cpu().numpy().copy()
    b = lib.Batch(ops, us, dt=dts, dt_mode="abs")
    b.run(10)
    torch.cuda.synchronize()
    dims = ops[0].dims
    off, w, _ = oracle.stencil(synth.tensor2d_field(100, *dims, 10.0))
    A = oracle.operator_matrix(dims, off, w)
    ref = oracle.explicit_steps(A, u0, dts[0], 10)
    got = us[0].cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12


def test_batch_rejects_bad_arguments(lib):
    import torch
    ops, us = _problems(lib, torch.float32)
    with pytest.raises(Exception):
        lib.Batch(ops, us[:-1])
    with pytest.raises(Exception):
        lib.Batch(ops[:1], us[:1], tmps=us[:1])  # u aliased with its scratch


def test_rebuild_in_place_keeps_the_batch_graph_valid(lib):
    """adlbr_operator_rebuild re-assembles an operator from new stencils
    into the same workspace: a batch whose graph was captured before the
    rebuild steps the new operators, bit-identical to operators created
    from scratch on the new stencils (2D and 3D, FP32)."""
    import torch
    ops, us = _problems(lib, torch.float32)
    b = lib.Batch(ops, us, dt=0.9, dt_mode="cfl")
    b.run(4)  # captures the graph for 4 steps
    torch.cuda.synchronize()
    fresh = []
    for k, op in enumerate(ops):
        dims = op.dims
        D = (synth.tensor2d_field(300 + k, *dims, 40.0) if len(dims) == 2
             else synth.tensor3d_field(300 + k, dims, 40.0))
        off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
        op.rebuild(off, w, check=True)
        fresh.append(lib.Operator(dims, off, w, storage=torch.float32))
    ref = [u.clone() for u in us]
    for op, u in zip(fresh, ref):
        op.step(u, 0.9, 4, cfl_fraction=True)
    b.run(4)  # the same graph, replayed
    torch.cuda.synchronize()
    for k, (u, r) in enumerate(zip(us, ref)):
        assert torch.equal(u, r), k
    for op, f in zip(ops, fresh):
        assert op.dt_cfl() == f.dt_cfl()


def test_tuner_cache_file_serves_a_new_batch(lib, tmp_path):
    """Tune, save the tuner's choices to a JSON file, forget them, load the
    file: a new batch of the same classes starts with the saved variants
    and chunk budgets (adlbr_batch_create takes them from the cache), and
    still steps bit-identically to single-operator steps."""
    import torch
    lib.tune_cache_clear()
    ops, us = _problems(lib, torch.float32)
    b = lib.Batch(ops, us, dt=0.9, dt_mode="cfl")
    tuned = b.tune(steps=2, use_cache=False)
    path = tmp_path / "tune.json"
    lib.tune_cache_save(path)
    lib.tune_cache_clear()
    # with an empty cache a new batch starts from the default variant
    fresh = lib.Batch(ops, [u.clone() for u in us], dt=0.9, dt_mode="cfl").variants()
    assert all(v["variant"] == 1 and v["chunk_bytes"] == 0 for v in fresh)
    lib.tune_cache_load(path)
    us2 = [u.clone() for u in us]
    b2 = lib.Batch(ops, us2, dt=0.9, dt_mode="cfl")
    got = b2.variants()
    key = lambda v: (v["class"], v["variant"], v["chunk_bytes"], v["problems"])
    assert sorted(map(key, got)) == sorted(map(key, tuned))
    ref = [u.clone() for u in us]
    for op, u in zip(ops, ref):
        op.step(u, 0.9, 5, cfl_fraction=True)
    b2.run(5)
    torch.cuda.synchronize()
    for k, (u, r) in enumerate(zip(us2, ref)):
        assert torch.equal(u, r), k
    lib.tune_cache_clear()


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_records_batch_bitwise(lib, dtype, periodic):
    """2D operators with records (ADLBR_OP_RECORDS) form a batch class of
    their own, whose grouped step reads each incoming weight from the
    entry's record.  With the same problems also present without records,
    every problem comes out bit-identical to its single-operator steps
    (which read the lists as without the flag), in both block orders, whole
    or cut into chunks."""
    import torch
    td = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
          "f16": torch.float16}[dtype]
    rops, rus = _problems(lib, td, periodic, records=True)
    pops, pus = _problems(lib, td, periodic)
    ops = rops + pops
    assert rops[0].workspace.numel() > pops[0].workspace.numel()  # the 2D records
    u0 = [u.clone() for u in rus + pus]
    ref = [u.clone() for u in u0]
    for op, u in zip(ops, ref):
        op.step(u, 0.9, 5, cfl_fraction=True)
    for variant, chunk_bytes in ((1, 300_000), (0, 0)):
        us = [u.clone() for u in u0]
        b = lib.Batch(ops, us, dt=0.9, dt_mode="cfl")
        keys = [v["class"] for v in b.variants()]
        assert sum(1 for k in keys if k // 1000 % 10 == 2) == 2  # 2D with and without records
        assert sum(1 for k in keys if k >= 100000) == 1
        for cls in range(len(keys)):
            b.set_variant(cls, variant, chunk_bytes)
        b.run(2)
        b.run(3)
        torch.cuda.synchronize()
        for k, (u, r) in enumerate(zip(us, ref)):
            assert torch.equal(u, r), (variant, k)


def test_records_need_the_list_layout(lib):
    import torch
    dims = (40, 30)
    D = synth.tensor2d_field(7, *dims, 5.0)
    off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
    with pytest.raises(lib.AdlbrError) as ei:
        lib.Operator(dims, off, w, storage=torch.float32, tiled=True, records=True)
    assert ei.value.code == lib.capi.E_UNSUPPORTED



@pytest.mark.parametrize("variant", [8, 9, 10, 12])
def test_two_chunks_in_flight_with_an_odd_chunk_count(lib, variant):
    """One problem per chunk, two chunks in flight: three image operators
    with records (a pair on the two streams, then the last chunk alone) and
    two without (one pair), each set in a batch of its own; graph replays
    and a direct run give the bits of single steps."""
    import torch
    ops, us = [], []
    for k, dims in enumerate([(40, 31), (64, 17), (23, 50), (80, 40), (9, 70)]):
        D = synth.tensor2d_field(300 + k, *dims, 20.0)
        off, w, _ = lib.build_stencils(torch.from_numpy(D).cuda(), dims)
        ops.append(lib.Operator(dims, off, w, storage=torch.float32, records=k % 2 == 0))
        us.append(torch.from_numpy(synth.uniform(400 + k, int(np.prod(dims)))).float().cuda())
    ref = [u.clone() for u in us]
    for op, u in zip(ops, ref):
        op.step(u, 0.9, 9, cfl_fraction=True)
    rec = [k for k in range(5) if k % 2 == 0]
    b = lib.Batch([ops[k] for k in rec], [us[k] for k in rec], dt=0.9, dt_mode="cfl")
    b.set_variant(0, variant, 1)
    assert b.variants()[0]["chunks"] == 3
    b.run(4)
    b.run(4)  # replay
    b.run(1, graph=False)
    b2 = lib.Batch([ops[k] for k in range(5) if k % 2], [us[k] for k in range(5) if k % 2],
                   dt=0.9, dt_mode="cfl")
    b2.set_variant(0, variant, 1)
    assert b2.variants()[0]["chunks"] == 2
    b2.run(9)
    torch.cuda.synchronize()
    for k, (u, r) in enumerate(zip(us, ref)):
        assert torch.equal(u, r), k
