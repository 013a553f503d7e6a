"""The 2D parity cases of the operator tests reach every path of the row
sort in the assembly.

The row pass sorts the incoming entries of each target with an 8-, 12- or
16-key network, chosen by the largest row of the target's wavefront (64
consecutive targets), and sorts rows of more than 16 entries serially. The
GPU parity tests of the operator (entries, diagonal, apply and step against
the oracle) only prove those paths if their inputs reach them; this counts
the incoming edges of every target from the oracle's stencils of the same
inputs (the GPU's are bit-identical to them) and checks that each path
occurs.
"""
import numpy as np

import oracle
from paper_1301_3925_amd import synth

# the 2D cases of the operator parity tests: (dims, tensor field, periodic)
CASES_2D = [
    ((64, 64), lambda: synth.tensor2d_field(1301, 64, 64, 10.0), False),
    ((97, 61), lambda: synth.tensor2d_field(11, 97, 61, 50.0), False),
    ((48, 40), lambda: synth.tensor2d_field(12, 48, 40, 10.0), True),
    ((2, 3000), lambda: synth.tensor2d_field(17, 2, 3000, 20.0), False),
    ((200, 150), lambda: synth.tensor2d_field(18, 200, 150, 250.0), False),
]


def _incoming_counts(dims, off, w, periodic):
    """Edges of positive weight that land on each target from another point
    (both signs of every offset, x fastest)."""
    nx, ny = dims
    n = nx * ny
    z = np.arange(n)
    x, y = z % nx, z // nx
    cnt = np.zeros(n, np.int64)
    for q in range(off.shape[0]):
        for s in (-1, 1):
            tx = x + s * off[q, 0].astype(np.int64)
            ty = y + s * off[q, 1].astype(np.int64)
            if periodic:
                t = tx % nx + nx * (ty % ny)
                ok = (w[q] > 0) & (t != z)
            else:
                ok = (w[q] > 0) & (tx >= 0) & (tx < nx) & (ty >= 0) & (ty < ny)
                t = tx + nx * ty
            np.add.at(cnt, t[ok], 1)
    return cnt


def _own_counts(dims, off, w, periodic):
    """Edges of positive weight that leave each point (to a point in the
    grid, other than itself)."""
    nx, ny = dims
    n = nx * ny
    z = np.arange(n)
    x, y = z % nx, z // nx
    own = np.zeros(n, np.int64)
    for q in range(off.shape[0]):
        for s in (-1, 1):
            tx = x + s * off[q, 0].astype(np.int64)
            ty = y + s * off[q, 1].astype(np.int64)
            if periodic:
                ok = (w[q] > 0) & (tx % nx + nx * (ty % ny) != z)
            else:
                ok = (w[q] > 0) & (tx >= 0) & (tx < nx) & (ty >= 0) & (ty < ny)
            own += ok
    return own


def test_counts_match_the_operator_matrix():
    """Row z of A couples z to its own targets and to its sources (each
    source reaches z by one edge at most), so its off-diagonal count lies
    between the larger of the two counts and their sum."""
    for dims, mk, per in (CASES_2D[1], CASES_2D[2]):
        off, w, _ = oracle.stencil(mk())
        cnt = _incoming_counts(dims, off, w, per)
        own = _own_counts(dims, off, w, per)
        A = oracle.operator_matrix(dims, off, w, periodic=per).tocsr()
        A.setdiag(0)
        A.eliminate_zeros()
        nnz = np.diff(A.indptr)
        assert np.all(nnz <= cnt + own) and np.all(nnz >= np.maximum(cnt, own))
        assert cnt.sum() == own.sum()  # every edge has one source and one target


def test_parity_cases_reach_every_sort_path():
    seen = {"<=8": 0, "9-12": 0, "13-16": 0, ">16 (serial rows)": 0}
    for dims, mk, per in CASES_2D:
        off, w, _ = oracle.stencil(mk())
        cnt = _incoming_counts(dims, off, w, per)
        cw = np.array([cnt[i:i + 64].max() for i in range(0, cnt.size, 64)])
        seen["<=8"] += int((cw <= 8).sum())
        seen["9-12"] += int(((cw > 8) & (cw <= 12)).sum())
        seen["13-16"] += int(((cw > 12) & (cw <= 16)).sum())
        seen[">16 (serial rows)"] += int((cnt > 16).sum())
    assert all(v > 0 for v in seen.values()), seen
