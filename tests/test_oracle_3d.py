"""Pins of the 3D oracle (greedy reduction, MakeObtuse, Selling).

The paper prints no 3D numbers, so the pins are closed forms (identity,
diagonal tensors), the identities it proves (Selling's lemma, obtuseness of
Proposition (MakeObtuse)) and brute force on tiny anisotropies.
"""
import numpy as np

import oracle
from oracle import brute
from paper_1301_3925_amd import synth


def _mat(D, z):
    return np.array([[D[0, z], D[1, z], D[2, z]],
                     [D[1, z], D[3, z], D[4, z]],
                     [D[2, z], D[4, z], D[5, z]]])


def test_identity_and_diagonal_give_axis_stencils():
    """D = Id gives the 7-point Laplacian; a diagonal D gives weight D_ii/2
    on the i-th axis and 0 elsewhere (Selling on the canonical superbase)."""
    D = np.zeros((6, 3))
    D[0], D[3], D[5] = [1.0, 2.0, 0.5], [1.0, 0.25, 3.0], [1.0, 4.0, 0.125]
    off, w, st = oracle.stencil3d(D)
    assert st.max() == 0
    for z in range(3):
        wf = brute.weight_function(off[:, :, z], w[:, z])
        assert wf == {(1, 0, 0): D[0, z] / 2, (0, 1, 0): D[3, z] / 2,
                      (0, 0, 1): D[5, z] / 2}


def _fields():
    return [synth.random_spd3(31, 2000, 10.0), synth.random_spd3(32, 500, 50.0),
            synth.tensor3d_field(1303, 12, 50.0)]


def test_selling_identity_and_nonnegativity():
    """Selling's lemma, eq. (DSum3D): D = sum_{e in V(z)} gamma(e) e e^T to
    1e-12 relative (scaled by r^4 eps for radius r > 10); gamma >= 0; 12
    offsets (6 slots)."""
    for D in _fields():
        off, w, st = oracle.stencil3d(D)
        assert st.max() == 0
        assert np.all(w >= 0)
        o = off.astype(np.float64)
        for z in range(D.shape[1]):
            S = sum(2 * w[q, z] * np.outer(o[q, :, z], o[q, :, z]) for q in range(6))
            Dz = _mat(D, z)
            r2 = (o[:, :, z] ** 2).sum(1).max()
            tol = max(1e-12, 1e-16 * r2 * r2)
            assert np.linalg.norm(S - Dz) <= tol * np.linalg.norm(Dz)


def test_superbase_is_obtuse_superbase():
    """Proposition (MakeObtuse): e0 + e1 + e2 + e3 = 0, |det(e1,e2,e3)| = 1
    and <e_i, D e_j> <= 0 for i != j; Selling offsets are c_ij = e_k x e_l."""
    for D in _fields():
        sb, st = oracle.superbase3d(D)
        assert st.max() == 0
        off, w, _ = oracle.stencil3d(D)
        pairs = [(0, 1, 2, 3), (0, 2, 1, 3), (0, 3, 1, 2), (1, 2, 0, 3), (1, 3, 0, 2), (2, 3, 0, 1)]
        for z in range(0, D.shape[1], 5):
            e = [sb[i, :, z].astype(np.float64) for i in range(4)]
            assert np.all(e[0] + e[1] + e[2] + e[3] == 0)
            assert abs(round(np.linalg.det(np.array(e[1:])))) == 1
            Dz = _mat(D, z)
            scale = np.abs(Dz).max()
            for i in range(4):
                for j in range(i + 1, 4):
                    tol = 1e-12 * scale * (1 + e[i] @ e[i]) * (1 + e[j] @ e[j])
                    assert e[i] @ Dz @ e[j] <= tol
            for q, (i, j, k, l) in enumerate(pairs):
                assert np.all(off[q, :, z] == np.cross(e[k], e[l]))


def test_greedy_basis_equals_brute_force_minima():
    """Definition 2: the greedy output attains the successive minima
    lambda_1..lambda_3 of Z^3 under D, found by enumeration (tiny kappa)."""
    D = synth.random_spd3(33, 120, 4.0)
    b, st = oracle.reduce3d(D)
    assert st.max() == 0
    for z in range(D.shape[1]):
        Dz = _mat(D, z)
        sm = brute.successive_minima(Dz)
        nb = np.array([b[i, :, z] @ Dz @ b[i, :, z] for i in range(3)], dtype=float)
        assert np.allclose(nb, sm, rtol=1e-12, atol=0)


def test_reduced_basis_inequality_lemma4():
    """Lemma 4 for d = 3: 2|<e_i, D e_j>| <= |e_i|_D^2 for i < j."""
    D = synth.random_spd3(34, 1000, 50.0)
    b, _ = oracle.reduce3d(D)
    for z in range(0, D.shape[1], 3):
        Dz = _mat(D, z)
        e = [b[i, :, z].astype(np.float64) for i in range(3)]
        for i in range(3):
            for j in range(i + 1, 3):
                tol = 1e-12 * np.abs(Dz).max() * (1 + e[i] @ e[i]) * (1 + e[j] @ e[j])
                assert 2 * abs(e[i] @ Dz @ e[j]) <= e[i] @ Dz @ e[i] + tol


def test_weight_function_same_for_every_obtuse_superbase():
    """Every D-obtuse superbase found by enumeration gives the oracle's
    weight function (the 3D analogue of Lemma 5, checked by brute force on
    tiny anisotropy; the paper proves it only in 2D)."""
    D = synth.random_spd3(35, 10, 1.8)
    off, w, _ = oracle.stencil3d(D)
    found = 0
    for z in range(D.shape[1]):
        Dz = _mat(D, z)
        ref = brute.weight_function(off[:, :, z], w[:, z])
        for sb in brute.obtuse_superbases_3d(Dz, box=1):
            found += 1
            o, ws = brute.selling_weights_3d(Dz, sb)
            wf = brute.weight_function(o, ws)
            keys = set(wf) | set(ref)
            assert max(abs(wf.get(k, 0.0) - ref.get(k, 0.0)) for k in keys) <= 1e-12
    assert found >= 10


def test_invalid_tensors_flagged():
    D = np.zeros((6, 3))
    D[0], D[3], D[5] = [1.0, -1.0, np.inf], [1.0, 1.0, 1.0], [1.0, 1.0, 1.0]
    _, w, st = oracle.stencil3d(D)
    assert st[0] == 0 and st[1] & 1 and st[2] & 1
    assert np.all(w[:, 1:] == 0)
