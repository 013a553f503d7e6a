"""Pins of the 2D oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  A plausible mistake in the oracle
(a dropped term, a wrong sign, a transposed operand, a wrong normalization)
fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1301_3925_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return rows


def _mat(D, z):
    return np.array([[D[0, z], D[1, z]], [D[1, z], D[2, z]]])


def _interior_row(k2, n=16):
    D = synth.tensor2d_const(math.pi / 6, math.sqrt(k2), n * n)
    off, w, st = oracle.stencil2d(D)
    assert st.max() == 0
    A = oracle.operator_matrix((n, n), off, w)
    z = n // 2 + n * (n // 2)
    row = A.getrow(z)
    coef = {}
    for c, v in zip(row.indices, row.data):
        coef[(int(c % n) - n // 2, int(c // n) - n // 2)] = float(v)
    return coef


def test_tables_1_2_adlbr_coefficients():
    """Tables 1-2, AD-LBR rows: stencil coefficients of -div(D grad) for
    D = R(pi/6) diag(1, kappa^-2) R(pi/6)^T (eq. (def:DTest)), to the printed
    2 decimals.  Pins the Lagrange reduction, the obtuse sign fix, the Lemma 1
    weights and the operator normalization A = 1/2 grad E_h together."""
    rows = _read_rows("table1_2_adlbr_coefficients.txt")
    by_k = {}
    for k2, dx, dy, c in rows:
        by_k.setdefault(k2, []).append((int(dx), int(dy), c))
    assert sorted(by_k) == [1, 2, 10, 50]
    for k2, entries in by_k.items():
        coef = _interior_row(k2)
        for dx, dy, printed in entries:
            got = coef.get((dx, dy), 0.0)
            assert abs(got - printed) <= 0.005 + 1e-9, (k2, dx, dy, got, printed)
        # the full stencil has 6 off-centre points (+ centre)
        assert len([v for k, v in coef.items() if k != (0, 0) and v != 0.0]) <= 6


def test_table_3_lambda_max():
    """Table 3, AD-LBR row: largest eigenvalue of -div(D grad) for the
    same four tensors (periodic grid, so the constant-coefficient spectrum
    is sampled on the 2 pi k / n frequencies)."""
    import scipy.sparse.linalg as sla
    for k2, ref in _read_rows("table3_lambda_max.txt"):
        n = 64
        D = synth.tensor2d_const(math.pi / 6, math.sqrt(k2), n * n)
        off, w, _ = oracle.stencil2d(D)
        A = oracle.operator_matrix((n, n), off, w, periodic=True)
        lam = sla.eigsh(A, k=1, which="LA", tol=1e-10)[0][0]
        assert abs(lam - ref) <= 0.005 + 1e-9, (k2, lam, ref)


def test_fig_radius_kappa10():
    """Stencil-radius figure: for kappa = 10 the AD-LBR radius over all
    orientations does not exceed 5.1 (and reaches it); the Remark on stencil
    radius bounds it by kappa."""
    (kappa, rmax), = _read_rows("fig_radius.txt")
    th = np.linspace(0.0, math.pi, 4001)
    D = synth.tensor2d_from_angle(th, kappa)
    off, w, st = oracle.stencil2d(D)
    assert st.max() == 0
    r = np.sqrt((off.astype(np.float64) ** 2).sum(1))
    r = np.where(w > 0, r, 0.0).max(0)  # zero-weight slots are not in V(z)
    assert r.max() <= rmax + 1e-9
    assert r.max() >= rmax - 0.01
    assert np.all(r <= kappa)


def test_fig_eigen_tensor_exact_stencil():
    """D = [[19/2, 6], [6, 4]] (spectral-convergence figure): slots +-(1,1),
    +-(2,1), +-(3,2) with weights exactly 1/2, 1/2, 1/4."""
    rows = _read_rows("fig_eigen_tensor.txt")
    D = np.array(rows[0]).reshape(3, 1)
    off, w, st = oracle.stencil2d(D)
    wf = brute.weight_function(off[:, :, 0], w[:, 0])
    want = {}
    for sx, sy, g in rows[1:]:
        o = (int(sx), int(sy))
        want[max(o, (-o[0], -o[1]))] = g
    assert wf == want  # bit-exact rationals


def test_fig_eigen_spectral_convergence():
    """Spectral correctness (Section 1, and the figure on the seven smallest
    eigenvalues): on the periodic unit square with h = 1/n, the smallest
    eigenvalues of h^-2 A converge to those of -div(D grad), i.e.
    4 pi^2 <k, D k> for k in Z^2."""
    D0 = np.array([[9.5, 6.0], [6.0, 4.0]])
    ks = [(a, b) for a in range(-4, 5) for b in range(-4, 5)]
    cont = np.sort([4 * math.pi ** 2 * np.array(k) @ D0 @ np.array(k) for k in ks])[:7]
    errs = []
    for n in (16, 32):
        D = np.repeat(np.array([[9.5], [6.0], [4.0]]), n * n, axis=1)
        off, w, _ = oracle.stencil2d(D)
        A = oracle.operator_matrix((n, n), off, w, periodic=True).toarray() * n * n
        ev = np.sort(np.linalg.eigvalsh(A))[:7]
        errs.append(np.max(np.abs(ev - cont) / np.maximum(cont, 1.0)))
    assert errs[1] < errs[0]
    assert errs[1] < 0.05


def test_identity_and_diagonal():
    """D = Id gives the 5-point Laplacian (Table 1, kappa = 1); a diagonal D
    gives weights Dxx/2, Dyy/2 on the axes and 0 on the third slot."""
    D = np.array([[1.0, 3.0, 0.25], [0.0, 0.0, 0.0], [1.0, 0.5, 2.0]])
    off, w, st = oracle.stencil2d(D)
    for z in range(3):
        wf = brute.weight_function(off[:, :, z], w[:, z])
        assert wf == {(1, 0): D[0, z] / 2, (0, 1): D[2, z] / 2}


def _random_fields():
    return [synth.random_spd2(7, 3000, 10.0), synth.random_spd2(8, 3000, 200.0),
            synth.tensor2d_field(1301, 64, 64, 10.0)]


def test_decomposition_identity_and_nonnegativity():
    """Eq. (DSum) via Lemma 1: sum_{e in V(z)} gamma(e) e e^T = D(z) to 1e-12
    relative (scaled by r^4 eps for stencil radius r > 10, since each weight
    is a difference of products of size |D| r^2); gamma >= 0; at most 6
    offsets."""
    for D in _random_fields():
        off, w, st = oracle.stencil2d(D)
        assert st.max() == 0
        assert np.all(w >= 0.0)
        o = off.astype(np.float64)
        S = np.zeros_like(D)
        for i in range(3):
            S[0] += 2 * w[i] * o[i, 0] * o[i, 0]
            S[1] += 2 * w[i] * o[i, 0] * o[i, 1]
            S[2] += 2 * w[i] * o[i, 1] * o[i, 1]
        norm = np.sqrt(D[0] ** 2 + 2 * D[1] ** 2 + D[2] ** 2)
        err = np.sqrt((S[0] - D[0]) ** 2 + 2 * (S[1] - D[1]) ** 2 + (S[2] - D[2]) ** 2)
        r2 = (o * o).sum(1).max(0)
        tol = np.maximum(1e-12, 1e-16 * r2 * r2)
        assert np.all(err / norm <= tol)
        assert np.max(np.where(r2 <= 100, err / norm, 0.0)) <= 1e-12


def test_obtuse_superbase_and_reduction_inequalities():
    """The slots form an M-obtuse superbase of Z^2 (Definition; Corollary 2):
    e + f + g = 0, |det(e, f)| = 1, pairwise <.,M.> <= 0, with the Corollary 2
    margins <e, M g> <= -|e|^2/2; the reduced pair satisfies Lemma 4,
    2|<e, M f>| <= |e|_M^2, and |e|_M <= |f|_M."""
    for D in _random_fields():
        off, w, _ = oracle.stencil2d(D)
        basis, it = oracle.reduce2d(D)
        for z in range(0, D.shape[1], 7):
            Dz = _mat(D, z)
            Q = np.array([[Dz[1, 1], -Dz[0, 1]], [-Dz[0, 1], Dz[0, 0]]])
            e, f, g = [off[i, :, z].astype(np.float64) for i in range(3)]
            assert np.all(e + f + g == 0)
            assert abs(e[0] * f[1] - e[1] * f[0]) == 1
            tol = 1e-12 * np.abs(Q).max() * (1 + e @ e + f @ f + g @ g)
            assert e @ Q @ f <= tol and f @ Q @ g <= tol and g @ Q @ e <= tol
            assert e @ Q @ g <= -0.5 * (e @ Q @ e) + tol
            assert f @ Q @ g <= -0.5 * (f @ Q @ f) + tol
            a, b = basis[0, :, z].astype(float), basis[1, :, z].astype(float)
            assert a @ Q @ a <= b @ Q @ b + tol
            assert 2 * abs(a @ Q @ b) <= a @ Q @ a + tol


def test_reduced_basis_equals_brute_force_minima():
    """Definition 2: the Lagrange output (e, f) attains the successive
    minima lambda_1, lambda_2 of Z^2 under M, found by enumerating every
    integer vector in a provably sufficient box (tiny kappa)."""
    D = synth.random_spd2(21, 150, 6.0)
    basis, it = oracle.reduce2d(D)
    for z in range(D.shape[1]):
        Dz = _mat(D, z)
        Q = np.array([[Dz[1, 1], -Dz[0, 1]], [-Dz[0, 1], Dz[0, 0]]])
        sm = brute.successive_minima(Q)
        nb = np.array([basis[i, :, z] @ Q @ basis[i, :, z] for i in range(2)], dtype=float)
        assert np.allclose(nb, sm, rtol=1e-12, atol=0)


def test_mu_identity():
    """mu(M) = |<e, M f>| = sqrt(lambda_1^2 lambda_2^2 - det M) for a
    reduced basis (eq. (def:orth)), with lambda_i from brute force."""
    D = synth.random_spd2(22, 60, 6.0)
    basis, _ = oracle.reduce2d(D)
    for z in range(D.shape[1]):
        Dz = _mat(D, z)
        M = np.sqrt(np.linalg.det(Dz)) * np.linalg.inv(Dz)  # det M = 1
        sm = brute.successive_minima(M)
        e, f = basis[0, :, z].astype(float), basis[1, :, z].astype(float)
        mu = abs(e @ M @ f)
        assert abs(mu - math.sqrt(max(sm[0] * sm[1] - np.linalg.det(M), 0.0))) <= 1e-9


def test_lemma5_weight_function_independent_of_superbase():
    """Lemma 5: every M-obtuse superbase gives the same weight function
    gamma_z on Z^2; enumerate them all among short vectors."""
    D = synth.random_spd2(23, 25, 4.0)
    off, w, _ = oracle.stencil2d(D)
    for z in range(D.shape[1]):
        Dz = _mat(D, z)
        ref = brute.weight_function(off[:, :, z], w[:, z])
        sbs = brute.obtuse_superbases_2d(Dz, box=5)
        assert len(sbs) >= 6
        for sb in sbs:
            wf = brute.weight_function(sb, brute.lemma1_weights_2d(Dz, sb))
            keys = set(wf) | set(ref)
            assert max(abs(wf.get(k, 0.0) - ref.get(k, 0.0)) for k in keys) <= 1e-12


def test_radius_bounded_by_kappa():
    """Remark on stencil radius: radius of V(z) bounded by kappa(D(z)).
    Reading: the bound holds for the reduced basis vectors e, f always, and
    for the whole stencil once kappa >= sqrt 2; a near-isotropic tensor
    gives the diagonal slot (length sqrt 2) a small positive weight, so there
    the radius is sqrt 2 > kappa."""
    D = synth.random_spd2(24, 5000, 200.0)
    off, w, _ = oracle.stencil2d(D)
    basis, _ = oracle.reduce2d(D)
    r = np.sqrt((off.astype(np.float64) ** 2).sum(1))
    r = np.where(w > 0, r, 0.0).max(0)
    rb = np.sqrt((basis.astype(np.float64) ** 2).sum(1)).max(0)
    ev = np.stack([np.linalg.eigvalsh(_mat(D, z)) for z in range(D.shape[1])])
    kappa = np.sqrt(ev[:, 1] / ev[:, 0])
    assert np.all(rb <= kappa * (1 + 1e-12))
    big = kappa >= math.sqrt(2.0)
    assert big.sum() > 1000
    assert np.all(r[big] <= kappa[big] * (1 + 1e-12))
    assert np.all(r <= math.sqrt(2.0) * np.maximum(kappa, 1.0) * (1 + 1e-12))


def test_lagrange_iterations_logarithmic():
    """The reduction costs O(ln kappa) iterations (Section 2)."""
    for kappa, cap in ((10.0, 6), (100.0, 8), (1000.0, 11)):
        th = np.linspace(0, math.pi, 2001)
        _, it = oracle.reduce2d(synth.tensor2d_from_angle(th, kappa))
        assert it.max() <= cap, (kappa, it.max())


def test_invalid_tensors_flagged():
    """Non-SPD or non-finite tensors are rejected, not silently used."""
    D = np.array([[1.0, -1.0, np.nan, 1.0], [0.0, 0.0, 0.0, 2.0], [1.0, 1.0, 1.0, 1.0]])
    _, w, st = oracle.stencil2d(D)
    assert st[0] == 0
    assert st[1] & 1 and st[2] & 1 and st[3] & 1
    assert np.all(w[:, 1:] == 0)
