"""Brute-force checkers on tiny inputs -- TEST INFRASTRUCTURE ONLY.

These pin the oracle to the mathematics independently of its own code:
  * successive minima of Z^d under a quadratic form, by enumerating every
    integer vector in a provably large enough box (Definition 2);
  * every obtuse superbase of Z^2 among short vectors, and the weight
    function each one defines (Lemma 1, Lemma 5);
  * every obtuse superbase of Z^3 among short vectors (Proposition
    (MakeObtuse), Selling's lemma) and its weight function;
  * the dense operator matrix read off the energy E_h by polarization
    (A = 1/2 grad E_h, eq. (def:E*)).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _box_radius(Q: np.ndarray) -> int:
    """Every vector reaching the d-th successive minimum lies in this box:
    lambda_d <= max_i |e_i|_Q over the canonical basis, and |v| <=
    |v|_Q / sqrt(lambda_min(Q))."""
    lmin = float(np.linalg.eigvalsh(Q).min())
    return int(math.ceil(math.sqrt(float(np.max(np.diag(Q))) / lmin))) + 1


def lattice_vectors(Q: np.ndarray):
    """All nonzero integer vectors in the box, sorted by Q-norm."""
    d = Q.shape[0]
    B = _box_radius(Q)
    rng = range(-B, B + 1)
    V = np.array([v for v in itertools.product(rng, repeat=d) if any(v)], dtype=np.int64)
    n2 = np.einsum("ki,ij,kj->k", V.astype(float), Q, V.astype(float))
    order = np.argsort(n2, kind="stable")
    return V[order], n2[order]


def successive_minima(Q: np.ndarray) -> np.ndarray:
    """Squared successive minima lambda_i(Q)^2, i = 1..d (Definition 2 for
    d <= 3, where they are attained by a basis)."""
    d = Q.shape[0]
    V, n2 = lattice_vectors(Q)
    chosen = []
    out = []
    for v, q in zip(V, n2):
        M = np.array(chosen + [v], dtype=float)
        if np.linalg.matrix_rank(M) == len(chosen) + 1:
            chosen.append(v)
            out.append(q)
            if len(chosen) == d:
                break
    return np.array(out)


def _weight_function(offsets, weights):
    """Canonical weight function: +-merged, zero weights dropped, as a dict
    {canonical offset: weight}."""
    wf = {}
    for o, w in zip(offsets, weights):
        o = tuple(int(c) for c in o)
        if w == 0.0 or not any(o):
            continue
        neg = tuple(-c for c in o)
        key = max(o, neg)
        wf[key] = wf.get(key, 0.0) + float(w)
    return wf


def weight_function(offsets, weights):
    return _weight_function(offsets, weights)


def obtuse_superbases_2d(D: np.ndarray, box: int = 6):
    """Every M-obtuse superbase (e, f, g) of Z^2 with entries in the box,
    M ~ adj(D) (Definition of obtuse superbase, Section 1)."""
    Q = np.array([[D[1, 1], -D[0, 1]], [-D[0, 1], D[0, 0]]])
    vs = [np.array(v) for v in itertools.product(range(-box, box + 1), repeat=2) if any(v)]
    out = []
    for e in vs:
        for f in vs:
            if abs(e[0] * f[1] - e[1] * f[0]) != 1:
                continue
            g = -e - f
            if e @ Q @ f <= 1e-12 and f @ Q @ g <= 1e-12 and g @ Q @ e <= 1e-12:
                out.append((e, f, g))
    return out


def lemma1_weights_2d(D: np.ndarray, sb):
    """gamma(+-e_i) = -1/2 <e_{i+1}^perp, D e_{i+2}^perp> (Lemma 1)."""
    perp = lambda v: np.array([-v[1], v[0]], dtype=float)
    w = []
    for i in range(3):
        a, b = sb[(i + 1) % 3], sb[(i + 2) % 3]
        w.append(-0.5 * perp(a) @ D @ perp(b))
    return w


def obtuse_superbases_3d(D: np.ndarray, box: int = 2):
    """Every D-obtuse superbase (e0..e3) of Z^3 with e1, e2, e3 in the box."""
    vs = [np.array(v) for v in itertools.product(range(-box, box + 1), repeat=3) if any(v)]
    G = {}
    out = []
    # all bases (e1, e2, e3) up to ordering: require e1 < e2 < e3 by index
    idx = range(len(vs))
    for i, j, k in itertools.combinations(idx, 3):
        e1, e2, e3 = vs[i], vs[j], vs[k]
        if abs(round(np.linalg.det(np.array([e1, e2, e3], dtype=float)))) != 1:
            continue
        e0 = -e1 - e2 - e3
        sb = [e0, e1, e2, e3]
        ok = True
        for a, b in itertools.combinations(range(4), 2):
            if sb[a] @ D @ sb[b] > 1e-12:
                ok = False
                break
        if ok:
            out.append(sb)
    del G
    return out


def selling_weights_3d(D: np.ndarray, sb):
    """Selling: gamma(e_k x e_l) = -1/2 <e_i, D e_j>, {i,j,k,l} = {0..3}."""
    offs, ws = [], []
    for i, j in itertools.combinations(range(4), 2):
        k, l = [m for m in range(4) if m not in (i, j)]
        offs.append(np.cross(sb[k], sb[l]))
        ws.append(-0.5 * sb[i] @ D @ sb[j])
    return offs, ws


def dense_operator_from_energy(energy, n: int) -> np.ndarray:
    """A with u^T A u = E(u) for the quadratic energy E, by polarization:
    A_ii = E(d_i), A_ij = (E(d_i + d_j) - E(d_i) - E(d_j)) / 2."""
    A = np.zeros((n, n))
    diag = np.zeros(n)
    for i in range(n):
        v = np.zeros(n)
        v[i] = 1.0
        diag[i] = energy(v)
        A[i, i] = diag[i]
    for i in range(n):
        for j in range(i + 1, n):
            v = np.zeros(n)
            v[i] = 1.0
            v[j] = 1.0
            a = 0.5 * (energy(v) - diag[i] - diag[j])
            A[i, j] = A[j, i] = a
    return A
