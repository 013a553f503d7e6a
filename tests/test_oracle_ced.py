"""Pins of the oracle's structure-tensor diffusion tensor (CED / EED).

The paper's only CED number (the largest eigenvalue at t = 0, Table on the
fingerprint) needs an image that is not available, so the values of the CED
tensor itself are "parity unpinned" by the paper.  What the paper and the
mathematics fix is pinned here: SPD with eigenvalues in [alpha, 1] and
anisotropy <= alpha^-1/2, D = alpha Id on a flat image, the coherence
direction along straight stripes, and exact invariance properties of the
Gaussian smoothing.
"""
import math

import numpy as np

import oracle
from paper_1301_3925_amd import synth

ALPHA, CC = 1e-2, 1e-5


def _eig2(D):
    a, b, c = D
    tr, det = a + c, a * c - b * b
    disc = np.sqrt(np.maximum((a - c) ** 2 / 4 + b * b, 0))
    return tr / 2 - disc, tr / 2 + disc


def test_ced2d_spd_eigen_range():
    """Section 5 (CED): eigenvalues of D are alpha and
    alpha + (1 - alpha) exp(-C/(mu1-mu2)^2), so D is SPD with spectrum in
    [alpha, 1] and kappa <= alpha^-1/2."""
    n = (96, 80)
    u = synth.ced_image2d(1302, *n)
    D = oracle.structure_tensor_d(u, n, 1.0, 4.0, ALPHA, CC)
    lo, hi = _eig2(D)
    assert np.all(lo >= ALPHA * (1 - 1e-12))
    assert np.all(hi <= 1 + 1e-12)
    assert np.all(np.sqrt(hi / lo) <= ALPHA ** -0.5 * (1 + 1e-9))
    assert np.sqrt(hi / lo).max() > 5.0  # the stripes do produce anisotropy


def test_ced_flat_image_gives_alpha_identity():
    """u constant => grad u_sigma = 0 => J = 0, mu1 = mu2 = 0, and with
    exp(-C/0) := 0 both eigenvalues are alpha: D = alpha Id."""
    for n in [(20, 17), (9, 8, 7)]:
        u = np.full(int(np.prod(n)), 0.37)
        D = oracle.structure_tensor_d(u, n, 1.0, 4.0, ALPHA, CC)
        diag = [0, 2] if len(n) == 2 else [0, 3, 5]
        offd = [1] if len(n) == 2 else [1, 2, 4]
        assert np.allclose(D[diag], ALPHA, rtol=1e-12, atol=0)
        assert np.all(np.abs(D[offd]) <= 1e-15)


def test_ced_straight_stripes_orientation():
    """Stripes u = sin(2 pi x / 8): the structure tensor's leading
    eigenvector is e_x (across the stripes) and gets lambda_1 = alpha; the
    coherence direction e_y gets nearly 1."""
    nx, ny = 64, 48
    x = np.tile(np.arange(nx, dtype=np.float64), ny)
    u = np.sin(2 * math.pi * x / 8.0)
    D = oracle.structure_tensor_d(u, (nx, ny), 0.5, 2.0, ALPHA, CC)
    inner = (x > 8) & (x < nx - 8)
    assert np.allclose(D[0][inner], ALPHA, rtol=1e-9)
    assert np.all(np.abs(D[1][inner]) < 1e-12)
    assert np.all(D[2][inner] > 0.99)


def test_ced3d_spd_eigen_range_and_eed():
    """3D CED (Section 5, 3D experiments): spectrum in [alpha, 1]; EED
    tensor: lambda_3 = 1 and the others in (0, 1]."""
    n = (16, 16, 16)
    u = synth.ced_image3d(2003, 16)
    for eig_map in (oracle.CED, oracle.EED):
        D = oracle.structure_tensor_d(u, n, 0.5, 2.0, ALPHA, 1e-3, eig_map)
        for z in range(0, D.shape[1], 37):
            M = np.array([[D[0, z], D[1, z], D[2, z]], [D[1, z], D[3, z], D[4, z]],
                          [D[2, z], D[4, z], D[5, z]]])
            ev = np.linalg.eigvalsh(M)
            if eig_map == oracle.CED:
                assert ev[0] >= ALPHA * (1 - 1e-9) and ev[2] <= 1 + 1e-9
            else:
                assert ev[0] > 0 and abs(ev[2] - 1.0) <= 1e-9


def test_ced_rotation_covariance():
    """Transposing the image (x <-> y) transposes the tensor field:
    D'(y, x) = P D(x, y) P with P the swap.  Catches a blur or gradient
    applied along the wrong axis."""
    nx, ny = 40, 40
    u = synth.ced_image2d(5, nx, ny, ndiscs=3)
    D = oracle.structure_tensor_d(u, (nx, ny), 1.0, 3.0, ALPHA, CC)
    uT = u.reshape(ny, nx).T.copy().reshape(-1)
    DT = oracle.structure_tensor_d(uT, (ny, nx), 1.0, 3.0, ALPHA, CC)
    sw = lambda a: a.reshape(ny, nx).T.reshape(-1)
    assert np.allclose(DT[0], sw(D[2]), atol=1e-12)
    assert np.allclose(DT[1], sw(D[1]), atol=1e-12)
    assert np.allclose(DT[2], sw(D[0]), atol=1e-12)
