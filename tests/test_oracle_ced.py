"""Pins of the oracle's structure-tensor diffusion tensor (CED / EED).

The paper's only CED number (the largest eigenvalue at t = 0, Table on the
fingerprint) needs an image that is not available.  What the paper and the
mathematics fix is pinned here instead:
- properties: SPD with eigenvalues in [alpha, 1] and anisotropy
  <= alpha^-1/2, D = alpha Id on a flat image, the coherence direction along
  straight stripes, transpose covariance;
- values: the whole pipeline against scipy's mirrored Gaussian filter and
  numpy's eigensolver (2D and 3D), and against closed forms on cosine
  images for which every stage is exact, with three distinct eigenvalues in
  3D so that the eigenvalue assignment is checked.
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
    """Section 4 (CED): eigenvalues of D are alpha and
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
    """3D CED (Section 4, 3D experiments): spectrum in [alpha, 1]; EED
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


# ----------------------------------------------------------------------------
# Value pins of the whole pipeline (Section 4: u_sigma = K_sigma * u,
# J = K_rho * (grad u_sigma grad u_sigma^T), eigenvalue map).  Two
# independent routes: a library one (scipy's Gaussian filter with mirror
# extension, numpy's symmetric eigensolver) on a generic image, and a closed
# form on images for which every stage is exact.

def _taps(s):
    r = math.ceil(3.0 * s)
    j = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-j * j / (2.0 * s * s))
    return j, g / g.sum(), r


def _eigmap(J, alpha, C, eig_map):
    """D from J (..., d, d) by the eigenvalue map of Section 4 (CED) or the
    edge-enhancing map, eigenvalues taken in descending order."""
    mu, V = np.linalg.eigh(J)          # ascending
    mu, V = mu[..., ::-1], V[..., :, ::-1]
    d = J.shape[-1]
    lam = np.empty_like(mu)
    if eig_map == oracle.CED:
        lam[..., 0] = alpha
        for k in range(1, d):
            dm = mu[..., 0] - mu[..., k]
            with np.errstate(divide="ignore"):
                e = np.where(dm == 0, 0.0, np.exp(-C / np.where(dm == 0, 1.0, dm) ** 2))
            lam[..., k] = alpha + (1 - alpha) * e
    else:
        for k in range(d - 1):
            m = mu[..., k]
            lam[..., k] = np.where(m == 0, 1.0, 1 - np.exp(-C / np.where(m == 0, 1.0, m) ** 2))
        lam[..., d - 1] = 1.0
    return np.einsum("...ik,...k,...jk->...ij", V, lam, V)


def _planes(Dm, dim):
    idx = [(0, 0), (0, 1), (1, 1)] if dim == 2 else \
        [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    return np.stack([Dm[..., a, b].reshape(-1) for a, b in idx])


def _scipy_pipeline(u, dims, sigma, rho, alpha, C, eig_map):
    """u: one image, or (C, N) components whose products g g^T are summed
    before the rho blur."""
    from scipy import ndimage
    dim = len(dims)
    blur = lambda f, s: ndimage.gaussian_filter(f, s, mode="reflect",
                                                radius=math.ceil(3 * s))
    prods = {}
    for comp in np.asarray(u).reshape(-1, int(np.prod(dims))):
        a = comp.reshape(dims[::-1])           # axes (z,) y, x
        pad = np.pad(blur(a, sigma), 1, mode="symmetric")  # half-sample mirror
        g = []
        for c in range(dim):                   # c = 0 is x, the last array axis
            ax = dim - 1 - c
            hi = [slice(1, -1)] * dim
            lo = [slice(1, -1)] * dim
            hi[ax], lo[ax] = slice(2, None), slice(None, -2)
            g.append(0.5 * (pad[tuple(hi)] - pad[tuple(lo)]))
        for i in range(dim):
            for j in range(i, dim):
                prods[i, j] = prods.get((i, j), 0.0) + g[i] * g[j]
    J = np.empty(tuple(dims[::-1]) + (dim, dim))
    for (i, j), pij in prods.items():
        J[..., i, j] = J[..., j, i] = blur(pij, rho)
    return _planes(_eigmap(J, alpha, C, eig_map), dim)


def test_ced2d_matches_scipy_gaussian_pipeline():
    """2D CED tensor of a generic image = the same definition evaluated by
    scipy.ndimage.gaussian_filter (mode 'reflect' is the half-sample mirror,
    radius ceil(3 s)) + mirrored central differences + numpy's eigh.  sigma
    = 1.5 and rho = 2.5 separate the readings: a variance instead of a
    standard deviation, unnormalized taps or another truncation radius each
    move D by far more than the tolerance."""
    dims = (41, 37)
    u = synth.ced_image2d(77, *dims, ndiscs=3)
    sig, rho, C = 1.5, 2.5, 1e-6
    D = oracle.structure_tensor_d(u, dims, sig, rho, ALPHA, C)
    R = _scipy_pipeline(u, dims, sig, rho, ALPHA, C, oracle.CED)
    assert np.abs(D - R).max() <= 1e-12


def test_ced3d_matches_scipy_gaussian_pipeline():
    """The same library cross-check in 3D, CED and edge-enhancing maps, on
    a volume of 3D synthetic type (Section 4, 3D experiments)."""
    dims = (15, 13, 12)
    rng = np.random.default_rng(9)
    u = synth.ced_image3d(4, 15)[: np.prod(dims)] + 0.1 * rng.standard_normal(np.prod(dims))
    sig, rho = 1.5, 2.5
    for eig_map, C in ((oracle.CED, 1e-7), (oracle.EED, 1e-6)):
        D = oracle.structure_tensor_d(u, dims, sig, rho, ALPHA, C, eig_map)
        R = _scipy_pipeline(u, dims, sig, rho, ALPHA, C, eig_map)
        assert np.abs(D - R).max() <= 1e-12, eig_map


def _closed_form_J(dims, a, b, m, sigma, rho):
    """Closed-form J for u = a cos(kx x') + b cos(ky y') (x' = x + 1/2,
    k = pi m / n): these cosines are even about both mirror points, so the
    mirrored Gaussian acts on them as the discrete transfer function
    G_s(k) = sum_j g_j cos(k j), and the central difference of cos(k x') is
    -sin(k) sin(k x').  J_xy is exact only where the rho-kernel stays in the
    grid.  Returns J (..., 3, 3) on the grid and the interior mask."""
    nx, ny = dims[0], dims[1]
    kx, ky = math.pi * m[0] / nx, math.pi * m[1] / ny
    G = lambda s, k: float(np.dot(_taps(s)[1], np.cos(k * _taps(s)[0])))
    Ax = a * G(sigma, kx) * math.sin(kx)
    Ay = b * G(sigma, ky) * math.sin(ky)
    shape = dims[::-1]
    idx = np.indices(shape)
    xp, yp = idx[-1] + 0.5, idx[-2] + 0.5
    J = np.zeros(shape + (3, 3))
    J[..., 0, 0] = 0.5 * Ax * Ax * (1 - G(rho, 2 * kx) * np.cos(2 * kx * xp))
    J[..., 1, 1] = 0.5 * Ay * Ay * (1 - G(rho, 2 * ky) * np.cos(2 * ky * yp))
    J[..., 0, 1] = J[..., 1, 0] = (Ax * Ay * G(rho, kx) * G(rho, ky)
                                   * np.sin(kx * xp) * np.sin(ky * yp))
    r = _taps(rho)[2]
    inner = ((idx[-1] >= r) & (idx[-1] < nx - r) & (idx[-2] >= r) & (idx[-2] < ny - r))
    return J, inner


def test_ced3d_closed_form_three_distinct_eigenvalues():
    """3D eigenvalue assignment (Section 4, 3D CED; edge-enhancing map).
    For u = a cos(kx x') + b cos(ky y'), constant in z, J is known in closed
    form: mu_3 = 0 on e_z, and mu_1 > mu_2 > 0 in the x-y plane.  C is set
    so that the three CED eigenvalues alpha, lambda_2, lambda_3 are far
    apart; an ascending sort, or lambda_2 and lambda_3 exchanged, moves D by
    O(1).  Expected D = sum lambda_k v_k v_k^T from the closed-form J."""
    dims = (40, 36, 6)
    a, b, m = 1.0, 0.6, (5, 4)
    sig, rho = 1.0, 2.0
    x = np.arange(dims[0]) + 0.5
    y = np.arange(dims[1]) + 0.5
    ux = a * np.cos(math.pi * m[0] / dims[0] * x)
    uy = b * np.cos(math.pi * m[1] / dims[1] * y)
    u = np.broadcast_to(ux[None, None, :] + uy[None, :, None], dims[::-1]).reshape(-1).copy()
    J, inner = _closed_form_J(dims, a, b, m, sig, rho)
    mu = np.linalg.eigvalsh(J[inner])[:, ::-1]
    assert np.all(mu[:, 2] == 0) and np.all(mu[:, 1] > 0.05 * mu[:, 0])
    C = float(np.median((mu[:, 0] - mu[:, 1]) ** 2))
    for eig_map in (oracle.CED, oracle.EED):
        Cm = C if eig_map == oracle.CED else float(np.median(mu[:, 1] ** 2))
        D = oracle.structure_tensor_d(u, dims, sig, rho, ALPHA, Cm, eig_map)
        E = _planes(_eigmap(J, ALPHA, Cm, eig_map), 3)
        sel = inner.reshape(-1)
        assert np.abs(D[:, sel] - E[:, sel]).max() <= 1e-10, eig_map
        # the assignment matters: at a good share of these points the three
        # eigenvalues of D are 0.1 apart, so any other assignment moves D by
        # at least that much there
        lam = np.linalg.eigvalsh(_eigmap(J[inner], ALPHA, Cm, eig_map))
        assert np.mean(np.min(np.diff(lam, axis=-1), axis=-1) > 0.1) > 0.3, eig_map


def test_ced2d_closed_form():
    """2D counterpart of the closed form (Section 4, CED): distinct mu_1 >
    mu_2 at interior points, lambda_1 = alpha across the structure."""
    dims = (44, 38)
    a, b, m = 1.0, 0.7, (6, 5)
    sig, rho = 1.5, 2.5
    x = np.arange(dims[0]) + 0.5
    y = np.arange(dims[1]) + 0.5
    u = (a * np.cos(math.pi * m[0] / dims[0] * x)[None, :]
         + b * np.cos(math.pi * m[1] / dims[1] * y)[:, None]).reshape(-1)
    J3, inner = _closed_form_J(dims + (1,), a, b, m, sig, rho)
    J = J3[0, :, :, :2, :2]
    inner = inner[0]
    mu = np.linalg.eigvalsh(J[inner])
    C = float(np.median((mu[:, 1] - mu[:, 0]) ** 2))
    D = oracle.structure_tensor_d(u, dims, sig, rho, ALPHA, C)
    E = _planes(_eigmap(J, ALPHA, C, oracle.CED), 2)
    sel = inner.reshape(-1)
    assert np.abs(D[:, sel] - E[:, sel]).max() <= 1e-10


# ----------------------------------------------------------------------------
# Vector-valued images (the Conclusion: the components share one tensor, the
# coupling is the tensor's).  The oracle sums the components' products
# grad u_c,sigma grad u_c,sigma^T before the rho blur.

def test_vector_tensor_matches_scipy_pipeline():
    """Three components, 2D and 3D, CED and edge-enhancing maps: the summed
    tensor equals the library route with the same sum."""
    for dims, mk in (((41, 37), lambda k: synth.ced_image2d(70 + k, 41, 37, ndiscs=3)),
                     ((15, 13, 12), lambda k: synth.uniform(80 + k, 15 * 13 * 12))):
        u = np.stack([mk(k).reshape(-1) for k in range(3)])
        for eig_map, C in ((oracle.CED, 1e-6), (oracle.EED, 1e-6)):
            D = oracle.structure_tensor_d(u, dims, 1.5, 2.5, ALPHA, C, eig_map)
            R = _scipy_pipeline(u, dims, 1.5, 2.5, ALPHA, C, eig_map)
            assert np.abs(D - R).max() <= 1e-12, (dims, eig_map)


def test_vector_tensor_sums_outer_products():
    """Components u and a u give the tensor of sqrt(1 + a^2) u: the products
    add (a sum of gradients before the product would give (1 + a)^2), and
    the CED map sees the scale through C / (mu_1 - mu_2)^2."""
    dims = (48, 40)
    u = synth.uniform(5, 48 * 40)
    a, C = 0.75, 1e-6       # C near (mu_1 - mu_2)^2 of this noise
    D2 = oracle.structure_tensor_d(np.stack([u, a * u]), dims, 1.0, 3.0, ALPHA, C)
    D1 = oracle.structure_tensor_d(math.sqrt(1 + a * a) * u, dims, 1.0, 3.0, ALPHA, C)
    Dw = oracle.structure_tensor_d((1 + a) * u, dims, 1.0, 3.0, ALPHA, C)
    assert np.abs(D2 - D1).max() <= 1e-12
    assert np.abs(D2 - Dw).max() > 0.1
    # a zero component changes nothing
    Dz = oracle.structure_tensor_d(np.stack([u, np.zeros(u.size)]), dims, 1.0, 3.0, ALPHA, C)
    D0 = oracle.structure_tensor_d(u, dims, 1.0, 3.0, ALPHA, C)
    assert np.array_equal(Dz, D0)


def test_vector_tensor_orthogonal_ramps_isotropic():
    """u_1 = x, u_2 = y: away from the mirrored border each component's
    gradient is a unit axis vector, their products sum to Id, so mu_1 = mu_2
    and the CED map gives D = alpha Id; either ramp alone gives the coherence
    direction along the other axis."""
    nx, ny = 40, 36
    x = np.tile(np.arange(nx, dtype=np.float64), ny)
    y = np.repeat(np.arange(ny, dtype=np.float64), nx)
    sig, rho = 1.0, 2.0
    D = oracle.structure_tensor_d(np.stack([x, y]), (nx, ny), sig, rho, ALPHA, 1e-3)
    m = math.ceil(3 * sig) + math.ceil(3 * rho) + 1
    inner = ((x >= m) & (x < nx - m) & (y >= m) & (y < ny - m))
    assert inner.sum() > 100
    assert np.allclose(D[0][inner], ALPHA, rtol=1e-12, atol=0)
    assert np.abs(D[1][inner]).max() <= 1e-12
    assert np.allclose(D[2][inner], ALPHA, rtol=1e-12, atol=0)
    Dx = oracle.structure_tensor_d(x, (nx, ny), sig, rho, ALPHA, 1e-3)
    lam2 = ALPHA + (1 - ALPHA) * math.exp(-1e-3)
    assert np.allclose(Dx[0][inner], ALPHA, rtol=1e-12)
    assert np.allclose(Dx[2][inner], lam2, rtol=1e-12)
