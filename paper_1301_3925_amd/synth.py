"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It holds none of the method's arithmetic: it only draws tensor
fields D, initial images u0 and right-hand sides.  Every generator uses
numpy's PCG64 with an explicit seed, works in float64, and returns arrays in
the library's layout (structure-of-arrays planes, x fastest):

* 2D tensor field: shape (3, N) with planes (Dxx, Dxy, Dyy)
* 3D tensor field: shape (6, N) with planes (Dxx, Dxy, Dxz, Dyy, Dyz, Dzz)
* scalar fields: shape (N,), index = x + nx*(y + ny*z)

The paper's own images (a fingerprint, an MRI volume) are not available;
these recipes stand in for them with the same sizes and anisotropy ranges.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "smooth_field", "tensor2d_from_angle", "tensor2d_const", "tensor2d_field",
    "tensor3d_from_rotvec", "tensor3d_field", "uniform", "ced_image2d",
    "ced_image3d", "batch_problems", "random_spd2", "random_spd3", "overflow_field3d",
    "restoration_problem",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def smooth_field(rng: np.random.Generator, shape, nfreq: int = 8) -> np.ndarray:
    """Sum of `nfreq` random-phase sinusoids with integer frequencies in
    {-3..3}^d (per domain length), normalized to [-1, 1].

    `shape` is (nx, ny) or (nx, ny, nz); the result is flattened x-fastest.
    """
    d = len(shape)
    coords = np.meshgrid(*[np.arange(n, dtype=np.float64) / n for n in shape],
                         indexing="ij")
    acc = np.zeros(shape, dtype=np.float64)
    total = 0.0
    for _ in range(nfreq):
        while True:
            p = rng.integers(-3, 4, size=d)
            if np.any(p != 0):
                break
        a = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        phase = sum(2.0 * math.pi * p[k] * coords[k] for k in range(d))
        acc += a * np.sin(phase + phi)
        total += a
    acc /= total
    # meshgrid with indexing="ij" puts x first; flatten x-fastest
    return np.ascontiguousarray(acc.transpose(*reversed(range(d)))).reshape(-1)


def tensor2d_from_angle(theta: np.ndarray, kappa) -> np.ndarray:
    """D = R(theta) diag(1, kappa^-2) R(theta)^T, returned as (3, N)."""
    theta = np.asarray(theta, dtype=np.float64)
    kappa = np.broadcast_to(np.asarray(kappa, dtype=np.float64), theta.shape)
    c, s = np.cos(theta), np.sin(theta)
    l1, l2 = 1.0, 1.0 / (kappa * kappa)
    dxx = l1 * c * c + l2 * s * s
    dxy = (l1 - l2) * c * s
    dyy = l1 * s * s + l2 * c * c
    return np.stack([dxx, dxy, dyy]).astype(np.float64)


def tensor2d_const(theta: float, kappa: float, n: int = 1) -> np.ndarray:
    """Constant tensor R(theta) diag(1, kappa^-2) R(theta)^T on n points."""
    return tensor2d_from_angle(np.full(n, theta), kappa)


def tensor2d_field(seed: int, nx: int, ny: int, kappa: float) -> np.ndarray:
    """Smooth random orientation field theta = pi*S with anisotropy kappa."""
    rng = _rng(seed)
    theta = math.pi * smooth_field(rng, (nx, ny))
    return tensor2d_from_angle(theta, kappa)


def tensor3d_from_rotvec(omega: np.ndarray, evals: np.ndarray) -> np.ndarray:
    """D = R diag(evals) R^T with R = exp([omega]_x) (Rodrigues).

    omega: (3, N); evals: (3, N).  Returns (6, N) planes xx,xy,xz,yy,yz,zz.
    """
    omega = np.asarray(omega, dtype=np.float64)
    th = np.sqrt((omega * omega).sum(0))
    small = th < 1e-12
    ths = np.where(small, 1.0, th)
    k = omega / ths
    kx, ky, kz = k
    c, s = np.cos(th), np.sin(th)
    v = 1.0 - c
    R = np.empty((3, 3) + th.shape)
    R[0, 0] = c + kx * kx * v
    R[0, 1] = kx * ky * v - kz * s
    R[0, 2] = kx * kz * v + ky * s
    R[1, 0] = ky * kx * v + kz * s
    R[1, 1] = c + ky * ky * v
    R[1, 2] = ky * kz * v - kx * s
    R[2, 0] = kz * kx * v - ky * s
    R[2, 1] = kz * ky * v + kx * s
    R[2, 2] = c + kz * kz * v
    for a in range(3):
        for b in range(3):
            R[a, b] = np.where(small, 1.0 if a == b else 0.0, R[a, b])
    lam = np.asarray(evals, dtype=np.float64)
    out = np.empty((6,) + th.shape)
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for q, (a, b) in enumerate(idx):
        out[q] = sum(R[a, m] * lam[m] * R[b, m] for m in range(3))
    return out


def tensor3d_field(seed: int, n, kappa_max: float) -> np.ndarray:
    """Mixed needle / plate / isotropic field with anisotropy <= kappa_max.

    R(x) = exp([omega]_x) with omega = pi*(S1,S2,S3); eigenvalues
    (1, kb^-2, ka^-2) where ka = kappa_max^t, kb = ka^s, t = (1+S4)/2,
    s = (1+S5)/2.
    """
    if isinstance(n, int):
        n = (n, n, n)
    rng = _rng(seed)
    S = [smooth_field(rng, n) for _ in range(5)]
    omega = math.pi * np.stack(S[:3])
    t = 0.5 * (1.0 + S[3])
    s = 0.5 * (1.0 + S[4])
    ka = kappa_max ** t
    kb = ka ** s
    evals = np.stack([np.ones_like(ka), kb ** -2.0, ka ** -2.0])
    return tensor3d_from_rotvec(omega, evals)


def uniform(seed: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """u0 ~ U[lo, hi) in float64."""
    return _rng(seed).uniform(lo, hi, size=n)


def _gauss_smooth_noise(rng, shape, std_px):
    from scipy.ndimage import gaussian_filter  # input synthesis only
    xi = rng.standard_normal(shape)
    xi = gaussian_filter(xi, std_px, mode="wrap")
    xi /= xi.std()
    return xi


def ced_image2d(seed: int, nx: int, ny: int, period: float = 12.0,
                ndiscs: int = 40) -> np.ndarray:
    """Oriented stripe texture with smooth noise and interrupted lines.

    u0 = clip(0.5 + 0.3 sin(2 pi (x cos psi + y sin psi)/period)
              + 0.15 xi, 0, 1), psi = pi*S a low-frequency orientation field,
    xi smoothed (std 2 px) unit-variance noise; `ndiscs` discs of radius
    6..20 px are set to 0.5 to interrupt the stripes.
    """
    rng = _rng(seed)
    psi = (math.pi * smooth_field(rng, (nx, ny))).reshape(ny, nx)
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")
    stripes = np.sin(2.0 * math.pi * (x * np.cos(psi) + y * np.sin(psi)) / period)
    xi = _gauss_smooth_noise(rng, (ny, nx), 2.0)
    u = np.clip(0.5 + 0.3 * stripes + 0.15 * xi, 0.0, 1.0)
    for _ in range(ndiscs):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        r = rng.uniform(6.0, 20.0)
        u[(x - cx) ** 2 + (y - cy) ** 2 <= r * r] = 0.5
    return np.ascontiguousarray(u).reshape(-1)


def ced_image3d(seed: int, n: int, noise_var: float = 0.5) -> np.ndarray:
    """cos(2 (r/R)^3) + Gaussian noise of the given variance, r the distance
    to the cube centre, R = 1/2, on n^3 voxels of [0,1]^3."""
    rng = _rng(seed)
    c = (np.arange(n, dtype=np.float64) + 0.5) / n - 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    u = np.cos(2.0 * (r / 0.5) ** 3) + math.sqrt(noise_var) * rng.standard_normal(r.shape)
    return np.ascontiguousarray(u).reshape(-1)


def random_spd2(seed: int, n: int, kappa_max: float = 10.0) -> np.ndarray:
    """Independent random 2x2 SPD tensors: random angle, random
    anisotropy in [1, kappa_max], random scale in [0.1, 10]."""
    rng = _rng(seed)
    theta = rng.uniform(0, math.pi, n)
    kappa = np.exp(rng.uniform(0, math.log(kappa_max), n))
    scale = np.exp(rng.uniform(math.log(0.1), math.log(10.0), n))
    return tensor2d_from_angle(theta, kappa) * scale


def random_spd3(seed: int, n: int, kappa_max: float = 10.0) -> np.ndarray:
    """Independent random 3x3 SPD tensors with anisotropy <= kappa_max."""
    rng = _rng(seed)
    omega = rng.normal(size=(3, n))
    omega *= (rng.uniform(0, math.pi, n) / np.sqrt((omega ** 2).sum(0)))
    l2 = np.exp(-2.0 * rng.uniform(0, math.log(kappa_max), n))
    l3 = np.exp(-2.0 * rng.uniform(0, math.log(kappa_max), n))
    scale = np.exp(rng.uniform(math.log(0.1), math.log(10.0), n))
    evals = np.stack([np.ones(n), l2, l3]) * scale
    return tensor3d_from_rotvec(omega, evals)


def batch_problems(seed: int, n2d: int = 64, n3d: int = 8,
                   side2d=(256, 1536), side3d=(64, 192), kappa_max: float = 50.0):
    """Uneven batch: n2d square images and n3d cubic volumes.

    Returns a list of dicts {dim, n: (nx, ny[, nz]), seed, kappa}; the
    fields themselves are drawn by tensor2d_field / tensor3d_field on demand.
    """
    rng = _rng(seed)
    probs = []
    for i in range(n2d):
        s = int(rng.integers(side2d[0], side2d[1] + 1))
        k = float(rng.uniform(1.0, kappa_max))
        probs.append({"dim": 2, "n": (s, s), "seed": seed * 1000 + i, "kappa": k})
    for j in range(n3d):
        s = int(rng.integers(side3d[0], side3d[1] + 1))
        probs.append({"dim": 3, "n": (s, s, s), "seed": seed * 1000 + 500 + j,
                      "kappa": kappa_max})
    return probs


def overflow_field3d():
    """A 17^3 tensor field whose stencils nearly all reach the centre c: at
    every y with v = c - y primitive, D(y) = v v^T / |v|^2 + 1e-3 Id, a
    needle along v; elsewhere D = Id.  Returns (dims, D (6, N), index of c).
    It exercises the limit of 255 incoming edges per point."""
    n = (17, 17, 17)
    c = np.array([8, 8, 8])
    N = int(np.prod(n))
    idx = np.arange(N)
    P = np.stack([idx % n[0], (idx // n[0]) % n[1], idx // (n[0] * n[1])])
    D = np.zeros((6, N))
    for i in range(N):
        v = c - P[:, i]
        if math.gcd(math.gcd(int(abs(v[0])), int(abs(v[1]))), int(abs(v[2]))) != 1:
            M = np.eye(3)
        else:
            vh = v / np.linalg.norm(v)
            M = np.outer(vh, vh) + 1e-3 * np.eye(3)
        D[:, i] = [M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]]
    return n, D, int(c[0] + n[0] * (c[1] + n[1] * c[2]))


def restoration_problem(n: int, kappa: float, alpha: float = 1.0 / 3.0, sub: int = 32):
    """Inputs of the restoration experiment on the unit square, n x n pixels
    with centres z = ((i + 1/2)/n, (j + 1/2)/n): the tensor
    D = [[1, s], [s, s^2 + kappa^-2]], s = 2 pi alpha sin(2 pi x), at the
    centres, and the image v = v0 o f with v0 = 1_{y < 1/2} and
    f(x, y) = (x, y + alpha cos(2 pi x)), averaged over each pixel (the
    area fraction below the stripe's edge y = 1/2 - alpha cos(2 pi x),
    exact in y, `sub` samples per pixel in x).
    Returns (D (3, n*n), v (n*n,)) in the library's layout."""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    x = np.tile(c, n)
    s = 2.0 * math.pi * alpha * np.sin(2.0 * math.pi * x)
    D = np.stack([np.ones_like(x), s, s * s + kappa ** -2.0])
    xs = (np.arange(n * sub, dtype=np.float64) + 0.5) / (n * sub)
    edge = 0.5 - alpha * np.cos(2.0 * math.pi * xs)
    lo = np.arange(n, dtype=np.float64) / n
    frac = np.clip((edge[None, :] - lo[:, None]) * n, 0.0, 1.0)
    v = frac.reshape(n, n, sub).mean(axis=2).reshape(-1)
    return D, v
