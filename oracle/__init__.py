"""AD-LBR FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the benchmark's cpu_baseline leg
import this package.  The HIP library never calls it and shares no code with
it.  Parity tests compare the HIP path against these functions.

What lives where:
  adlbr_oracle.c   stencils (2D Lagrange + obtuse superbase + Lemma 1
                   weights; 3D greedy reduction + MakeObtuse + Selling),
                   COO scatter of the operator, structure-tensor D (CED/EED)
  this module      ctypes wrappers, the operator as a scipy sparse matrix,
                   explicit Euler, CFL, energy E_h by its definition
  brute.py         brute-force checks on tiny inputs (successive minima,
                   obtuse-superbase enumeration, dense operator from E_h)
  solvers.py       Jacobi-PCG / flexible CG / the CNN preconditioner (FP64)

Every function cites the passage of the paper it follows.  Functions that no
paper value, closed form or brute force pins say "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adlbr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=c99", "-Wall"]


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.or_reduce2d.argtypes = [P, I64, P, P]
        lib.or_stencil2d.argtypes = [P, I64, P, P, P]
        lib.or_reduce3d.argtypes = [P, I64, P, P]
        lib.or_superbase3d.argtypes = [P, I64, P, P]
        lib.or_stencil3d.argtypes = [P, I64, P, P, P]
        lib.or_operator_coo.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P, P, P]
        lib.or_operator_coo.restype = I64
        lib.or_structure_tensor_d.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(D):
    return np.ascontiguousarray(D, dtype=np.float64)


# ------------------------------------------------------------- stencils --

def reduce2d(D):
    """Lagrange-reduced basis (e, f) for the metric of each 2D tensor
    (Section 2, eq. (GaussAlgo), from the canonical basis).
    Returns basis int64 (2, 2, N) [vector][component][point] and iterations."""
    D = _f64(D)
    n = D.shape[1]
    basis = np.zeros((2, 2, n), np.int64)
    it = np.zeros(n, np.int32)
    _load().or_reduce2d(_p(D), n, _p(basis), _p(it))
    return basis, it


def stencil2d(D):
    """2D AD-LBR stencils (Section 1, eqs. (def:Vz), (def:GammaZ);
    construction steps (i)-(iii) of Section 2).
    Returns offsets int16 (3, 2, N), weights f64 (3, N), status int32 (N,)."""
    D = _f64(D)
    n = D.shape[1]
    off = np.zeros((3, 2, n), np.int16)
    w = np.zeros((3, n), np.float64)
    st = np.zeros(n, np.int32)
    _load().or_stencil2d(_p(D), n, _p(off), _p(w), _p(st))
    return off, w, st


def reduce3d(D):
    """Greedy D-reduced basis of Z^3 (Definition 2; the algorithm of the
    references cited in Section 2).  Returns (3, 3, N) int64 and status."""
    D = _f64(D)
    n = D.shape[1]
    b = np.zeros((3, 3, n), np.int64)
    st = np.zeros(n, np.int32)
    _load().or_reduce3d(_p(D), n, _p(b), _p(st))
    return b, st


def superbase3d(D):
    """D-obtuse superbase (e0..e3) from Proposition (MakeObtuse).
    Returns (4, 3, N) int64 and status."""
    D = _f64(D)
    n = D.shape[1]
    sb = np.zeros((4, 3, n), np.int64)
    st = np.zeros(n, np.int32)
    _load().or_superbase3d(_p(D), n, _p(sb), _p(st))
    return sb, st


def stencil3d(D):
    """3D AD-LBR stencils: Selling's decomposition on the obtuse superbase
    (Section 2, definition of V(z) and gamma_z in 3D, Lemma (Selling)).
    Returns offsets int16 (6, 3, N), weights f64 (6, N), status (N,)."""
    D = _f64(D)
    n = D.shape[1]
    off = np.zeros((6, 3, n), np.int16)
    w = np.zeros((6, n), np.float64)
    st = np.zeros(n, np.int32)
    _load().or_stencil3d(_p(D), n, _p(off), _p(w), _p(st))
    return off, w, st


def stencil(D):
    """Dispatch on the number of tensor planes (3 -> 2D, 6 -> 3D)."""
    return stencil2d(D) if np.shape(D)[0] == 3 else stencil3d(D)


# ------------------------------------------------------------- operator --

def operator_matrix(dims, off, w, periodic: bool = False, reflect: bool = False):
    """The AD-LBR operator A = 1/2 grad E_h with h = 1 (eq. (def:E*) and
    its gradient flow, Section 1), assembled by scattering every directed
    edge; Neumann truncation V(z; h) drops edges leaving the grid,
    periodic wraps them, reflect mirrors them back into the grid (the
    reflecting boundary of the restoration test, Section 4).
    Returns a scipy.sparse CSR matrix (duplicates summed)."""
    import scipy.sparse as sp
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    off = np.ascontiguousarray(off, dtype=np.int16)
    w = _f64(w)
    n = int(np.prod(dims))
    K = w.shape[0]
    cap = 4 * 2 * K * n
    ri = np.empty(cap, np.int64)
    ci = np.empty(cap, np.int64)
    v = np.empty(cap, np.float64)
    nd = np.array(list(dims) + [1] * (3 - dim), np.int64)
    mode = 2 if reflect else int(bool(periodic))
    t = _load().or_operator_coo(dim, _p(nd), mode, _p(off), _p(w),
                                _p(ri), _p(ci), _p(v))
    A = sp.coo_matrix((v[:t], (ri[:t], ci[:t])), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def cfl(A) -> float:
    """Explicit-Euler bound 1 / max_z A_zz: with dt <= this, I - dt A is
    entrywise non-negative (the discrete maximum principle)."""
    return 1.0 / float(A.diagonal().max())


def apply(A, u):
    """(A u) in FP64."""
    return A @ np.asarray(u, dtype=np.float64)


def explicit_steps(A, u0, dt: float, nsteps: int):
    """Explicit Euler u^{n+1} = u^n - dt A u^n (Section 4, CED time
    discretization), in FP64."""
    u = np.array(u0, dtype=np.float64)
    for _ in range(nsteps):
        u = u - dt * (A @ u)
    return u


def energy(dims, off, w, u, periodic: bool = False, reflect: bool = False) -> float:
    """E_h(u) = sum_z sum_{e in V(z;h)} gamma_z(e) |u(z+e) - u(z)|^2 with
    h = 1 (eq. (def:E*)), evaluated literally (vectorized over z); with
    reflect, u(z+e) outside the grid is u at the mirrored point."""
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    u = np.asarray(u, dtype=np.float64)
    n = u.size
    coords = np.indices(dims[::-1]).reshape(dim, -1)[::-1]  # x, y[, z]
    total = 0.0
    K = np.shape(w)[0]
    for i in range(K):
        for s in (-1, 1):
            q = coords + s * np.asarray(off[i], dtype=np.int64)
            if periodic:
                for c in range(dim):
                    q[c] %= dims[c]
                ok = np.ones(n, bool)
            elif reflect:
                for c in range(dim):
                    m = q[c] % (2 * dims[c])
                    q[c] = np.where(m < dims[c], m, 2 * dims[c] - 1 - m)
                ok = np.ones(n, bool)
            else:
                ok = np.all([(q[c] >= 0) & (q[c] < dims[c]) for c in range(dim)], axis=0)
            lin = q[0] + dims[0] * q[1] + (dims[0] * dims[1] * q[2] if dim == 3 else 0)
            lin = np.where(ok, lin, 0)
            du = np.where(ok, u[lin] - u, 0.0)
            total += float(np.sum(np.asarray(w[i], dtype=np.float64) * du * du))
    return total


# ------------------------------------------------------- structure tensor --

CED, EED = 0, 1


def structure_tensor_d(u, dims, sigma, rho, alpha, C, eig_map: int = CED):
    """Diffusion tensor from the structure tensor of u (Section 4:
    coherence-enhancing diffusion in 2D and 3D, edge-enhancing in 3D).
    u of shape (C, N) is a vector-valued image whose components share the
    tensor built from the sum of their gradient products (the Conclusion
    leaves that coupling to the tensor).  Returns D (3, N) in 2D or (6, N)
    in 3D, FP64."""
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    n = int(np.prod(dims))
    u = _f64(u).reshape(-1, n)
    nd = np.array(list(dims) + [1] * (3 - dim), np.int64)
    D = np.zeros((3 if dim == 2 else 6, n), np.float64)
    _load().or_structure_tensor_d(dim, _p(nd), _p(u), int(u.shape[0]), float(sigma),
                                  float(rho), float(alpha), float(C), int(eig_map), _p(D))
    return D


# ------------------------------------------------------------ restoration --

def restoration_exact(n: int, kappa: float, lam: float, alpha: float = 1.0 / 3.0):
    """Exact solution of the restoration test (Section 4, eq. (elliptic),
    -lambda div(D grad u) + u = v on the whole plane) at the n x n cell
    centres of the unit square: u = u0 o f with f(x, y) = (x, y +
    alpha cos(2 pi x)), where u0 solves the one-dimensional problem
    -lambda kappa^-2 u0'' + u0 = 1_{y < 1/2}:
        u0(y) = 1 - exp(-(1/2 - y)/l) / 2   (y < 1/2)
        u0(y) = exp(-(y - 1/2)/l) / 2       (y >= 1/2),   l = sqrt(lambda)/kappa.
    (The paper states the Fourier multiplier 1/(1 + <xi, D0 xi>) without
    the factors lambda and 4 pi^2; the elliptic equation fixes them.)"""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    return restoration_exact_at(np.tile(c, n), np.repeat(c, n), kappa, lam, alpha)


def restoration_exact_at(x, y, kappa: float, lam: float, alpha: float = 1.0 / 3.0):
    """restoration_exact at arbitrary points (x, y) of the plane."""
    t = np.asarray(y, dtype=np.float64) + alpha * np.cos(2.0 * np.pi * np.asarray(x))
    ell = np.sqrt(lam) / kappa
    return np.where(t < 0.5, 1.0 - 0.5 * np.exp(-np.abs(0.5 - t) / ell),
                    0.5 * np.exp(-np.abs(t - 0.5) / ell))


def restoration_errors(u_h, u, n: int):
    """Relative errors of a discrete solution against the exact one: the
    L2 norm over the grid points, and the H1 semi-norm with forward
    differences along x and y (the measures of the restoration test)."""
    e = (np.asarray(u_h, dtype=np.float64) - u).reshape(n, n)
    U = np.asarray(u, dtype=np.float64).reshape(n, n)
    l2 = np.linalg.norm(e) / np.linalg.norm(U)
    ge = np.concatenate([np.diff(e, axis=0).ravel(), np.diff(e, axis=1).ravel()])
    gu = np.concatenate([np.diff(U, axis=0).ravel(), np.diff(U, axis=1).ravel()])
    return float(l2), float(np.linalg.norm(ge) / np.linalg.norm(gu))
