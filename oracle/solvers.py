"""FP64 oracle for the implicit step and its preconditioners -- TEST
INFRASTRUCTURE ONLY.

The implicit step of the diffusion equation, (I + dt A) x = b with A the
AD-LBR operator, is the linear system the paper solves by conjugate
gradients for the restoration problem -lambda div(D grad u) + u = v
(Section 4, eq. (elliptic)).  Here:

  jacobi_pcg   textbook preconditioned CG with P = diag(K)
  fcg          flexible CG (truncation 1, Polak-Ribiere form) for a
               preconditioner that may change between iterations
  net_*        the learned preconditioner z = r / diag(K) + N(r): a 4-layer,
               16-channel stack of 3x3 (3x3x3) zero-padded convolutions on
               r, each output multiplied by per-point gates that a small
               gate net computes once per operator from stencil features;
               N is linear in r, so flexible CG sees a fixed linear
               preconditioner.  Forward and backward by the chain rule.
  energy_loss  the training objective (1/2 z^T K z - z^T r) / (r^T r)

The learned preconditioner is not in the paper ("parity unpinned" by the
paper); these functions are pinned by dense solves, textbook identities and
finite differences in tests/test_oracle_solvers.py.
"""
from __future__ import annotations

import numpy as np


def system_matrix(A, dt):
    """K = I + dt A (A from oracle.operator_matrix)."""
    import scipy.sparse as sp
    return (sp.identity(A.shape[0], format="csr") + dt * A).tocsr()


def _true_rel(K, b, x):
    return float(np.linalg.norm(b - K @ x) / np.linalg.norm(b))


def jacobi_pcg(K, b, tol=1e-6, max_iter=10000, x0=None, precond=True, history=False):
    """Preconditioned CG on K x = b with P = diag(K)^-1 (or P = I when
    precond is False).  Stops when the true relative residual
    |b - K x| / |b| <= tol (the recurrence residual triggers the check).
    Returns (x, iterations, relative residual[, residual history])."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    inv = 1.0 / K.diagonal() if precond else np.ones_like(b)
    r = b - K @ x
    z = inv * r
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while it < max_iter:
        if np.linalg.norm(r) <= tol * nb and _true_rel(K, b, x) <= tol:
            break
        q = K @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = inv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        hist.append(np.linalg.norm(r) / nb)
    out = (x, it, _true_rel(K, b, x))
    return out + (hist,) if history else out


def fcg(K, b, precond, tol=1e-6, max_iter=10000, x0=None, history=False):
    """Flexible CG with truncation 1: z_k = precond(r_k) may vary with k;
    beta_k = <z_k, r_k - r_{k-1}> / <z_{k-1}, r_{k-1}>,
    p_k = z_k + beta_k p_{k-1}, alpha_k = <z_k, r_k> / <p_k, K p_k>.
    With a fixed SPD linear preconditioner it generates the PCG iterates.
    Returns (x, iterations, relative residual, fell_back[, history]); on a
    non-descent direction (<z, r> <= 0 or <p, K p> <= 0), a non-finite
    value, or a stall
    (the smallest residual norm of the last 20 iterations is not 1% below
    the smallest one before them; CG residual norms need not decrease
    monotonically, hence the minima) it restarts from the current x with
    Jacobi-PCG."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - K @ x
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    it = 0
    p = None
    zr_prev = None
    r_prev = None
    while it < max_iter:
        if np.linalg.norm(r) <= tol * nb and _true_rel(K, b, x) <= tol:
            break
        z = precond(r)
        zr = z @ r
        stalled = it >= 20 and min(hist[-20:]) > 0.99 * min(hist[:-20])
        if not np.isfinite(zr) or zr <= 0.0 or stalled:
            xj, itj, rel = jacobi_pcg(K, b, tol, max_iter - it, x0=x)
            out = (xj, it + itj, rel, True)
            return out + (hist,) if history else out
        if p is None:
            p = z.copy()
        else:
            beta = (zr - z @ r_prev) / zr_prev
            p = z + beta * p
        q = K @ p
        pq = p @ q
        if not np.isfinite(pq) or pq <= 0.0:  # breakdown: x is left as it is
            xj, itj, rel = jacobi_pcg(K, b, tol, max_iter - it, x0=x)
            out = (xj, it + itj, rel, True)
            return out + (hist,) if history else out
        alpha = zr / pq
        x += alpha * p
        r_prev = r.copy()
        r = r - alpha * q
        zr_prev = zr
        it += 1
        hist.append(np.linalg.norm(r) / nb)
    out = (x, it, _true_rel(K, b, x), False)
    return out + (hist,) if history else out


# ------------------------------------------------------------------ CNN --

def _pad(x, dim):
    return np.pad(x, [(0, 0)] + [(1, 1)] * dim)


def _taps(dim):
    import itertools
    return list(itertools.product(range(3), repeat=dim))


def conv(x, W, b):
    """Cross-correlation with zero padding: out[o, p] = b[o] +
    sum_{i, t} W[o, i, t] x[i, p + t - 1] (p, t over the spatial axes)."""
    dim = x.ndim - 1
    xp = _pad(x, dim)
    shp = x.shape[1:]
    out = np.broadcast_to(b.reshape((-1,) + (1,) * dim), (W.shape[0],) + shp).copy()
    for t in _taps(dim):
        sl = (slice(None),) + tuple(slice(t[k], t[k] + shp[k]) for k in range(dim))
        out += np.einsum("oi,i...->o...", W[(slice(None), slice(None)) + t], xp[sl])
    return out


def conv_adjoint(y, W):
    """Adjoint of the zero-padded correlation x -> conv(x, W, 0):
    out[i, p] = sum_{o, t} W[o, i, t] y[o, p - t + 1]."""
    dim = y.ndim - 1
    shp = y.shape[1:]
    gxp = np.zeros((W.shape[1],) + tuple(s + 2 for s in shp))
    for t in _taps(dim):
        sl = (slice(None),) + tuple(slice(t[k], t[k] + shp[k]) for k in range(dim))
        gxp[sl] += np.einsum("oi,o...->i...", W[(slice(None), slice(None)) + t], y)
    return gxp[(slice(None),) + tuple(slice(1, 1 + s) for s in shp)]


def conv_backward(x, W, g):
    """Gradients of sum(g * conv(x, W, b)) w.r.t. x, W and b."""
    dim = x.ndim - 1
    xp = _pad(x, dim)
    shp = x.shape[1:]
    gW = np.zeros_like(W)
    for t in _taps(dim):
        sl = (slice(None),) + tuple(slice(t[k], t[k] + shp[k]) for k in range(dim))
        gW[(slice(None), slice(None)) + t] = (g.reshape(g.shape[0], -1)
                                              @ xp[sl].reshape(xp.shape[0], -1).T)
    gb = g.reshape(g.shape[0], -1).sum(1)
    return conv_adjoint(g, W), gW, gb


# ------------------------------------------------------ learned preconditioner --
# z = r / diag(K) + N(r) with N = B^T diag(g2) B and B = C2 diag(g1) C1,
# C1, C2 zero-padded 3^d correlations (1 -> W -> W channels, no bias) and
# g1, g2 in (0, 1) gates from a small gate net on per-point features.  N is
# symmetric positive semi-definite by construction, so the preconditioner
# diag(K)^-1 + N is SPD and flexible CG never meets <z, r> <= 0 in exact
# arithmetic.  Applied, it is four correlations: C1, C2, C2^T, C1^T.
# Parameter layout (flat FP32 vector, in this order):
#   gate layer A  WA (H, nf, T), bA (H)         conv 3^d, ReLU
#   gate layer B  WB (2W, H),    bB (2W)        1x1, sigmoid -> g1, g2
#   r path        W1 (W, 1, T), W2 (W, W, T)
# with T = 3^d taps in (dz,) dy, dx row-major order over offsets -1, 0, +1.

def net_shapes(dim, width=16, hidden=16):
    nf = 1 + (3 if dim == 2 else 6) + (3 if dim == 2 else 6)
    G = 2 * width
    return [("WA", (hidden, nf) + (3,) * dim), ("bA", (hidden,)),
            ("WB", (G, hidden)), ("bB", (G,)),
            ("W1", (width, 1) + (3,) * dim), ("W2", (width, width) + (3,) * dim)]


def net_init(seed, dim, width=16, hidden=16):
    """He-style initialization for the gate net, gate biases +2 (gates near
    0.88) and r-path weights at 0.3 x He scale, so the untrained N is a mild
    positive addition to Jacobi."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = {}
    for name, shp in net_shapes(dim, width, hidden):
        if name.startswith("b"):
            P[name] = np.full(shp, 2.0 if name == "bB" else 0.0)
        else:
            fan_in = int(np.prod(shp[1:]))
            scale = np.sqrt(2.0 / fan_in) * (0.3 if name in ("W1", "W2") else 1.0)
            P[name] = rng.normal(0.0, scale, size=shp)
    return P


def net_pack(P, dim, width=16, hidden=16):
    return np.concatenate([np.asarray(P[n], dtype=np.float64).reshape(-1)
                           for n, _ in net_shapes(dim, width, hidden)])


def net_unpack(flat, dim, width=16, hidden=16):
    P, o = {}, 0
    for n, shp in net_shapes(dim, width, hidden):
        k = int(np.prod(shp))
        P[n] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return P


def net_features(dims, off, w, diag, dt):
    """Per-point inputs of the gate net: 1 / (1 + dt A_zz), the weights
    dt w_q / (1 + dt A_zz), and D / tr D with D = sum_{e in V(z)} gamma e e^T
    recovered from the stencil (eq. (DSum)).  Shape (nf,) + spatial."""
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    shp = dims[::-1]
    kd = 1.0 + dt * np.asarray(diag, dtype=np.float64)
    ch = [1.0 / kd] + [dt * np.asarray(w[q], dtype=np.float64) / kd for q in range(w.shape[0])]
    o = np.asarray(off, dtype=np.float64)
    pairs = [(0, 0), (0, 1), (1, 1)] if dim == 2 else \
        [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    Dc = [sum(2.0 * np.asarray(w[q], dtype=np.float64) * o[q, a] * o[q, b]
              for q in range(w.shape[0])) for a, b in pairs]
    tr = Dc[0] + Dc[2] if dim == 2 else Dc[0] + Dc[3] + Dc[5]
    tr = np.where(tr > 0, tr, 1.0)
    ch += [c / tr for c in Dc]
    return np.stack([c.reshape(shp) for c in ch])


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def net_gates(P, F, keep=False):
    """Gates G = sigmoid(WB relu(conv(F; WA) + bA) + bB), shape (2W,) + spatial:
    g1 = G[:W], g2 = G[W:]."""
    h = conv(F, P["WA"], P["bA"])
    hr = np.maximum(h, 0.0)
    g = np.einsum("gh,h...->g...", P["WB"], hr) + P["bB"].reshape((-1,) + (1,) * (F.ndim - 1))
    G = _sigmoid(g)
    return (G, h, hr) if keep else G


def _net_B(P, G, v):
    """B v = C2 (g1 * C1 v); returns (B v, C1 v, g1 * C1 v)."""
    W = P["W1"].shape[0]
    a1 = conv(v, P["W1"], np.zeros(W))
    x1 = a1 * G[:W]
    return conv(x1, P["W2"], np.zeros(W)), a1, x1


def net_apply(P, G, r, shape):
    """N(r) = B^T (g2 * B r), B^T y = C1^T (g1 * C2^T y)."""
    W = P["W1"].shape[0]
    x = np.asarray(r, dtype=np.float64).reshape((1,) + tuple(shape))
    Br, _, _ = _net_B(P, G, x)
    y = G[W:] * Br
    return conv_adjoint(G[:W] * conv_adjoint(y, P["W2"]), P["W1"])[0]


def net_precondition(P, G, r, kd):
    """z = r / diag(K) + N(r)."""
    kd = np.asarray(kd, dtype=np.float64)
    out = net_apply(P, G, r, G.shape[1:])
    return np.asarray(r, dtype=np.float64) / kd + out.reshape(-1)


def net_backward(P, F, r, gz):
    """Gradient of s = <gz, N(r)> = <B gz, g2 * B r> w.r.t. every parameter
    (dict of arrays).  The g2 gradient is B gz * B r; B's parameters get the
    backward of B at input r with cotangent g2 * B gz plus the backward at
    input gz with cotangent g2 * B r; then the gate net by the chain rule."""
    G, h, hr = net_gates(P, F, keep=True)
    shp = G.shape[1:]
    W = P["W1"].shape[0]
    vr = np.asarray(r, dtype=np.float64).reshape((1,) + shp)
    vg = np.asarray(gz, dtype=np.float64).reshape((1,) + shp)
    Br, a1r, x1r = _net_B(P, G, vr)
    Bg, a1g, x1g = _net_B(P, G, vg)
    gG = np.zeros_like(G)
    gG[W:] = Bg * Br
    grads = {"W1": np.zeros_like(P["W1"]), "W2": np.zeros_like(P["W2"])}
    for v, a1, x1, cot in ((vr, a1r, x1r, G[W:] * Bg), (vg, a1g, x1g, G[W:] * Br)):
        gx1, gW2, _ = conv_backward(x1, P["W2"], cot)
        grads["W2"] += gW2
        gG[:W] += gx1 * a1
        _, gW1, _ = conv_backward(v, P["W1"], gx1 * G[:W])
        grads["W1"] += gW1
    gg = gG * G * (1.0 - G)                       # sigmoid'
    grads["bB"] = gg.reshape(gg.shape[0], -1).sum(1)
    grads["WB"] = gg.reshape(gg.shape[0], -1) @ hr.reshape(hr.shape[0], -1).T
    ghr = np.einsum("gh,g...->h...", P["WB"], gg)
    gh = ghr * (h > 0.0)
    _, gWA, gbA = conv_backward(F, P["WA"], gh)
    grads["WA"], grads["bA"] = gWA, gbA
    return grads


def energy_loss(K, z, r):
    """(1/2 z^T K z - z^T r) / (r^T r): minimal at z = K^-1 r; its value
    plus 1/2 r^T K^-1 r / r^T r is the squared K-norm error of z, halved.
    Returns (loss, gradient w.r.t. z)."""
    Kz = K @ z
    rr = r @ r
    return (0.5 * z @ Kz - z @ r) / rr, (Kz - r) / rr
