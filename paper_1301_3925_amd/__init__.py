"""MI355X-native AD-LBR: Python binding of libadlbr.so.

Thin wrappers with the C ABI's names.  They allocate outputs and workspaces
as torch tensors on the current device, pass raw pointers and the current
HIP stream, and raise on a non-zero return code.  Every arithmetic step runs
in the HIP kernels of libadlbr.so; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes

from . import capi
from .capi import AdlbrError

__all__ = ["build_stencils", "Operator", "structure_tensor", "grid", "AdlbrError",
           "status_flags"]


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    codes = {torch.float64: capi.F64, torch.float32: capi.F32,
             torch.bfloat16: capi.BF16, torch.float16: capi.F16}
    if t not in codes:
        raise TypeError(f"unsupported dtype {t}")
    return codes[t]


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("tensor must live on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")


def grid(dims, periodic: bool = False, reflect: bool = False) -> capi.Grid:
    dims = [int(d) for d in dims]
    g = capi.Grid()
    g.dim = len(dims)
    g.boundary = capi.REFLECT if reflect else capi.PERIODIC if periodic else capi.NEUMANN
    for i in range(3):
        g.n[i] = dims[i] if i < len(dims) else 1
    return g


def _npoints(dims):
    n = 1
    for d in dims:
        n *= int(d)
    return n


def build_stencils(D, dims, w_dtype=None, periodic: bool = False, stream=None, out=None):
    """AD-LBR stencils of a tensor field (adlbr_build_stencils).

    D: [3|6, N] float64/float32 on the GPU.  Returns (offsets int16
    [S, d, N], weights [S, N], status int32[2]) on the same device; `out`
    may pass that triple preallocated."""
    torch = _torch()
    lib = capi.load()
    _require_cuda(D)
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    S = 3 if dim == 2 else 6
    N = _npoints(dims)
    if tuple(D.shape) != ((3 if dim == 2 else 6), N):
        raise ValueError(f"D must have shape ({3 if dim == 2 else 6}, {N})")
    w_dtype = w_dtype or D.dtype
    if out is not None:
        off, w, st = out
        w_dtype = w.dtype
    else:
        off = torch.empty((S, dim, N), dtype=torch.int16, device=D.device)
        w = torch.empty((S, N), dtype=w_dtype, device=D.device)
        st = torch.empty(2, dtype=torch.int32, device=D.device)
    g = grid(dims, periodic)
    capi.check(lib.adlbr_build_stencils(ctypes.byref(g), _ptr(D), _dtype_code(D.dtype),
                                        _ptr(off), _ptr(w), _dtype_code(w_dtype), _ptr(st),
                                        _stream(stream)))
    return off, w, st


_OP_ERRORS = {capi.ST_RANGE: "an offset does not fit the operator's storage",
              capi.ST_STENCIL: "slots are not built from a superbase",
              capi.ST_INCOMING: "more than 255 stencils reach one point"}


def status_flags(status) -> int:
    """The OR of ADLBR_ST_* flags of a device status word (synchronizes)."""
    return int(status[1].item())


class Operator:
    """The assembled operator A = 1/2 grad E_h (adlbr_operator_create).

    tiled=True asks for the tiled layout (ADLBR_OP_TILED: explicit steps
    with tile + halo staged in LDS, near edges unlisted; Neumann grids,
    F32/BF16/F16 storage; not for solve).  records=True keeps every 2D
    incoming entry with its weight (ADLBR_OP_RECORDS), which a Batch of
    such operators reads instead of gathering the weights.

    Holds its device workspace (a torch uint8 tensor) for its lifetime.
    With check=True (the default) the constructor synchronizes and raises
    AdlbrError when the device status word reports a bad operator (an
    offset out of range, slots that are not a superbase, a point reached by
    more than 255 stencils).  wide=None picks int8 compact offsets and falls
    back to int16 when an offset does not fit (needs check=True); with
    check=False the caller reads self.status itself."""

    def __init__(self, dims, offsets, weights, storage=None, periodic: bool = False,
                 wide=None, stream=None, workspace=None, check: bool = True,
                 tiled: bool = False, reflect: bool = False, records: bool = False):
        self._h = ctypes.c_void_p()
        self.tiled = bool(tiled)
        self.records = bool(records)
        self.reflect = bool(reflect)
        self._create(dims, offsets, weights, storage, periodic, bool(wide), stream, workspace)
        if not check:
            return
        flags = status_flags(self.status)
        if wide is None and flags & capi.ST_RANGE:
            self.close()
            self._create(dims, offsets, weights, storage, periodic, True, stream, workspace)
            flags = status_flags(self.status)
        bad = [msg for f, msg in _OP_ERRORS.items() if flags & f]
        if bad:
            first = int(self.status[0].item())
            self.close()
            raise AdlbrError(capi.E_RANGE, "operator_create: " + "; ".join(bad) +
                             f" (first point {first})")

    def _create(self, dims, offsets, weights, storage, periodic, wide, stream, workspace):
        torch = _torch()
        lib = capi.load()
        _require_cuda(offsets, weights)
        self.dims = tuple(int(d) for d in dims)
        self.N = _npoints(self.dims)
        self.storage = storage or torch.float32
        self.device = weights.device
        self.wide = wide
        self._grid = grid(self.dims, periodic, self.reflect)
        flags = ((capi.OP_WIDE if wide else 0) | (capi.OP_TILED if self.tiled else 0) |
                 (capi.OP_RECORDS if self.records else 0))
        nbytes = ctypes.c_size_t()
        capi.check(lib.adlbr_operator_workspace(ctypes.byref(self._grid),
                                                _dtype_code(self.storage), flags,
                                                ctypes.byref(nbytes)))
        if workspace is not None and workspace.numel() >= nbytes.value:
            self.workspace = workspace
        else:
            self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.status = torch.empty(2, dtype=torch.int32, device=self.device)
        h = ctypes.c_void_p()
        capi.check(lib.adlbr_operator_create(
            ctypes.byref(self._grid), _ptr(offsets), _ptr(weights), _dtype_code(weights.dtype),
            _dtype_code(self.storage), flags, _ptr(self.workspace), self.workspace.numel(),
            _ptr(self.status), _stream(stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def rebuild(self, offsets, weights, stream=None, check: bool = False):
        """Re-assemble in place from new stencils of the same grid
        (adlbr_operator_rebuild): device addresses stay, so a Batch over
        this operator stays valid.  Asynchronous unless check=True."""
        _require_cuda(offsets, weights)
        capi.check(capi.load().adlbr_operator_rebuild(
            self._h, _ptr(offsets), _ptr(weights), _dtype_code(weights.dtype),
            _ptr(self.status), _stream(stream)))
        if check:
            flags = status_flags(self.status)
            bad = [msg for f, msg in _OP_ERRORS.items() if flags & f]
            if bad:
                raise AdlbrError(capi.E_RANGE, "operator_rebuild: " + "; ".join(bad))
        return self

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            capi.load().adlbr_operator_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dt_cfl(self, stream=None) -> float:
        out = ctypes.c_double()
        capi.check(capi.load().adlbr_operator_dt_cfl(self._h, ctypes.byref(out), _stream(stream)))
        return out.value

    def diagonal(self, dtype=None, stream=None):
        torch = _torch()
        dtype = dtype or torch.float64
        d = torch.empty(self.N, dtype=dtype, device=self.device)
        capi.check(capi.load().adlbr_operator_diagonal(self._h, _ptr(d), _dtype_code(dtype),
                                                       _stream(stream)))
        return d

    def _check_u(self, u):
        _require_cuda(u)
        if u.dtype != self.storage or u.numel() != self.N:
            raise ValueError(f"u must be {self.N} values of {self.storage}")

    def apply(self, u, out=None, stream=None):
        """A u (adlbr_apply)."""
        torch = _torch()
        self._check_u(u)
        out = torch.empty_like(u) if out is None else out
        self._check_u(out)
        capi.check(capi.load().adlbr_apply(self._h, _ptr(u), _ptr(out), _stream(stream)))
        return out

    def step(self, u, dt: float, nsteps: int, cfl_fraction: bool = False, u_tmp=None,
             stream=None):
        """nsteps explicit Euler steps in place on u (adlbr_step).  With
        cfl_fraction=True, dt is a fraction of 1 / max A_zz."""
        torch = _torch()
        self._check_u(u)
        u_tmp = torch.empty_like(u) if u_tmp is None else u_tmp
        self._check_u(u_tmp)
        mode = capi.DT_CFL if cfl_fraction else capi.DT_ABS
        capi.check(capi.load().adlbr_step(self._h, _ptr(u), _ptr(u_tmp), float(dt), mode,
                                          int(nsteps), _stream(stream)))
        return u


    def step_multi(self, u, dt: float, nsteps: int, cfl_fraction: bool = False, u_tmp=None,
                   stream=None):
        """nsteps explicit steps of every component of u ([C, N], in place)
        with this one operator (adlbr_step_multi)."""
        torch = _torch()
        _require_cuda(u)
        if u.dim() != 2 or u.shape[1] != self.N or u.dtype != self.storage:
            raise ValueError(f"u must be [C, {self.N}] of {self.storage}")
        u_tmp = torch.empty_like(u) if u_tmp is None else u_tmp
        mode = capi.DT_CFL if cfl_fraction else capi.DT_ABS
        capi.check(capi.load().adlbr_step_multi(self._h, _ptr(u), _ptr(u_tmp), int(u.shape[0]),
                                                float(dt), mode, int(nsteps), _stream(stream)))
        return u

    def solve(self, b, dt: float, method: str = "jacobi", tol: float = 1e-6,
              max_iter: int = 10000, check_every: int = 10, x=None, net=None,
              workspace=None, stream=None):
        """Solve (I + dt A) x = b (adlbr_solve).  Returns (x, report dict);
        report["converged"] is 0 when max_iter was reached."""
        torch = _torch()
        lib = capi.load()
        self._check_u(b)
        code = capi.SOLVE_FCG_NET if method == "fcg" else capi.SOLVE_JACOBI_PCG
        nbytes = ctypes.c_size_t()
        capi.check(lib.adlbr_solve_workspace(self._h, code, ctypes.byref(nbytes)))
        if workspace is None or workspace.numel() < nbytes.value:
            workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        x0_zero = x is None
        x = torch.empty_like(b) if x is None else x
        self._check_u(x)
        p = capi.SolveParams(code, int(max_iter), int(check_every), int(x0_zero), float(tol),
                             None if net is None else net.handle)
        rep = capi.SolveReport()
        rc = lib.adlbr_solve(self._h, float(dt), _ptr(b), _ptr(x), ctypes.byref(p),
                             _ptr(workspace), workspace.numel(), ctypes.byref(rep),
                             _stream(stream))
        if rc != capi.E_NOT_CONVERGED:
            capi.check(rc)
        return x, rep.as_dict()


def tune_cache_save(path) -> None:
    """Write the batch tuner's choices of this process to a JSON file
    (adlbr_batch_tune_save)."""
    capi.check(capi.load().adlbr_batch_tune_save(str(path).encode()))


def tune_cache_load(path) -> None:
    """Merge a tuner cache file into this process's cache
    (adlbr_batch_tune_load); later batches take its choices untimed."""
    capi.check(capi.load().adlbr_batch_tune_load(str(path).encode()))


def tune_cache_clear() -> None:
    capi.check(capi.load().adlbr_batch_tune_clear())


def tune_cache_lookup(class_key: int, points: int, nprob: int):
    """(variant, chunk_bytes) cached for a class, or None."""
    found, var, cb = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
    capi.check(capi.load().adlbr_batch_tune_lookup(int(class_key), int(points), int(nprob),
                                                   ctypes.byref(found), ctypes.byref(var),
                                                   ctypes.byref(cb)))
    return (var.value, cb.value) if found.value else None


class Batch:
    """Many operators stepped together (adlbr_batch_*): one grouped launch
    per class and step, the whole run captured into one HIP graph.
    us[i] is stepped in place; tmps[i] (allocated if not given) is scratch.
    dt is one value or one per problem; dt_mode "cfl" scales each problem's
    own 1 / max A_zz, "abs" takes dt as the step."""

    def __init__(self, ops, us, tmps=None, dt=0.9, dt_mode: str = "cfl", stream=None):
        torch = _torch()
        lib = capi.load()
        n = len(ops)
        if n == 0 or len(us) != n:
            raise ValueError("need one state per operator")
        for op, u in zip(ops, us):
            op._check_u(u)
        self.ops, self.us = list(ops), list(us)
        self.tmps = [torch.empty_like(u) for u in us] if tmps is None else list(tmps)
        dts = [float(dt)] * n if isinstance(dt, (int, float)) else [float(d) for d in dt]
        nb = ctypes.c_size_t()
        capi.check(lib.adlbr_batch_workspace(n, ctypes.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=ops[0].device)
        P = ctypes.c_void_p * n
        self._ops = P(*[op.handle.value for op in ops])
        self._u = P(*[u.data_ptr() for u in self.us])
        self._t = P(*[t.data_ptr() for t in self.tmps])
        self._dt = (ctypes.c_double * n)(*dts)
        h = ctypes.c_void_p()
        mode = capi.DT_CFL if dt_mode == "cfl" else capi.DT_ABS
        capi.check(lib.adlbr_batch_create(n, self._ops, self._u, self._t, self._dt, mode,
                                          _ptr(self.ws), self.ws.numel(), _stream(stream),
                                          ctypes.byref(h)))
        self._h = h

    def tune(self, steps: int = 5, use_cache: bool = True, stream=None):
        capi.check(capi.load().adlbr_batch_tune(self._h, int(steps), int(use_cache),
                                                _stream(stream)))
        return self.variants()

    def set_variant(self, cls: int, variant: int, chunk_bytes: int = 0, stream=None):
        capi.check(capi.load().adlbr_batch_set_variant(self._h, int(cls), int(variant),
                                                       int(chunk_bytes), _stream(stream)))

    def variants(self):
        lib = capi.load()
        out, k = [], 0
        while True:
            key, var, n, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            cb = ctypes.c_size_t()
            if lib.adlbr_batch_variant(self._h, k, ctypes.byref(key), ctypes.byref(var),
                                       ctypes.byref(n), ctypes.byref(nc), ctypes.byref(cb)) != 0:
                return out
            out.append({"class": key.value, "variant": var.value, "problems": n.value,
                        "chunks": nc.value, "chunk_bytes": cb.value})
            k += 1

    def run(self, nsteps: int, graph: bool = True, stream=None):
        capi.check(capi.load().adlbr_batch_run(self._h, int(nsteps), int(graph), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            capi.load().adlbr_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def structure_tensor(u, dims, sigma: float, rho: float, alpha: float, C: float,
                     eig_map: str = "ced", out=None, workspace=None, stream=None):
    """Diffusion tensor from the structure tensor of u (adlbr_structure_tensor).
    u of shape [C, N] is a vector-valued image: its components share one
    tensor built from the sum of their gradient products
    (adlbr_structure_tensor_vec)."""
    torch = _torch()
    lib = capi.load()
    _require_cuda(u)
    dims = tuple(int(d) for d in dims)
    g = grid(dims)
    code = _dtype_code(u.dtype)
    nbytes = ctypes.c_size_t()
    capi.check(lib.adlbr_tensor_workspace(ctypes.byref(g), code, ctypes.byref(nbytes)))
    if workspace is None or workspace.numel() < nbytes.value:
        workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=u.device)
    nj = 3 if len(dims) == 2 else 6
    npts = 1
    for d in dims:
        npts *= d
    if u.dim() not in (1, 2) or u.shape[-1] != npts or not u.is_contiguous():
        raise ValueError(f"u must be a contiguous [{npts}] or [C, {npts}] tensor")
    out = torch.empty((nj, npts), dtype=u.dtype, device=u.device) if out is None else out
    p = capi.TensorParams(float(sigma), float(rho), float(alpha), float(C),
                          capi.MAP_CED if eig_map == "ced" else capi.MAP_EED)
    if u.dim() == 1:
        capi.check(lib.adlbr_structure_tensor(ctypes.byref(g), _ptr(u), code, ctypes.byref(p),
                                              _ptr(out), _ptr(workspace), workspace.numel(),
                                              _stream(stream)))
    else:
        capi.check(lib.adlbr_structure_tensor_vec(ctypes.byref(g), _ptr(u), int(u.shape[0]),
                                                  code, ctypes.byref(p), _ptr(out),
                                                  _ptr(workspace), workspace.numel(),
                                                  _stream(stream)))
    return out


def structure_tensor_noalloc(u, dims, sigma: float, rho: float, alpha: float, C: float,
                             eig_map: str = "ced", out=None, stream=None):
    """adlbr_structure_tensor_noalloc: the same tensor with the library's
    static device scratch instead of a workspace (nothing is allocated when
    `out` is given).  Calls that overlap on one GPU race."""
    torch = _torch()
    lib = capi.load()
    _require_cuda(u)
    dims = tuple(int(d) for d in dims)
    g = grid(dims)
    nj = 3 if len(dims) == 2 else 6
    out = torch.empty((nj, u.numel()), dtype=u.dtype, device=u.device) if out is None else out
    p = capi.TensorParams(float(sigma), float(rho), float(alpha), float(C),
                          capi.MAP_CED if eig_map == "ced" else capi.MAP_EED)
    capi.check(lib.adlbr_structure_tensor_noalloc(ctypes.byref(g), _ptr(u), _dtype_code(u.dtype),
                                                  ctypes.byref(p), _ptr(out), _stream(stream)))
    return out


class Net:
    """Learned preconditioner z = r / diag(K) + N(r) of an FP32 operator
    (adlbr_net_*).  Holds the parameters and the per-operator buffers."""

    def __init__(self, op: "Operator", params=None, seed: int = 0):
        torch = _torch()
        lib = capi.load()
        self.op = op
        self.dim = len(op.dims)
        self.N = op.N
        cnt = ctypes.c_size_t()
        capi.check(lib.adlbr_net_param_count(self.dim, 16, 16, ctypes.byref(cnt)))
        self.nparams = cnt.value
        dev = op.device
        if params is None:
            params = self.init_params(self.dim, seed)
        self.params = params.to(device=dev, dtype=torch.float32).contiguous()
        if self.params.numel() != self.nparams:
            raise ValueError(f"need {self.nparams} parameters")
        nf = 7 if self.dim == 2 else 13
        N = self.N
        self.features = torch.empty((nf, N), dtype=torch.float32, device=dev)
        self.hidden_act = torch.empty((16, N), dtype=torch.float32, device=dev)
        self.gates = torch.empty((49, N), dtype=torch.float32, device=dev)
        self.gates8 = torch.empty((N, 32), dtype=torch.uint8, device=dev)
        self.scratch = torch.empty((32, N), dtype=torch.float32, device=dev)
        T = 3 ** self.dim
        self.layers = torch.empty(2 * 16 * 17 * T + 7168, dtype=torch.float32, device=dev)
        self._s = capi.NetStruct(self.dim, 16, 16, nf, self.params.data_ptr(),
                                 self.features.data_ptr(), self.hidden_act.data_ptr(),
                                 self.gates.data_ptr(), self.gates8.data_ptr(),
                                 self.scratch.data_ptr(), self.layers.data_ptr())
        self._ws = None

    @staticmethod
    def init_params(dim: int, seed: int = 0):
        """He-style random initialization (host, seeded) of the gate net, gate
        biases +2, r-path weights at 0.3 x He scale, so the untrained N is a
        mild positive addition to Jacobi.  Order as in adlbr.h."""
        import numpy as np
        torch = _torch()
        rng = np.random.Generator(np.random.PCG64(seed))
        T = 3 ** dim
        nf = 7 if dim == 2 else 13
        parts = [rng.normal(0, (2.0 / (nf * T)) ** 0.5, 16 * nf * T), np.zeros(16),
                 rng.normal(0, (2.0 / 16) ** 0.5, 32 * 16), np.full(32, 2.0),
                 rng.normal(0, 0.3 * (2.0 / T) ** 0.5, 16 * T),
                 rng.normal(0, 0.3 * (2.0 / (16 * T)) ** 0.5, 16 * 16 * T)]
        return torch.from_numpy(np.concatenate(parts)).float()

    @property
    def handle(self):
        return ctypes.cast(ctypes.pointer(self._s), ctypes.c_void_p)

    def workspace(self):
        torch = _torch()
        if self._ws is None:
            nb = ctypes.c_size_t()
            capi.check(capi.load().adlbr_net_workspace(self.op.handle, self.handle,
                                                       ctypes.byref(nb)))
            self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.op.device)
        return self._ws

    def prepare(self, dt: float, stream=None):
        """Features of the operator at dt, then the gates (adlbr_net_features,
        adlbr_net_gates)."""
        lib = capi.load()
        capi.check(lib.adlbr_net_features(self.op.handle, float(dt), self.handle, _stream(stream)))
        self.refresh_gates(stream)

    def refresh_gates(self, stream=None):
        capi.check(capi.load().adlbr_net_gates(self.op.handle, self.handle, _stream(stream)))

    def forward(self, r, saved=None, out=None, stream=None):
        torch = _torch()
        z = torch.empty_like(r) if out is None else out
        capi.check(capi.load().adlbr_net_forward(self.op.handle, self.handle, _ptr(r), _ptr(z),
                                                 None if saved is None else _ptr(saved),
                                                 _stream(stream)))
        return z

    def precondition(self, r, out=None, stream=None):
        """The inference path used inside flexible CG (adlbr_net_precondition)."""
        torch = _torch()
        z = torch.empty_like(r) if out is None else out
        capi.check(capi.load().adlbr_net_precondition(self.op.handle, self.handle, _ptr(r),
                                                      _ptr(z), _stream(stream)))
        return z

    def backward(self, r, gz, saved, gparams, ggates, stream=None):
        ws = self.workspace()
        capi.check(capi.load().adlbr_net_backward(self.op.handle, self.handle, _ptr(r), _ptr(gz),
                                                  _ptr(saved), _ptr(gparams), _ptr(ggates),
                                                  _ptr(ws), ws.numel(), _stream(stream)))

    def gates_backward(self, ggates, gparams, stream=None):
        ws = self.workspace()
        capi.check(capi.load().adlbr_net_gates_backward(self.op.handle, self.handle, _ptr(ggates),
                                                        _ptr(gparams), _ptr(ws), ws.numel(),
                                                        _stream(stream)))

    def loss_grad(self, dt, r, z, gz, loss, stream=None):
        ws = self.workspace()
        capi.check(capi.load().adlbr_net_loss_grad(self.op.handle, float(dt), _ptr(r), _ptr(z),
                                                   _ptr(gz), _ptr(loss), _ptr(ws), ws.numel(),
                                                   _stream(stream)))


def residual(op: "Operator", b, x, dt: float, out=None, stream=None):
    """r = b - (I + dt A) x (adlbr_residual)."""
    torch = _torch()
    r = torch.empty_like(b) if out is None else out
    capi.check(capi.load().adlbr_residual(op.handle, float(dt), _ptr(b), _ptr(x), _ptr(r),
                                          _stream(stream)))
    return r


def adam(params, grads, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
         grad_scale: float = 1.0, stream=None):
    """Adam step on grad_scale * grads (adlbr_net_adam)."""
    capi.check(capi.load().adlbr_net_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v),
                                          params.numel(), int(step), float(grad_scale),
                                          float(lr), float(beta1), float(beta2), float(eps),
                                          _stream(stream)))


def train_net(op: "Operator", dt: float, rhs_seeds, steps: int = 400, batch: int = 4,
              lr: float = 2e-3, seed: int = 0, snapshot_iters=(1, 2, 4, 8, 16, 32),
              log_every: int = 0, on_policy: bool = False, refresh: int = 1, log=None):
    """Train the preconditioner on residuals the solver itself generates:
    for each right-hand side, Jacobi-PCG stopped after k iterations leaves a
    residual r_k = b - K x_k (adlbr_residual); each Adam step takes `batch`
    of them, minimizes the energy loss (adlbr_net_loss_grad) through the
    network's own backward kernels and updates with adlbr_net_adam.  With
    on_policy, the residuals of flexible CG with the network as it stands
    (stopped after the same k) join the pool `refresh` times, evenly spaced
    after the first half of the steps.  log(step, loss), if given, is called
    with every logged loss (every log_every steps).
    Returns (net, history of losses)."""
    import numpy as np
    from . import synth
    torch = _torch()
    dev = op.device
    net = Net(op, seed=seed)
    net.prepare(dt)
    samples = []
    for s in rhs_seeds:
        b = torch.from_numpy(synth.uniform(s, op.N)).float().to(dev)
        for k in snapshot_iters:
            x, _ = op.solve(b, dt, max_iter=k, check_every=k)
            samples.append(residual(op, b, x, dt))
    R = torch.stack(samples)
    saved = torch.empty((batch, 49, op.N), dtype=torch.float32, device=dev)
    z = torch.empty((batch, op.N), dtype=torch.float32, device=dev)
    gz = torch.empty_like(z)
    gparams = torch.zeros(net.nparams, dtype=torch.float32, device=dev)
    ggates = torch.zeros((49, op.N), dtype=torch.float32, device=dev)
    m = torch.zeros_like(gparams)
    v = torch.zeros_like(gparams)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    hist = []
    for it in range(1, steps + 1):
        marks = {steps // 2 + 1 + (steps // 2) * j // max(1, refresh) for j in range(refresh)}
        if on_policy and it in marks:
            more = []
            for sd in rhs_seeds:
                b = torch.from_numpy(synth.uniform(sd, op.N)).float().to(dev)
                for k in snapshot_iters:
                    x, _ = op.solve(b, dt, method="fcg", net=net, max_iter=k, check_every=k)
                    more.append(residual(op, b, x, dt))
            R = torch.cat([R, torch.stack(more)])
        idx = rng.choice(R.shape[0], size=batch, replace=False)
        gparams.zero_()
        ggates.zero_()
        loss.zero_()
        for j, k in enumerate(idx):
            r = R[int(k)]
            net.forward(r, saved=saved[j], out=z[j])
            net.loss_grad(dt, r, z[j], gz[j], loss)
            net.backward(r, gz[j], saved[j], gparams, ggates)
        net.gates_backward(ggates, gparams)
        adam(net.params, gparams, m, v, it, lr, grad_scale=1.0 / batch)
        net.refresh_gates()
        if log_every and (it % log_every == 0 or it == 1):
            hist.append((it, float(loss.item()) / batch))
            if log is not None:
                log(it, hist[-1][1])
    return net, hist
