// Implicit step K x = b, K = I + dt A, by preconditioned conjugate gradients.
//
// All scalars live on the device (CgState); every reduction is a per-block
// FP64 partial sum finished by a one-block kernel in block order, so a solve
// is deterministic and needs no host round trip per iteration.  The update
// kernel's finisher raises `done` when the recurrence residual drops below
// tol |b|; later kernels of the same batch are then no-ops, so the iteration
// count is exact although the host only looks every check_every
// iterations.  The host confirms convergence with the true residual
// |b - K x| in FP64.
//
// Jacobi-PCG per iteration: update (x, r, z = r / diag K, <r,z>, <r,r>,
// beta) -> direction (q = K z + beta q, p = z + beta p, <p,q>, alpha).
// Flexible CG (Section 4 solves the restoration system by CG; the flexible
// variant admits the learned preconditioner): update (x, r, <r,r>) ->
// z = N(r) with the dots <z,r>, <z,r_prev> -> scalars (|r|^2 checks, beta)
// -> direction.
#include <algorithm>
#include <utility>
#include <vector>

#include "common.h"

namespace adlbr {
namespace {

constexpr int kBS = 256;

struct SolveState {
    CgState cg;
    double tol2bb;  // tol^2 |b|^2
    double rr_true;
};

template <typename TD> __device__ __forceinline__ double inv_kd(const TD *diag, long long z, double dt) {
    return 1.0 / (1.0 + dt * (double)diag[z]);
}

// x0 = 0: x64 = 0, r = b; otherwise r = b - K x64 is already in r.
// z = r / diag K (Jacobi); partial sums of <r, z> and <b, b>.
template <typename T, typename TD>
__global__ __launch_bounds__(kBS) void k_init(long long N, const T *__restrict__ b,
                                              double *__restrict__ x64, T *__restrict__ r,
                                              T *__restrict__ z, const TD *__restrict__ diag,
                                              int x0_zero, int jacobi, const SolveState *st,
                                              double *part) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    double rz = 0.0, bb = 0.0;
    if (i < N) {
        const T bi = b[i];
        T ri;
        if (x0_zero) {
            x64[i] = 0.0;
            ri = bi;
            r[i] = ri;
        } else {
            ri = r[i];
        }
        if (jacobi) {
            const T zi = (T)((double)ri * inv_kd(diag, i, st->cg.dt));
            z[i] = zi;
            rz = (double)ri * (double)zi;
        }
        bb = (double)bi * (double)bi;
    }
    block_partial_sum(rz, part);
    block_partial_sum(bb, part + gridDim.x);
}

__global__ __launch_bounds__(kBS) void k_init_fin(SolveState *st, const double *part, long long nb,
                                                  double tol2) {
    const double rz = reduce_partials(part, nb);
    const double bb = reduce_partials(part + nb, nb);
    if (threadIdx.x != 0) return;
    st->cg.rz = rz;
    st->cg.beta = 0.0;
    st->cg.iter = 0;
    st->cg.bad = 0;
    st->cg.done = 0;
    st->cg.bb = bb;
    st->tol2bb = tol2 * bb;
    st->cg.rr = bb;
}

// Jacobi-PCG update: x += alpha p, r -= alpha q, z = r / diag K; partials
// of <r, z> and <r, r>.
template <typename T, typename TD>
__global__ __launch_bounds__(kBS) void k_pcg_update(long long N, double *__restrict__ x,
                                                    T *__restrict__ r, T *__restrict__ z,
                                                    const T *__restrict__ p, const T *__restrict__ q,
                                                    const TD *__restrict__ diag,
                                                    const SolveState *st, double *part) {
    const bool skip = st->cg.done || st->cg.bad;
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < N && !skip) {
        const T a = (T)st->cg.alpha;
        x[i] += st->cg.alpha * (double)p[i];
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        const T zi = (T)((double)ri * inv_kd(diag, i, st->cg.dt));
        z[i] = zi;
        rz = (double)ri * (double)zi;
        rr = (double)ri * (double)ri;
    }
    block_partial_sum(rz, part);
    block_partial_sum(rr, part + gridDim.x);
}

// Finish a PCG iteration: beta, history, convergence flag.
__global__ __launch_bounds__(kBS) void k_pcg_scalars(SolveState *st, const double *part,
                                                     long long nb, double *hist, int max_hist) {
    const double rzn = reduce_partials(part, nb);
    const double rr = reduce_partials(part + nb, nb);
    if (threadIdx.x != 0 || st->cg.done || st->cg.bad) return;
    if (!isfinite(rzn) || !isfinite(rr) || !(st->cg.rz > 0.0)) st->cg.bad = 1;
    st->cg.beta = st->cg.bad ? 0.0 : rzn / st->cg.rz;
    st->cg.rz_old = st->cg.rz;
    st->cg.rz = rzn;
    st->cg.rr = rr;
    const int it = st->cg.iter + 1;
    st->cg.iter = it;
    if (it < max_hist) hist[it] = rr;
    if (rr <= st->tol2bb) st->cg.done = 1;
}

// Flexible-CG update: x += alpha p, r_new = r - alpha q; partials of <r_new, r_new>.
template <typename T>
__global__ __launch_bounds__(kBS) void k_fcg_update(long long N, double *__restrict__ x,
                                                    const T *__restrict__ r, T *__restrict__ rn,
                                                    const T *__restrict__ p,
                                                    const T *__restrict__ q, const SolveState *st,
                                                    double *prr) {
    const bool skip = st->cg.done || st->cg.bad;
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    double rr = 0.0;
    if (i < N && !skip) {
        const T a = (T)st->cg.alpha;
        x[i] += st->cg.alpha * (double)p[i];
        const T ri = r[i] - a * q[i];
        rn[i] = ri;
        rr = (double)ri * (double)ri;
    }
    block_partial_sum(rr, prr);
}

// Finish a flexible-CG iteration (one block): unless first, the update's
// |r|^2 from its partials prr (iteration count, history, breakdown and
// convergence flags); then, from the dot partials part (nparts each),
// beta = (<z, r> - <z, r_prev>) / <z_prev, r_prev> (first: beta = 0).
__global__ __launch_bounds__(kBS) void k_fcg_scalars(SolveState *st, const double *part,
                                                     long long nparts, const double *prr,
                                                     long long nb, double *hist, int max_hist,
                                                     int first) {
    const double rr = first ? 0.0 : reduce_partials(prr, nb);
    const double zr = reduce_partials(part, nparts);
    const double zrp = reduce_partials(part + nparts, nparts);
    if (threadIdx.x != 0 || st->cg.done || st->cg.bad) return;
    if (!first) {
        st->cg.rr = rr;
        const int it = st->cg.iter + 1;
        st->cg.iter = it;
        if (it < max_hist) hist[it] = rr;
        if (!isfinite(rr)) {
            st->cg.bad = 1;
            return;
        }
        if (rr <= st->tol2bb) {
            st->cg.done = 1;
            return;
        }
    }
    if (!isfinite(zr) || !(zr > 0.0) || !isfinite(zrp)) {
        st->cg.bad = 1;
        return;
    }
    st->cg.beta = first ? 0.0 : (zr - zrp) / st->cg.rz;
    st->cg.rz_old = st->cg.rz;
    st->cg.rz = zr;
}

// Zero the whole state and set dt; a kernel rather than a host copy so no
// host buffer has to outlive the enqueue.
__global__ void k_state_reset(SolveState *st, double dt) {
    uint32_t *w = (uint32_t *)st;
    constexpr int nw = (int)(sizeof(SolveState) / 4);
    for (int k = threadIdx.x; k < nw; k += blockDim.x) w[k] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) st->cg.dt = dt;
}

// Residual replacement: r already holds b - K x (from the true residual);
// recompute the Jacobi z and partials of <r, z>; k_restart_fin restarts the
// direction (beta = 0) and keeps the iteration count.
template <typename T, typename TD>
__global__ __launch_bounds__(kBS) void k_restart(long long N, const T *__restrict__ r,
                                                 T *__restrict__ z, const TD *__restrict__ diag,
                                                 int jacobi, const SolveState *st, double *part) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    double rz = 0.0;
    if (i < N && jacobi) {
        const T ri = r[i];
        const T zi = (T)((double)ri * inv_kd(diag, i, st->cg.dt));
        z[i] = zi;
        rz = (double)ri * (double)zi;
    }
    block_partial_sum(rz, part);
}

__global__ __launch_bounds__(kBS) void k_restart_fin(SolveState *st, const double *part,
                                                     long long nb) {
    const double t = reduce_partials(part, nb);
    if (threadIdx.x != 0) return;
    st->cg.rz = t;
    st->cg.beta = 0.0;
    st->cg.rr = st->rr_true;
    st->cg.done = 0;
}

template <typename TA, typename TB> __global__ void k_convert(long long N, const TA *a, TB *b) {
    const long long i = (long long)blockIdx.x * kBS + threadIdx.x;
    if (i < N) b[i] = (TB)a[i];
}

// Most dot partials the inference leaves: the 2D fused kernel's persistent
// grid has at most 3 blocks per CU on 256 CUs; the 3D path leaves one per
// 8 x 8 x 4 tile.
constexpr size_t kDotParts = 768;

size_t dot_parts(const GridInfo &g) {
    const size_t nb = (size_t)((g.N + kBS - 1) / kBS);
    size_t m = std::max(nb, kDotParts);
    if (g.dim == 3)
        m = std::max(m, (size_t)((g.nx + 7) / 8) * ((g.ny + 7) / 8) * ((g.nz + 3) / 4));
    return m;
}

struct SolveLayout {
    size_t st, hist, part, x64, vec[6], total;
};

SolveLayout solve_layout(const GridInfo &g, size_t esz, int max_hist) {
    SolveLayout L;
    size_t o = 0;
    const long long N = g.N;
    const size_t nb = (size_t)((N + kBS - 1) / kBS);
    L.st = o;   o += align_up(sizeof(SolveState));
    L.hist = o; o += align_up(8 * (size_t)max_hist);
    // two regions of dot partials (up to dot_parts each), then |r|^2
    L.part = o; o += align_up(8 * (2 * dot_parts(g) + nb) + 64);
    L.x64 = o;  o += align_up(8 * (size_t)N);
    for (int k = 0; k < 6; ++k) {
        L.vec[k] = o;
        o += align_up(esz * (size_t)N);
    }
    L.total = o;
    return L;
}

constexpr int kMaxHist = 1 << 16;

template <typename T, typename TD>
int solve_impl(adlbr_operator *op, double dt, const T *b, T *x, const adlbr_solve_params *p,
               char *ws, adlbr_solve_report *rep, hipStream_t s) {
    const GridInfo &g = operator_grid(op);
    const long long N = g.N;
    const unsigned nb = (unsigned)((N + kBS - 1) / kBS);
    const SolveLayout L = solve_layout(g, sizeof(T), kMaxHist);
    SolveState *st = (SolveState *)(ws + L.st);
    double *hist = (double *)(ws + L.hist);
    double *part = (double *)(ws + L.part);
    // partials of |r|^2 of the flexible-CG update, after the dot partials
    double *prr = part + 2 * (long long)dot_parts(g);
    T *r = (T *)(ws + L.vec[0]);
    T *r2 = (T *)(ws + L.vec[1]);
    T *z = (T *)(ws + L.vec[2]);
    T *pv = (T *)(ws + L.vec[3]);
    T *q = (T *)(ws + L.vec[4]);
    double *x64 = (double *)(ws + L.x64);
    const TD *diag = (const TD *)operator_diag(op);
    const bool net = p->method == ADLBR_SOLVE_FCG_NET;
    CgState *cg = &st->cg;

    EventPair ev;
    ADLBR_CHECK_HIP(ev.create());
    const hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
    ADLBR_CHECK_HIP(hipEventRecord(e0, s));
    // clear the state, set dt
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st, dt);
    // the iterate is accumulated in FP64 (x64); the vectors and recurrences
    // are in the storage dtype
    if (!p->x0_zero) {
        hipLaunchKernelGGL((k_convert<T, double>), dim3(nb), dim3(kBS), 0, s, N, (const T *)x, x64);
        int rc = true_residual(op, dt, b, x64, &st->rr_true, part, r, s);
        if (rc) return rc;
    }
    hipLaunchKernelGGL((k_init<T, TD>), dim3(nb), dim3(kBS), 0, s, N, b, x64, r, z, diag,
                       p->x0_zero, (int)!net, (const SolveState *)st, part);
    hipLaunchKernelGGL(k_init_fin, dim3(1), dim3(kBS), 0, s, st, (const double *)part,
                       (long long)nb, p->tol * p->tol);
    int rc = ADLBR_OK;
    bool use_net = net;
    int fell_back = 0, net_iters = 0, restarts = 0, reason = 0;
    int first = 1;
    T *rc_ = r, *ro = r2;  // current and previous residual (flexible CG)
    auto start_iteration = [&]() -> int {
        if (use_net) {
            // z = N(r) with the dots <z, r>, <z, r_prev> fused where possible
            long long np = 0;
            int e = net_apply_dots(p->net, op, (const float *)rc_,
                                   first ? nullptr : (const float *)ro, (float *)z, part, &np, cg,
                                   s);
            if (e) return e;
            hipLaunchKernelGGL(k_fcg_scalars, dim3(1), dim3(kBS), 0, s, st, (const double *)part,
                               np, (const double *)prr, (long long)nb, hist, kMaxHist, first);
        }
        int e = cg_direction(op, z, q, pv, cg, part, first, s);
        first = 0;
        return e;
    };
    rc = start_iteration();
    if (rc) return rc;
    const int check = p->check_every > 0 ? p->check_every : 10;
    int issued = 0;
    bool converged = false;
    CgState h;
    // stall detection for the learned preconditioner: (iteration, |r|^2)
    // at each host check
    std::vector<std::pair<int, double>> trail;
    while (issued < p->max_iter) {
        const int batch = std::min(check, p->max_iter - issued);
        for (int k = 0; k < batch; ++k) {
            if (use_net) {
                hipLaunchKernelGGL((k_fcg_update<T>), dim3(nb), dim3(kBS), 0, s, N, x64,
                                   (const T *)rc_, ro, (const T *)pv, (const T *)q,
                                   (const SolveState *)st, prr);
                std::swap(rc_, ro);  // ro now holds r_k (previous), rc_ r_{k+1}
            } else {
                hipLaunchKernelGGL((k_pcg_update<T, TD>), dim3(nb), dim3(kBS), 0, s, N, x64, rc_, z,
                                   (const T *)pv, (const T *)q, diag, (const SolveState *)st, part);
                hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(kBS), 0, s, st, (const double *)part,
                                   (long long)nb, hist, kMaxHist);
            }
            rc = start_iteration();
            if (rc) return rc;
        }
        issued += batch;
        ADLBR_CHECK_HIP(hipMemcpyAsync(&h, cg, sizeof h, hipMemcpyDeviceToHost, s));
        ADLBR_CHECK_HIP(hipStreamSynchronize(s));
        if (use_net) {
            net_iters = h.iter;
            // stall: the smallest |r|^2 seen at the checks of the last 20
            // iterations is not (1%)^2 below the smallest one before them
            // (residual norms of CG are not monotone, hence the minima)
            double old_min = -1.0, new_min = h.rr;
            for (const auto &e : trail) {
                if (h.iter - e.first >= 20)
                    old_min = old_min < 0.0 ? e.second : std::min(old_min, e.second);
                else
                    new_min = std::min(new_min, e.second);
            }
            if (!h.done && !h.bad && old_min >= 0.0 && new_min > 0.99 * 0.99 * old_min) {
                h.bad = 1;
                reason = 2;
            }
            trail.emplace_back(h.iter, h.rr);
        }
        if (h.bad) {
            if (!use_net) break;  // Jacobi-PCG broke down: report as not converged
            // learned preconditioner failed: restart from x with Jacobi-PCG
            use_net = false;
            fell_back = 1;
            if (!reason) reason = 1;
            first = 1;
            const int keep_iter = h.iter;
            hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st, dt);
            rc = true_residual(op, dt, b, x64, &st->rr_true, part, r, s);
            if (rc) return rc;
            hipLaunchKernelGGL((k_init<T, TD>), dim3(nb), dim3(kBS), 0, s, N, b, x64, r, z, diag,
                               0, 1, (const SolveState *)st, part);
            hipLaunchKernelGGL(k_init_fin, dim3(1), dim3(kBS), 0, s, st, (const double *)part,
                               (long long)nb, p->tol * p->tol);
            rc_ = r;
            ro = r2;
            rc = start_iteration();
            if (rc) return rc;
            issued = keep_iter;
            net_iters = keep_iter;
            continue;
        }
        if (h.done) {
            rc = true_residual(op, dt, b, x64, &st->rr_true, part, nullptr, s);
            if (rc) return rc;
            double rt = 0.0, t2 = 0.0;
            ADLBR_CHECK_HIP(hipMemcpyAsync(&rt, &st->rr_true, 8, hipMemcpyDeviceToHost, s));
            ADLBR_CHECK_HIP(hipMemcpyAsync(&t2, &st->tol2bb, 8, hipMemcpyDeviceToHost, s));
            ADLBR_CHECK_HIP(hipStreamSynchronize(s));
            if (rt <= t2) {
                converged = true;
                break;
            }
            // the recurrence residual drifted from the true one: replace it
            // and restart the direction from the current iterate
            rc = true_residual(op, dt, b, x64, &st->rr_true, part, rc_, s);
            if (rc) return rc;
            hipLaunchKernelGGL((k_restart<T, TD>), dim3(nb), dim3(kBS), 0, s, N, (const T *)rc_, z,
                               diag, (int)!use_net, (const SolveState *)st, part);
            hipLaunchKernelGGL(k_restart_fin, dim3(1), dim3(kBS), 0, s, st, (const double *)part,
                               (long long)nb);
            first = 1;
            rc = start_iteration();
            if (rc) return rc;
            trail.clear();
            ++restarts;
        }
    }
    // final report (a confirmed convergence has just computed the true
    // residual of this x)
    int32_t iters = 0;
    double bb = 0.0;
    if (!converged) {
        rc = true_residual(op, dt, b, x64, &st->rr_true, part, nullptr, s);
        if (rc) return rc;
    }
    hipLaunchKernelGGL((k_convert<double, T>), dim3(nb), dim3(kBS), 0, s, N, (const double *)x64, x);
    double rt = 0.0;
    ADLBR_CHECK_HIP(hipMemcpyAsync(&iters, &cg->iter, 4, hipMemcpyDeviceToHost, s));
    ADLBR_CHECK_HIP(hipMemcpyAsync(&bb, &cg->bb, 8, hipMemcpyDeviceToHost, s));
    ADLBR_CHECK_HIP(hipMemcpyAsync(&rt, &st->rr_true, 8, hipMemcpyDeviceToHost, s));
    ADLBR_CHECK_HIP(hipEventRecord(e1, s));
    ADLBR_CHECK_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep) {
        rep->iters = fell_back ? net_iters + iters : iters;
        rep->converged = converged;
        rep->fell_back = fell_back;
        rep->net_iters = net ? (fell_back ? net_iters : iters) : 0;
        rep->rel_res = bb > 0.0 ? sqrt(rt / bb) : 0.0;
        rep->time_ms = ms;
        rep->restarts = restarts;
        rep->fallback_reason = reason;
    }
    if (!converged) {
        set_error("adlbr_solve: not converged after %d iterations (relative residual %.3e)",
                  rep ? rep->iters : iters, bb > 0.0 ? sqrt(rt / bb) : 0.0);
        return ADLBR_E_NOT_CONVERGED;
    }
    return ADLBR_OK;
}

}  // namespace
}  // namespace adlbr

using namespace adlbr;

extern "C" int adlbr_solve_workspace(adlbr_operator *op, int method, size_t *bytes) {
    clear_error();
    if (!op || !bytes || (method != ADLBR_SOLVE_JACOBI_PCG && method != ADLBR_SOLVE_FCG_NET)) {
        set_error("adlbr_solve_workspace: bad argument");
        return ADLBR_E_INVALID;
    }
    const int sto = operator_storage(op);
    if (sto != ADLBR_F32 && sto != ADLBR_F64) {
        set_error("adlbr_solve_workspace: the operator's storage must be ADLBR_F32 or ADLBR_F64");
        return ADLBR_E_UNSUPPORTED;
    }
    *bytes = solve_layout(operator_grid(op), dtype_size(sto), kMaxHist).total;
    return ADLBR_OK;
}

extern "C" int adlbr_solve(adlbr_operator *op, double dt, const void *b, void *x,
                           const adlbr_solve_params *p, void *workspace, size_t ws_bytes,
                           adlbr_solve_report *report, void *stream) {
    clear_error();
    if (!op || !b || !x || !p || !workspace || b == x) {
        set_error("adlbr_solve: null or aliased argument");
        return ADLBR_E_INVALID;
    }
    if (!(dt >= 0.0) || !(p->tol > 0.0) || p->max_iter < 1 ||
        (p->method != ADLBR_SOLVE_JACOBI_PCG && p->method != ADLBR_SOLVE_FCG_NET) ||
        (p->method == ADLBR_SOLVE_FCG_NET && !p->net)) {
        set_error("adlbr_solve: need dt >= 0, tol > 0, max_iter >= 1, a known method (and a net for FCG)");
        return ADLBR_E_INVALID;
    }
    if (operator_tiled(op)) {
        set_error("adlbr_solve: the operator has the tiled layout; the solvers need the list "
                  "layout (create it without ADLBR_OP_TILED)");
        return ADLBR_E_UNSUPPORTED;
    }
    size_t need = 0;
    int rc = adlbr_solve_workspace(op, p->method, &need);
    if (rc) return rc;
    if (ws_bytes < need) {
        set_error("adlbr_solve: workspace has %zu bytes, %zu needed", ws_bytes, need);
        return ADLBR_E_NOMEM;
    }
    hipStream_t s = as_stream(stream);
    if (operator_storage(op) == ADLBR_F32)
        return solve_impl<float, float>(op, dt, (const float *)b, (float *)x, p, (char *)workspace,
                                        report, s);
    return solve_impl<double, double>(op, dt, (const double *)b, (double *)x, p, (char *)workspace,
                                      report, s);
}
