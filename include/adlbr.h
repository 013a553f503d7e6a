/*
 * adlbr.h -- C ABI of the MI355X AD-LBR library (libadlbr.so).
 *
 * AD-LBR (Fehrenbach & Mirebeau, "Sparse non-negative stencils for
 * anisotropic diffusion") discretizes the energy E(u) = int |grad u|_D^2
 * (Section 1) on a Cartesian grid with, at every point z, a symmetric stencil
 * V(z) of at most 6 (2D) or 12 (3D) integer offsets and non-negative weights
 * gamma_z (eq. (def:E*)).  This library builds those stencils on the GPU,
 * assembles the operator A = 1/2 grad E_h for a gather-based apply, steps
 * du/dt = -A u explicitly, computes solution-dependent tensors from the
 * structure tensor, and solves (I + dt A) x = b.
 *
 * Conventions shared by every entry point
 *  - Grids: n[0] is x (fastest), then y, then z; point index
 *    z = x + n0*(y + n1*z).  Grid spacing h = 1 (a caller with h != 1 scales
 *    dt by h^-2).  N = n0*n1[*n2] must be < 2^28.
 *  - Tensor fields are structure-of-arrays planes: 2D (Dxx, Dxy, Dyy) as
 *    [3][N]; 3D (Dxx, Dxy, Dxz, Dyy, Dyz, Dzz) as [6][N].
 *  - Stencils are exported as K/2 representative offsets ("slots") per point
 *    (K/2 = 3 in 2D, 6 in 3D); V(z) is {+o, -o : o a slot} and gamma(+-o) is
 *    the slot's weight.  offsets: int16 [K/2][d][N]; weights: [K/2][N].
 *  - Every pointer argument named as device memory must point to GPU memory
 *    of the current HIP device; host pointers are marked "host".  The caller
 *    owns all memory.  The library never allocates device memory: calls that
 *    need scratch take a caller-allocated workspace whose size a *_workspace
 *    query returns.  Opaque plan objects (adlbr_operator) live in host
 *    memory and hold only pointers into the caller's workspace.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous on `stream` unless they return a value through a host
 *    pointer, which synchronizes `stream`.
 *  - Return value: ADLBR_OK (0) or a negative ADLBR_E_* code; the message of
 *    the last failing call on the calling thread is adlbr_last_error().  No
 *    C++ exception crosses this boundary.  Data-dependent problems detected
 *    on the device (a tensor that is not SPD, an offset out of range) are
 *    reported through a caller-provided device status word instead, so that
 *    no call has to synchronize.
 *  - Device status words (int32[2], device): [0] = smallest offending point
 *    index or -1, [1] = OR of ADLBR_ST_* flags.  Each call that takes one
 *    resets it first.
 */
#ifndef ADLBR_H
#define ADLBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define ADLBR_OK               0
#define ADLBR_E_INVALID       (-1) /* bad argument (null pointer, size, dtype) */
#define ADLBR_E_NOT_SPD       (-2) /* reserved for host-side checks          */
#define ADLBR_E_RANGE         (-3) /* size outside the supported range       */
#define ADLBR_E_NOMEM         (-4) /* workspace smaller than required        */
#define ADLBR_E_HIP           (-5) /* a HIP runtime call failed              */
#define ADLBR_E_NOT_CONVERGED (-6) /* solver hit max_iter                    */
#define ADLBR_E_UNSUPPORTED   (-7) /* combination not implemented            */

/* device status flags */
#define ADLBR_ST_NOT_SPD   1  /* tensor not symmetric positive definite or not finite */
#define ADLBR_ST_RANGE     2  /* an offset does not fit the storage format           */
#define ADLBR_ST_ITER      4  /* reduction iteration cap reached                     */
#define ADLBR_ST_CLAMPED   8  /* a weight rounded below 0 was clamped to 0 (benign)  */
#define ADLBR_ST_STENCIL  16  /* slots are not built from a superbase                */
#define ADLBR_ST_INCOMING 32  /* more than 255 stencils reach one point              */

typedef enum { ADLBR_F64 = 0, ADLBR_F32 = 1, ADLBR_BF16 = 2, ADLBR_F16 = 3 } adlbr_dtype;
/* Boundary of the operator: an edge whose target leaves the grid is
 * dropped (ADLBR_NEUMANN: the truncation V(z;h) of Section 1), wrapped
 * (ADLBR_PERIODIC) or mirrored back at the half-sample points -1/2 and
 * n - 1/2 (ADLBR_REFLECT: u extended evenly, the reflecting boundary of the
 * restoration test, Section 4).  A folded target that is the point itself
 * is no edge. */
typedef enum { ADLBR_NEUMANN = 0, ADLBR_PERIODIC = 1, ADLBR_REFLECT = 2 } adlbr_boundary;

typedef struct adlbr_grid {
    int32_t dim;      /* 2 or 3 */
    int32_t boundary; /* adlbr_boundary */
    int64_t n[3];     /* n[2] ignored in 2D */
} adlbr_grid;

typedef struct adlbr_operator adlbr_operator;

/* Message of the last failing call on this thread ("" if none). */
const char *adlbr_last_error(void);

/* ABI version (major*100 + minor). */
int adlbr_version(void);

/* ------------------------------------------------------------------ *
 * Stencil construction (Section 2).
 * 2D: Lagrange's reduction (eq. (GaussAlgo)) of Z^2 for the metric
 * M ~ adj(D) starting from the canonical basis; flip f when <e, M f> > 0
 * (Corollary 2); superbase (e, f, g = -e-f); weights
 * gamma(+-e_i) = -1/2 <e_{i+1}^perp, D e_{i+2}^perp> (Lemma 1, eq.
 * (def:GammaZ)).  Slots are exported in the order (e, f, g).
 * 3D: greedy D-reduced basis (Definition 2), Proposition (MakeObtuse),
 * then Selling's decomposition: for pairs (i,j) in the order (0,1), (0,2),
 * (0,3), (1,2), (1,3), (2,3), slot c_ij = e_k x e_l ({k<l} the complement)
 * with weight -1/2 <e_i, D e_j>.
 * All decisions are taken in FP64; offsets are exact integers.
 *
 *   D        device, [3|6][N] of D_dtype (ADLBR_F64 or ADLBR_F32)
 *   offsets  device out, int16 [K/2][d][N]
 *   weights  device out, [K/2][N] of w_dtype (ADLBR_F64 or ADLBR_F32)
 *   status   device out, int32[2]; flags NOT_SPD, RANGE, ITER (the point's
 *            slots and weights are then written as 0), CLAMPED.
 * Errors: ADLBR_E_INVALID for null pointers, dim not 2/3, N out of range
 * or an unsupported dtype.
 * ------------------------------------------------------------------ */
int adlbr_build_stencils(const adlbr_grid *g, const void *D, int D_dtype,
                         int16_t *offsets, void *weights, int w_dtype,
                         int32_t *status, void *stream);

/* ------------------------------------------------------------------ *
 * Operator assembly: A = 1/2 grad E_h with E_h of eq. (def:E*), h = 1.
 * Row z of A gathers the point's own slots and every other point's slot
 * that reaches z:
 *   (A u)(z) = sum_{o in V(z;h)} gamma_z(o) (u(z) - u(z+o))
 *            + sum_{(y,o): o in V(y;h), y+o = z} gamma_y(o) (u(z) - u(y)).
 * V(z;h) drops offsets that leave the grid (Neumann truncation, Section 1);
 * with ADLBR_PERIODIC they wrap instead.  The incoming lists are built once
 * here, sorted per row, so every apply is deterministic.
 *
 * The slots must come from a superbase, as adlbr_build_stencils writes them
 * (2D: o2 = -o0-o1; 3D: o3 = -(o0+o1), o4 = o0-o2, o5 = o1+o2); otherwise
 * status gets ADLBR_ST_STENCIL.  Compact offsets are stored as int8 unless
 * flags has ADLBR_OP_WIDE (int16); an offset that does not fit sets
 * ADLBR_ST_RANGE and that point keeps no edge (its weights are stored as 0,
 * so A stays symmetric).  A point reached by more than 255 stencils sets
 * ADLBR_ST_INCOMING; its row keeps 255 of them.  In both cases every
 * later call still reads only memory inside the workspace and the grid,
 * but A is not the operator of the input: the caller must check status.
 *
 * adlbr_operator_workspace: bytes of device workspace for this grid,
 *   storage dtype and flags (an upper bound, independent of the data).
 * adlbr_operator_create:
 *   offsets, weights  device, as exported by adlbr_build_stencils
 *                     (weights ADLBR_F64 or ADLBR_F32, given by w_dtype)
 *   storage           dtype in which the operator keeps its weights and in
 *                     which apply/step read and write u: ADLBR_F64 (FP64
 *                     arithmetic), ADLBR_F32, ADLBR_BF16 or ADLBR_F16 (FP32
 *                     arithmetic)
 *   workspace         device, >= adlbr_operator_workspace() bytes, must
 *                     outlive the operator
 *   status            device out, int32[2]
 *   op                host out, the new plan; free with adlbr_operator_destroy
 * ------------------------------------------------------------------ */
#define ADLBR_OP_WIDE 1
/* Tiled layout (Neumann grids, storage F32, BF16 or F16): the explicit step
 * stages u over a tile of targets and its halo h in LDS; edges whose offset
 * components are all within h (h = the operator's largest offset
 * component, capped at 8 in 2D and 2 in 3D) are found from the staged
 * sources instead of being listed, and only the longer edges keep incoming
 * lists.  Apply, step, batches, dt_cfl and the diagonal work as with the
 * list layout (results equal to rounding; each layout is deterministic);
 * adlbr_solve and the residual need the list layout (ADLBR_E_UNSUPPORTED). */
#define ADLBR_OP_TILED 2
/* Records (list layout; 2D, since 3D operators always keep them): every
 * incoming entry is also stored with its edge's weight (8 bytes per edge
 * for F32 storage, entry and weight side by side), and a batch of such 2D
 * operators reads the weight from there instead of gathering it from the
 * source's weights.  The batch's grouped step is faster; the assembly
 * writes the extra 6 x N records per rebuild and the workspace grows by
 * them.  Single-operator calls (apply, step, solve) read the lists as
 * without the flag, and results are bit-identical either way.  Operators
 * with and without records fall in different batch classes.  With
 * ADLBR_OP_TILED: ADLBR_E_UNSUPPORTED. */
#define ADLBR_OP_RECORDS 4

int adlbr_operator_workspace(const adlbr_grid *g, int storage, int flags,
                             size_t *bytes);
int adlbr_operator_create(const adlbr_grid *g, const int16_t *offsets,
                          const void *weights, int w_dtype, int storage,
                          int flags, void *workspace, size_t ws_bytes,
                          int32_t *status, void *stream, adlbr_operator **op);
int adlbr_operator_destroy(adlbr_operator *op);
/* Rebuild op in place from new stencils of the same grid (offsets and
 * weights as for adlbr_operator_create; the storage dtype and flags stay):
 * the stencils change when D does, e.g. every few steps of coherence-
 * enhancing diffusion (Section 4).  The operator keeps its workspace and
 * every device address in it, so batches and captured graphs that use op
 * stay valid.  Asynchronous on `stream`; status as for create. */
int adlbr_operator_rebuild(adlbr_operator *op, const int16_t *offsets, const void *weights,
                           int w_dtype, int32_t *status, void *stream);

/* Largest explicit-Euler step keeping I - dt A entrywise non-negative
 * (discrete maximum principle): 1 / max_z A_zz.  Host out; synchronizes. */
int adlbr_operator_dt_cfl(adlbr_operator *op, double *dt_max, void *stream);

/* The diagonal A_zz (device out, [N] of dtype ADLBR_F64 or ADLBR_F32). */
int adlbr_operator_diagonal(adlbr_operator *op, void *diag, int dtype,
                            void *stream);

/* Au = A u.  u, Au: device [N] in the operator's storage dtype; must not
 * alias. */
int adlbr_apply(adlbr_operator *op, const void *u, void *Au, void *stream);

/* Explicit Euler, u^{n+1} = u^n - dt A u^n (Section 4), nsteps times.
 * u: device [N] in/out (storage dtype); u_tmp: device [N] scratch of the
 * same dtype.  dt_mode ADLBR_DT_ABS: dt is the step; ADLBR_DT_CFL: the step
 * is dt * (1 / max A_zz), read on the device (no synchronization). */
#define ADLBR_DT_ABS 0
#define ADLBR_DT_CFL 1
int adlbr_step(adlbr_operator *op, void *u, void *u_tmp, double dt,
               int dt_mode, int64_t nsteps, void *stream);

/* Explicit steps of a vector-valued image (the Conclusion: AD-LBR applies to
 * each component independently; the components are coupled only through
 * the common tensor, e.g. adlbr_structure_tensor_vec).
 * u, u_tmp: device [ncomp][N] planes of the storage dtype (u in/out).  Up
 * to four components share one kernel that loads each row's stencil and
 * incoming lists once; every component is bit-identical to adlbr_step on
 * that component alone.  List layout only (ADLBR_E_UNSUPPORTED for the
 * tiled layout). */
int adlbr_step_multi(adlbr_operator *op, void *u, void *u_tmp, int ncomp, double dt,
                     int dt_mode, int64_t nsteps, void *stream);

/* ------------------------------------------------------------------ *
 * Batched explicit steps (an extension: many images and volumes of uneven
 * sizes advanced together).  Every problem i is one operator ops[i] with
 * its state u[i] (device [N_i], in/out) and scratch u_tmp[i] (same size
 * and dtype), stepped as adlbr_step(ops[i], u[i], u_tmp[i], dt[i],
 * dt_mode, nsteps) would step it -- results are bit-identical.  Problems of
 * one class (dim, offset width, boundary, storage, 2D records) share one grouped
 * launch per step; adlbr_batch_run captures the nsteps of all classes
 * into one HIP graph (on the batch's own stream, ordered after and before
 * `stream` by events) and replays it on later calls with the same nsteps.
 * The operators and buffers must stay valid while the batch lives.
 *   workspace: device, >= adlbr_batch_workspace(nprob) bytes (descriptors).
 * ------------------------------------------------------------------ */
typedef struct adlbr_batch adlbr_batch;
int adlbr_batch_workspace(int nprob, size_t *bytes);
int adlbr_batch_create(int nprob, adlbr_operator *const *ops, void *const *u,
                       void *const *u_tmp, const double *dt, int dt_mode, void *workspace,
                       size_t ws_bytes, void *stream, adlbr_batch **batch);
/* Autotuner: for every class, time each launch variant with each chunk
 * budget over `steps` steps from u into u_tmp (u is not modified) and keep
 * the fastest; the choice is cached per process by class, total size and
 * problem count, and reused without timing when use_cache is set.
 * Variants, bit by bit: 0 = XCD-contiguous block order of the grouped
 * launch, 1 = largest problems first, 2 = one launch per problem instead of
 * one grouped launch (bits 0 and 2 together are not timed), 3 = two chunks
 * in flight: chunks 2i and 2i + 1 take their steps at the same time on two
 * streams (two branches of the captured graph), so that each step's launch
 * tail overlaps the other chunk's work (not timed without chunks).  Chunk
 * budgets (0, 64, 128, 224 MiB): the class is cut, in the variant's problem
 * order, into chunks whose working sets (u, u_tmp and the operator's
 * arrays) stay within the budget, and each chunk takes all its steps before
 * the next one starts, so that it runs out of the 256 MB last-level cache
 * (with bit 3, two chunks share it); 0 keeps the class whole.  Every choice
 * computes the same bits.  Synchronizes `stream`. */
int adlbr_batch_tune(adlbr_batch *batch, int steps, int use_cache, void *stream);
/* The tuner's cache on disk (a JSON file, so that one process's timings
 * serve later ones):
 *   {"format": "adlbr-batch-tune", "version": 1, "entries": [
 *     {"class": K, "log2_points": L, "problems": P, "variant": V,
 *      "chunk_bytes": B}, ...]}
 * with K the class key (adlbr_batch_variant), L = floor(log2 of the class's
 * points), P its problem count.  save writes every choice this process
 * holds; load merges a file's entries into it (all or nothing:
 * ADLBR_E_INVALID, cache unchanged, on an unreadable or malformed file);
 * adlbr_batch_create and adlbr_batch_tune(use_cache = 1) then take a
 * class's cached choice without timing.  clear empties the process's cache;
 * lookup reports (found = 0/1) the choice for one class.  Host only. */
int adlbr_batch_tune_save(const char *path);
int adlbr_batch_tune_load(const char *path);
int adlbr_batch_tune_clear(void);
int adlbr_batch_tune_lookup(int class_key, int64_t points, int nprob, int *found, int *variant,
                            size_t *chunk_bytes);
/* Force launch variant (0..15) and chunk budget (bytes, 0 = no chunks; a
 * problem larger than the budget gets a chunk of its own) for class cls
 * instead of tuning.  Synchronizes `stream`; ADLBR_E_INVALID for a bad
 * class or variant. */
int adlbr_batch_set_variant(adlbr_batch *batch, int cls, int variant, size_t chunk_bytes,
                            void *stream);
/* Class cls (0-based, in order of first appearance): its class key
 * (records*100000 + tiled*10000 + dim*1000 + wide*100 + periodic*10 +
 * storage, records = 1 for 2D operators created with ADLBR_OP_RECORDS),
 * launch variant, number of
 * problems and, where the pointers are not NULL, number of chunks and chunk
 * budget in bytes.  ADLBR_E_INVALID past the last class. */
int adlbr_batch_variant(const adlbr_batch *batch, int cls, int *key, int *variant, int *nprob,
                        int *nchunks, size_t *chunk_bytes);
/* nsteps explicit steps of every problem; use_graph = 0 launches directly
 * on `stream` instead of through the captured graph.  The results land in
 * u (an odd nsteps ends with a grouped copy). */
int adlbr_batch_run(adlbr_batch *batch, int64_t nsteps, int use_graph, void *stream);
int adlbr_batch_destroy(adlbr_batch *batch);

/* ------------------------------------------------------------------ *
 * Solution-dependent diffusion tensor from the structure tensor
 * (Section 4, coherence-enhancing diffusion; edge-enhancing in 3D):
 *   u_sigma = K_sigma * u, J = K_rho * (grad u_sigma grad u_sigma^T),
 *   D = sum_k lambda_k v_k v_k^T over the eigenpairs (mu_k, v_k) of J,
 *   mu_1 >= mu_2 (>= mu_3), with
 *   ADLBR_MAP_CED: lambda_1 = alpha,
 *                  lambda_k = alpha + (1-alpha) exp(-C/(mu_1-mu_k)^2)
 *   ADLBR_MAP_EED: lambda_k = 1 - exp(-C/mu_k^2) for k < d, lambda_d = 1
 * sigma and rho are standard deviations; Gaussians truncated at
 * ceil(3 s) (s <= 10) and normalized; mirror boundary; central differences.
 *   u  device [N] (ADLBR_F32 or ADLBR_F64, = dtype); D device out
 *      [3|6][N] of dtype; workspace device >= adlbr_tensor_workspace().
 * ------------------------------------------------------------------ */
#define ADLBR_MAP_CED 0
#define ADLBR_MAP_EED 1
typedef struct adlbr_tensor_params {
    double sigma, rho, alpha, C;
    int32_t eig_map;
} adlbr_tensor_params;

int adlbr_tensor_workspace(const adlbr_grid *g, int dtype, size_t *bytes);
int adlbr_structure_tensor(const adlbr_grid *g, const void *u, int dtype,
                           const adlbr_tensor_params *p, void *D,
                           void *workspace, size_t ws_bytes, void *stream);

/* The common tensor of a vector-valued image (the Conclusion leaves the
 * coupling of components to the tensor, which is the caller's choice; this
 * is the usual one): J = K_rho * sum_c grad u_c,sigma grad u_c,sigma^T over
 * the ncomp >= 1 components, then the same eigenvalue map.  u: device
 * [ncomp][N] planes of dtype; the workspace is the single-component size.
 * ncomp = 1 is adlbr_structure_tensor (bit-identical). */
int adlbr_structure_tensor_vec(const adlbr_grid *g, const void *u, int ncomp, int dtype,
                               const adlbr_tensor_params *p, void *D,
                               void *workspace, size_t ws_bytes, void *stream);

/* adlbr_structure_tensor without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  The scratch is a device array
 * of 128 MiB that the library holds on every GPU it runs on until the
 * process ends; the call itself allocates nothing.  Same arguments and
 * results as adlbr_structure_tensor (bit-identical output); ADLBR_E_NOMEM
 * when adlbr_tensor_workspace() for this grid and dtype exceeds 128 MiB
 * (e.g. 2D FP32 up to 5.59e6 points, 3D FP32 up to 2.79e6).  All calls on
 * one GPU share that array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialized by the caller. */
int adlbr_structure_tensor_noalloc(const adlbr_grid *g, const void *u, int dtype,
                                   const adlbr_tensor_params *p, void *D, void *stream);

/* ------------------------------------------------------------------ *
 * Implicit step: solve K x = b with K = I + dt A by conjugate gradients.
 * This is the linear system of the restoration problem
 * -lambda div(D grad u) + u = v (Section 4, eq. (elliptic), lambda = dt,
 * which the paper solves by CG) and of one backward-Euler step of the
 * diffusion equation.  Vectors are in the operator's storage dtype, which
 * must be ADLBR_F32 or ADLBR_F64; scalars and dot products are FP64, and
 * the iterate itself is accumulated in FP64 (an FP32-rounded solution could
 * not reach a small true residual when |K| is large); x receives its
 * rounding and report.rel_res is the true residual of the FP64 iterate.
 *
 * ADLBR_SOLVE_JACOBI_PCG: preconditioned CG with P = diag(K)^-1.
 * ADLBR_SOLVE_FCG_NET:    flexible CG (truncation 1,
 *     beta_k = <z_k, r_k - r_{k-1}> / <z_{k-1}, r_{k-1}>) with the learned
 *     preconditioner z = r / diag(K) + N(r) of adlbr_net; if a direction is
 *     not a descent direction (<z, r> <= 0) or a value is not finite it
 *     restarts from the current x with Jacobi-PCG (report.fell_back = 1).
 * Stopping: every check_every iterations the host reads the recurrence
 * residual; when it is below tol |b| the true residual |b - K x| is
 * recomputed with FP64 accumulation and the solve stops if that is below
 * tol |b| too.  report (host out) then holds the iteration count and the
 * true relative residual.  Returns ADLBR_E_NOT_CONVERGED (report filled)
 * when max_iter is reached.
 *   b         device [N] right-hand side
 *   x         device [N] in/out: initial guess unless x0_zero, then solution
 *   workspace device >= adlbr_solve_workspace() bytes
 * Synchronizes `stream` (every check_every iterations and at the end).
 * ------------------------------------------------------------------ */
#define ADLBR_SOLVE_JACOBI_PCG 0
#define ADLBR_SOLVE_FCG_NET 1

/* ------------------------------------------------------------------ *
 * Learned preconditioner (an extension; the paper has none).
 *   z = r / diag(K) + N(r),  K = I + dt A,
 *   N = B^T diag(g2) B,  B = C2 diag(g1) C1,
 * C1, C2 zero-padded 3x3 (3x3x3) correlations (1 -> W -> W channels, no
 * bias); g1, g2 point-wise gates in (0, 1), G = [g1, g2] =
 * sigmoid(WB relu(conv(F; WA) + bA) + bB) (2W channels), computed once per
 * operator by a small gate net from per-point features
 *   F = [1/diag(K), dt w_q / diag(K) (S slots), D / tr D (3 or 6)],
 *   D = sum_{e in V(z)} gamma e e^T recovered from the stencil (eq. (DSum)).
 * N is linear in r and symmetric positive semi-definite, so the
 * preconditioner is SPD and flexible CG sees a fixed linear one.  It is
 * applied as four correlations C1, C2, C2^T, C1^T (a 1->W->W->W->1 stack).
 * params: FP32, in this order (T = 3^d taps, (dz,) dy, dx row-major over
 * offsets -1, 0, +1):
 *   WA [hidden][nfeat][T], bA [hidden], WB [2W][hidden], bB [2W],
 *   W1 [W][1][T], W2 [W][W][T].
 * The struct is plain data owned by the caller; every array is device
 * memory (N = the operator's grid points):
 *   features [nfeat][N] FP32   (adlbr_net_features)
 *   hidden   [hidden][N] FP32  pre-activation of the gate net (adlbr_net_gates)
 *   gates    [3W+1][N] FP32    gates of the four-layer stack, [g1, g2, g1, 1]
 *                              (adlbr_net_gates)
 *   gates8   [N][2W] uint8     g1, g2 per point as round(255 g) for the
 *                              inference kernel
 *   scratch  [2W][N] FP32      working planes of the FP32 forward path
 *   layers   [2W(W+1)T + 7168] FP32  weights of the four-layer stack, [W1,
 *                              W2, flip(W2)^T, flip(W1)^T], then the BF16
 *                              MFMA operands packed per lane (2D: all four
 *                              layers; 3D: the two W -> W layers)
 *                              (adlbr_net_gates)
 * adlbr_net_gates must run again after params change.
 * ------------------------------------------------------------------ */
typedef struct adlbr_net {
    int32_t dim;    /* 2 or 3 */
    int32_t width;  /* r-path channels, 16 */
    int32_t hidden; /* gate-net channels, 16 */
    int32_t nfeat;  /* 7 in 2D, 13 in 3D */
    float *params;
    float *features;
    float *hidden_act;
    float *gates;
    uint8_t *gates8;
    float *scratch;
    float *layers;
} adlbr_net;

/* Number of FP32 parameters for (dim, width, hidden). */
int adlbr_net_param_count(int dim, int width, int hidden, size_t *count);
/* Features of the operator at time step dt into net->features. */
int adlbr_net_features(adlbr_operator *op, double dt, adlbr_net *net, void *stream);
/* Gate net forward: net->hidden_act, net->gates and net->gates8, and the
 * expanded weights net->layers. */
int adlbr_net_gates(adlbr_operator *op, adlbr_net *net, void *stream);
/* z = r / diag(K) + N(r).  r, z: device [N] FP32.  If saved is not null
 * (device [3W+1][N] FP32) the pre-gate outputs of the four layers are kept
 * for adlbr_net_backward. */
int adlbr_net_forward(adlbr_operator *op, const adlbr_net *net, const float *r, float *z,
                      float *saved, void *stream);
/* The inference path flexible CG uses, with net->gates8 set: in 2D the
 * fused MFMA kernel (BF16 operands, FP32 accumulation, 8-bit gates); in 3D
 * (also net->scratch) the W -> W layers on MFMA and the thin layers in
 * FP32, BF16 activations between layers; otherwise the FP32 path of
 * adlbr_net_forward. */
int adlbr_net_precondition(adlbr_operator *op, const adlbr_net *net, const float *r, float *z,
                           void *stream);
/* Backward of sum(gz * z) for one sample: adds the r-path weight
 * gradients (W1, W2, both uses of each tied weight) to gparams (device,
 * param_count FP32) and the gradients of the four-layer gates to ggates
 * (device [3W+1][N] FP32).  workspace >= adlbr_net_workspace(). */
int adlbr_net_backward(adlbr_operator *op, const adlbr_net *net, const float *r,
                       const float *gz, const float *saved, float *gparams, float *ggates,
                       void *workspace, size_t ws_bytes, void *stream);
/* Backward through the gate net: adds the gate-net weight gradients from
 * ggates (accumulated over a batch) to gparams. */
int adlbr_net_gates_backward(adlbr_operator *op, const adlbr_net *net, const float *ggates,
                             float *gparams, void *workspace, size_t ws_bytes, void *stream);
int adlbr_net_workspace(adlbr_operator *op, const adlbr_net *net, size_t *bytes);
/* Energy loss of the preconditioned residual, the training objective:
 * loss += (1/2 z^T K z - z^T r) / (r^T r)  (device double), and
 * gz = (K z - r) / (r^T r).  r, z, gz: device [N] FP32. */
int adlbr_net_loss_grad(adlbr_operator *op, double dt, const float *r, const float *z,
                        float *gz, double *loss, void *workspace, size_t ws_bytes,
                        void *stream);
/* Adam step (step counts from 1) on the scaled gradient g = grad_scale *
 * grads (grad_scale > 0, e.g. 1/batch to average summed per-sample
 * gradients): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr mhat / (sqrt(vhat) + eps).  All device FP32 [n]. */
int adlbr_net_adam(float *params, const float *grads, float *m, float *v, int64_t n,
                   int32_t step, double grad_scale, double lr, double beta1, double beta2,
                   double eps, void *stream);
/* r = b - (I + dt A) x (device, the operator's storage dtype). */
int adlbr_residual(adlbr_operator *op, double dt, const void *b, const void *x, void *r,
                   void *stream);

typedef struct adlbr_solve_params {
    int32_t method;
    int32_t max_iter;
    int32_t check_every;
    int32_t x0_zero;
    double tol;
    const adlbr_net *net; /* required for ADLBR_SOLVE_FCG_NET */
} adlbr_solve_params;

typedef struct adlbr_solve_report {
    int32_t iters;
    int32_t converged;
    int32_t fell_back;
    int32_t net_iters; /* iterations done with the learned preconditioner */
    double rel_res;    /* true relative residual, FP64 */
    double time_ms;    /* wall time of the solve on the stream */
    int32_t restarts;  /* residual replacements (recurrence met tol, true residual did not) */
    int32_t fallback_reason; /* 0 none, 1 breakdown (<z,r> <= 0 or non-finite), 2 stall */
} adlbr_solve_report;

int adlbr_solve_workspace(adlbr_operator *op, int method, size_t *bytes);
int adlbr_solve(adlbr_operator *op, double dt, const void *b, void *x,
                const adlbr_solve_params *p, void *workspace, size_t ws_bytes,
                adlbr_solve_report *report, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ADLBR_H */
