/*
 * ps.h -- two-stage preconditioned FGMRES for fully-implicit multiphase
 * poromechanics Jacobians on one AMD MI355X (gfx950).
 *
 * Method (White, Castelletto, Klevtsov, Bui, Osei-Kuffuor, Tchelepi, "A Two-Stage
 * Preconditioner for Multiphase Poromechanics in Reservoir Simulation"):
 *   - the Jacobian system of Sec. 4 (eq. jac_system) is solved with right-
 *     preconditioned (flexible) GMRES, Sec. 4;
 *   - the preconditioner is Algorithm 1: the block lower-triangular operator of
 *     eq. blk_tr_prec with a separate-displacement-component AMG for the
 *     mechanics (Sec. 5.2), the fixed-stress Schur approximation of eq.
 *     Schur_1_FS, and the two-stage CPR flow preconditioner of eq. mult_prec_op
 *     (quasi-IMPES global stage eq. S1_prec with a pressure AMG, then a local
 *     block-ILU(0) or block-Jacobi stage, Sec. 5.3);
 *   - setup and iteration phases are separate (Sec. 5.4); the mechanics AMG
 *     can be shared by handles whose displacement block is identical (Sec. 5.2).
 *
 * Conventions for every entry point:
 *   - Every call returns a status code (PS_OK = 0, errors < 0); nothing aborts.
 *   - Host arrays passed in are copied; the caller keeps ownership and may free
 *     them after the call returns.
 *   - Vectors passed to ps_solve / ps_submit / ps_apply_precond / ps_spmv are
 *     DEVICE pointers (HIP global memory, e.g. torch tensors on "cuda"), FP64,
 *     of length N = 3 n_nodes + nf n_cells, ordered
 *       [u_0x u_0y u_0z  u_1x ... | f_0,0 .. f_0,nf-1  f_1,0 ...]
 *     (displacements interleaved per node, then flow dofs interleaved per cell).
 *   - A handle is used by one host thread at a time; a context may be shared.
 */
#ifndef PS_H
#define PS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define PS_OK          0
#define PS_PENDING     1   /* ps_poll: request not finished yet */
#define PS_EINVAL     -1   /* bad shape, unsorted/duplicate columns, missing diagonal,
                              non-finite value, rtol <= 0, bad option */
#define PS_ENOMEM     -2   /* device or host allocation failed / over budget */
#define PS_EDEVICE    -3   /* a HIP runtime call failed */
#define PS_ENOTSETUP  -4   /* ps_solve before ps_setup */
#define PS_ESINGULAR  -5   /* singular D_ss block, BILU pivot block or coarse matrix */
#define PS_EMAXIT     -6   /* maxit reached; x holds the last iterate */
#define PS_EPRECISION -7   /* non-finite preconditioner output in the FP32 path */
#define PS_EBUSY      -8   /* context is shutting down / queue full */
#define PS_EBREAKDOWN -9   /* Arnoldi breakdown with a singular Hessenberg matrix */

/* ---- options ------------------------------------------------------------ */
#define PS_FP64       0    /* preconditioner data and arithmetic in FP64 */
#define PS_FP32_PREC  1    /* preconditioner in FP32; FGMRES, A z, residual in FP64 */
#define PS_CHEB2      0    /* AMG smoother: Chebyshev degree 2 on D^-1 A */
#define PS_L1JAC      1    /* AMG smoother: l1-Jacobi */
#define PS_BILU0      0    /* local stage M_L: block ILU(0) on S_ff^(fs) */
#define PS_BJACOBI    1    /* local stage M_L: block Jacobi on S_ff^(fs) */
#define PS_MCGS       2    /* local stage M_L: hybrid block Gauss-Seidel in multicolour order */
#define PS_FGMRES      0   /* outer iteration: right-preconditioned flexible GMRES (Sec. 4) */
#define PS_RICHARDSON  1   /* outer iteration: x += M^-1 (b - A x), the sequential fixed-stress
                              scheme (remark after Algorithm 1) */
#define PS_QUASI_IMPES 0   /* D_ss, D_ps: diagonal (cell) blocks of A_ss, A_ps (Sec. 5.3) */
#define PS_TRUE_IMPES  1   /* D_ss, D_ps: column-sum lumping, eq. CPR_CSL (Sec. 5.3) */
#define PS_FS_GIVEN    0   /* fixed-stress diagonals: the system's d_sp, d_pp (eq. FS_Dps_Dpp) */
#define PS_FS_RSL      1   /* fixed-stress diagonals by row-sum lumping, eq. FS_RSL: -diag(A_fu
                              A_uu^-1 A_up e), with A_uu^-1 approximated by fs_iters Richardson
                              steps preconditioned by the mechanics V-cycle */
#define PS_CGS2        0   /* classical Gram-Schmidt applied twice: three passes over the basis
                              per iteration */
#define PS_DCGS2       1   /* classical Gram-Schmidt with delayed re-orthogonalisation (Bielich
                              et al., Parallel Computing 112, 2022): the vector entering the
                              preconditioner has had one pass; its second pass and its
                              normalisation share the next iteration's pass over the basis,
                              so two passes per iteration.  Same iterates in exact arithmetic */

/* Block CSR matrix (host arrays).  Row-major br x bc blocks; rowptr has nbrows+1
 * entries starting at 0; colind sorted and unique within each block row. */
typedef struct {
    int32_t nbrows, nbcols, br, bc, nblocks;
    const int32_t *rowptr;
    const int32_t *colind;
    const double  *vals;     /* nblocks * br * bc */
} ps_bsr;

/* One linearised system, eq. jac_system partitioned as in eq. LU.
 * Auu: 3x3 blocks (n_nodes x n_nodes), diagonal block present in every row.
 * Auf: 3 x nf blocks (n_nodes x n_cells); contains A_us and A_up.
 * Afu: nf x 3 blocks (n_cells x n_nodes); contains A_su and A_pu.
 * Aff: nf x nf blocks (n_cells x n_cells), interleaved {s.., p} per cell (the
 *      permutation P of Sec. 5.3 is the identity), diagonal block in every row.
 * d_sp: n_cells * (nf-1) fixed-stress entries added to the (s_l, p) entry of
 *       each diagonal cell block; d_pp: n_cells entries added to (p, p)
 *       (eq. FS_Dps_Dpp and the multi-component remark after it).
 * nf: 2 or 3.  p_index: which cell dof is the pressure (and which cell row the
 * pressure equation); this library requires p_index == nf - 1.
 * mech_key: non-zero -> handles created with the same key in one context have
 * identical A_uu and share one mechanics AMG hierarchy (Sec. 5.2: set up once).
 * Handles whose hierarchy options differ (smoother, theta, coarse_max,
 * max_levels) get a hierarchy of their own; a handle whose A_uu pattern (node
 * count, block count, row pointers and columns) differs from the one the shared
 * hierarchy was built for is refused by ps_create with PS_EINVAL.
 * ml_part: optional (NULL = none) subdomain id of each cell.  With it the BILU(0)
 * local stage is processor-local as in the paper's second example (Sec. 6): the
 * factorisation drops the couplings between cells of different subdomains, which
 * shortens the chain of dependent sweep levels; step 6 still uses all of S_ff^(fs). */
typedef struct {
    int32_t n_nodes, n_cells, nf, p_index;
    ps_bsr Auu, Auf, Afu, Aff;
    const double *d_sp;
    const double *d_pp;
    uint64_t mech_key;
    const int32_t *ml_part;
} ps_system;

typedef struct {
    int32_t precision;    /* PS_FP64 | PS_FP32_PREC                       (PS_FP64)   */
    int32_t restart;      /* FGMRES restart length m, 1..200              (100)       */
    int32_t maxit;        /* total iteration cap                          (1000)      */
    int32_t smoother;     /* PS_CHEB2 | PS_L1JAC                          (PS_CHEB2)  */
    int32_t ml_kind;      /* PS_BILU0 | PS_BJACOBI | PS_MCGS              (PS_BILU0)  */
    int32_t ml_sweeps;    /* sweeps of the local stage, 1..16             (1)         */
    int32_t coarse_max;   /* AMG: stop coarsening at n <= coarse_max      (256)       */
    int32_t max_levels;   /* AMG: at most this many levels                (25)        */
    int32_t fp32_fallback;/* FP32 path: retry in FP64 on PS_EPRECISION    (0)         */
    double  theta;        /* AMG strength threshold                       (0.25)      */
    int32_t method;       /* PS_FGMRES | PS_RICHARDSON                    (PS_FGMRES) */
    int32_t reduction;    /* PS_QUASI_IMPES | PS_TRUE_IMPES               (quasi)     */
    int32_t fixed_stress; /* PS_FS_GIVEN | PS_FS_RSL                      (given)     */
    int32_t fs_iters;     /* PS_FS_RSL: V-cycle iterations for A_uu^-1    (10)        */
    int32_t orth;         /* FGMRES Arnoldi step: PS_CGS2 | PS_DCGS2      (PS_CGS2)   */
} ps_options;

typedef struct {
    int32_t status, iterations, restarts;
    double  rel_residual;   /* true |b - A x| / |b| in FP64 at return */
    double  setup_s, solve_s;
} ps_result;

typedef struct ps_ctx ps_ctx;
typedef struct ps_handle ps_handle;

/* Fill *o with the defaults listed above. */
void ps_default_options(ps_options *o);

/* Context for one HIP device.  hbm_budget_bytes bounds the device memory of the
 * handles that the serving scheduler admits concurrently (0 = 90% of free). */
int  ps_ctx_create(int device, size_t hbm_budget_bytes, ps_ctx **out);
void ps_ctx_destroy(ps_ctx *ctx);

/* Validate and copy a system (host arrays) into a new handle; the FP64 system
 * matrix is uploaded to the device.  opts may be NULL (defaults). */
int  ps_create(ps_ctx *ctx, const ps_system *sys, const ps_options *opts, ps_handle **out);

/* Replace the state-dependent blocks (Afu, Aff values, d_sp, d_pp and optionally
 * Auf; same patterns; NULL = unchanged) as after a Newton step (Sec. 4): the values are
 * copied into the device layout in place, A_uu and the mechanics hierarchy stay (Sec.
 * 5.2: built once); the next ps_setup rebuilds the flow stage only (Sec. 5.4).  Host
 * arrays, copied; PS_EINVAL on a non-finite value, PS_EBUSY while a request is in
 * flight. */
int  ps_update_flow(ps_handle *h, const double *afu_vals, const double *aff_vals,
                    const double *d_sp, const double *d_pp, const double *auf_vals);

/* Setup phase (Sec. 5.4): fixed-stress and quasi-IMPES operators, pressure AMG,
 * BILU(0) factors, FP32 mirrors; the mechanics AMG is built on the first call
 * (or taken from another handle with the same mech_key) and kept.  Every call
 * rebuilds the flow stage: the first on host threads and the device (it also lays out
 * the patterns), later ones, with l1-Jacobi smoothing and subdomain BILU(0), on the
 * device from the system's A_ff and fixed-stress terms, with the same results bit for
 * bit.  Synchronous. */
int  ps_setup(ps_handle *h);

/* Solve A x = rhs to |b - A x| <= rtol |b| with FGMRES(restart) and Algorithm 1
 * (Sec. 4, right preconditioning), or with options.method = PS_RICHARDSON by the
 * preconditioned Richardson iteration x += M^-1 (b - A x) (the sequential fixed-stress
 * scheme of the remark after Algorithm 1; `iterations` counts its steps, `restarts` is
 * 0).  rhs, x: device pointers (N doubles); x is overwritten (x0 = 0).  stream: a
 * hipStream_t or NULL for the legacy default stream.  Blocking; res may be NULL. */
int  ps_solve(ps_handle *h, const double *rhs, double *x, double rtol, void *stream,
              ps_result *res);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ps_solve with the FGMRES
 * workspace -- the basis V ((restart+1) x N FP64), Z (restart x N, FP32 in the FP32
 * path, else FP64), the Hessenberg matrix, rotations, reduction partials and the
 * residual vector -- placed in a static device array of PS_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device it runs on until the process ends.  The call
 * allocates nothing: the handle must be set up (ps_setup allocates the preconditioner),
 * and the array's device address and a 64-byte pinned scalar mirror are set up once per
 * device by ps_ctx_create.  Same arguments, results and statuses as ps_solve, except:
 *  - PS_EINVAL when the workspace does not fit: about (restart+1) N 8 + restart N s
 *    + N 8 bytes (s = 4 in the FP32 path, 8 otherwise), so N <= about 220,000 at
 *    restart 100 with the FP32 preconditioner (the 16^3 to 32^3 grids);
 *  - no FP64 retry after PS_EPRECISION (fp32_fallback is ignored).
 * Every call on a device shares that device's array, which keeps the last call's
 * contents: calls on one device are serialised by a lock inside the library (two
 * processes on one device each have their own copy); the call is blocking. */
#define PS_NOALLOC_SCRATCH_BYTES (256u << 20)
int  ps_solve_noalloc(ps_handle *h, const double *rhs, double *x, double rtol, void *stream,
                      ps_result *res);

/* One application of the preconditioner, z = M^{-1} v (Algorithm 1), in the
 * handle's precision (v, z device FP64 arrays of length N).  Stream-ordered: the
 * work is enqueued on `stream` and the call returns without waiting for it. */
int  ps_apply_precond(ps_handle *h, const double *v, double *z, void *stream);

/* y = A x with the full FP64 system matrix (device arrays of length N).
 * Stream-ordered like ps_apply_precond. */
int  ps_spmv(ps_handle *h, const double *x, double *y, void *stream);

/* Serving: enqueue a solve (FGMRES only: PS_EINVAL for PS_RICHARDSON); rhs/x must
 * stay valid until completion.  The
 * context's scheduler admits requests by device-memory footprint and advances
 * each admitted request by one FGMRES iteration (or cycle end) as soon as its
 * previous one has completed, on the request's own stream (continuous batching).
 * Work already enqueued on `stream` (e.g. the copy that fills rhs) completes
 * before the request starts; NULL = legacy default stream. */
int  ps_submit(ps_handle *h, const double *rhs, double *x, double rtol, void *stream, uint64_t *ticket);
/* Step 1 of the admitted requests that share a mechanics hierarchy (same mech_key grid
 * and precision) and are ready together runs as one batch: each V-cycle kernel is launched
 * once for up to 8 requests (gridDim.y), reading the shared level operators once per
 * request slice, with every slice computing what the request computes alone (results are
 * bitwise those of a solo solve).  PS_SERVING_BATCH=0 in the environment turns it off.
 * ps_ctx_batches reports, since ps_ctx_create, the batched step-1 launch sequences and the
 * requests they covered (NULL to skip). */
int  ps_ctx_batches(ps_ctx *ctx, uint64_t *launches, uint64_t *requests);
/* PS_PENDING while running; the request's final status once done (result copied). */
int  ps_poll(ps_ctx *ctx, uint64_t ticket, ps_result *res);
/* Block until the request finishes; returns its status. */
int  ps_wait(ps_ctx *ctx, uint64_t ticket, ps_result *res);

/* Device bytes held by the handle (system matrix, hierarchy, Krylov space). */
int  ps_footprint(ps_handle *h, size_t *bytes);

/* Instrumentation.  ps_kernel_timing(mask) clears the totals and starts bracketing the
 * instrumented kernels whose bit is set -- bit i for kernel idx i of ps_kernel_stats: the
 * system SpMV (both block-row kernels, idx 0), the three CGS2 passes over the Krylov basis,
 * the subdomain BILU(0) sweeps, and the level-0 pre-smoothing, restriction, prolongation
 * and post-smoothing of the SDC and the pressure V-cycles -- with HIP events recorded on
 * the stream each runs on, adding each launch's algorithmic bytes (values, indices and
 * vectors the kernel must move, not what the caches do).  PS_KT_ALL brackets every one;
 * 0 stops.  Each bracket adds two event records (a few microseconds) to the stream, so a
 * timed run brackets only the kernels it reports.  Process-wide. */
#define PS_KT_ALL (-1)
int  ps_kernel_timing(int enable);
/* Totals of instrumented kernel idx = 0, 1, ... (PS_EINVAL past the last): its name
 * (NUL-terminated, truncated to len bytes), launches, event seconds and algorithmic
 * bytes.  Waits for the events still pending. */
int  ps_kernel_stats(int idx, char *name, size_t len, int64_t *launches, double *seconds, double *bytes);

/* Level `lvl` of the quasi-IMPES pressure AMG hierarchy built by the last ps_setup
 * (Sec. 5.3, M_pp = amg(S_pp)); its coarse operators R (A P) are formed on the device
 * (PS_GALERKIN=host in the environment: on host threads; the two agree bit for bit).
 * Copies into caller buffers, NULL to skip: *nlevels, the level's operator (n x n,
 * nnz entries, CSR with sorted columns: rowptr[n+1], colind[nnz], vals[nnz]) and its
 * C/F splitting cf[n] (1 = C, -1 = F, 0 on the coarsest level).  For inspection and
 * tests; PS_ENOTSETUP before the first ps_setup, PS_EINVAL for a level out of range. */
int  ps_pressure_level(ps_handle *h, int lvl, int32_t *nlevels, int32_t *n, int32_t *nnz, int32_t *rowptr,
                       int32_t *colind, double *vals, int8_t *cf);

/* Release a handle.  A handle created with a non-zero mech_key and set up is kept by
 * its context (at most 4 per key, within a quarter of the context's budget) and given to
 * the next ps_create whose system has the same mech_key, options, sizes, block patterns
 * and ml_part: that handle keeps the device layouts and workspaces, takes the new
 * system's values, and its first ps_setup runs the device path (what serving requests on
 * an already-served grid need).  Other handles are freed; ps_ctx_destroy frees the kept
 * ones. */
void ps_destroy(ps_handle *h);
const char *ps_strerror(int status);
/* Message of the last error raised on the calling thread ("" if none). */
const char *ps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PS_H */
