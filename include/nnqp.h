/*
 * nnqp.h - C ABI of the MI355X (gfx950) non-negative diffusion QP library.
 *
 * The library assembles the P1 Galerkin stiffness matrix K of anisotropic
 * diffusion on a simplicial mesh and solves the bound-constrained quadratic
 * program
 *
 *     minimise 1/2 <c; K c> - <c; f>   subject to   0 <= c          (*)
 *
 * of Chang, Karra & Nakshatrala, arXiv:1506.08435, Sec. 2.1.3
 * (eq. non-negative), with an active-set projected-Newton / trust-region
 * method in the style of TRON (Lin & More, SIAM J. Optim. 9(4), 1999), the
 * solver the paper uses through TAO (Sec. 3.1).  Every step of the solve runs
 * in hand-written HIP kernels; the host only sequences launches and reads
 * back a few scalars.
 *
 * Conventions (apply to every entry point):
 *  - Every function returns nn_status; NN_OK (0) on success.  No C++
 *    exception crosses this boundary.  On error, nn_last_error(ctx) returns a
 *    message describing the last failure on that context.
 *  - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *    pointers are HIP device memory on the context's device, owned by the
 *    caller unless stated otherwise.  Nothing keeps a caller pointer after
 *    the call returns.
 *  - Vectors over the free degrees of freedom (DOFs) are dense float64
 *    arrays of length n (nn_matrix_info), in DOF order: the non-Dirichlet
 *    nodes in increasing node id.
 *  - All device work is enqueued on the context's stream.  Entry points that
 *    fill an nn_stats or return sizes synchronise that stream before
 *    returning; nn_matvec does not (it is stream-ordered).
 *  - A context is not thread-safe; use one context per host thread.
 *    Different contexts may run calls at the same time from different
 *    threads (each on its own stream).  A matrix may be used by any context
 *    on its device, but by one call at a time: solves add lazily formed
 *    copies to it (float32 values, paired layouts, M/dt + K).
 */
#ifndef NNQP_H
#define NNQP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NN_OK = 0,
    NN_EINVAL = 1,      /* bad argument: null pointer, size, dimension, option value */
    NN_ENONFINITE = 2,  /* NaN/Inf met in the input or during the iteration */
    NN_ENOTSPD = 3,     /* non-positive diagonal or curvature: K is not SPD on the free set */
    NN_EMAXIT = 4,      /* iteration cap reached; c holds the last feasible iterate */
    NN_EOOM = 5,        /* device or host allocation failed */
    NN_EHIP = 6,        /* a HIP runtime call failed */
    NN_EBUDGET = 7      /* request exceeds the byte budget given by the caller */
} nn_status;

typedef enum {
    NN_FP64 = 0,        /* all values, vectors and reductions in float64 */
    NN_MIXED = 1        /* float32 K values and CG vectors, float64 reductions,
                           float64 outer iterative-refinement residual f - K c */
} nn_precision;

typedef struct nn_ctx nn_ctx;        /* opaque; one device + one stream */
typedef struct nn_matrix nn_matrix;  /* opaque; device CSR owned by the library */

/* Simplicial mesh (host arrays, row-major).  P1 elements: triangles for
 * dim = 2, tetrahedra for dim = 3 (Sec. 2.1.3, P^k spaces with k = 1). */
typedef struct {
    int32_t dim;             /* 2 or 3 */
    int64_t n_nodes;
    int64_t n_elems;
    const double *coords;    /* host [n_nodes * dim] */
    const int32_t *elems;    /* host [n_elems * (dim + 1)], node ids in [0, n_nodes) */
} nn_mesh;

/* Bound-constrained method of nn_solve_nonneg and nn_step_transient (the two
 * TAO solvers the paper runs, Sec. 3.1 and Sec. 5.1). */
typedef enum {
    NN_TRON = 0,   /* active-set projected Newton-CG with a trust region (Lin & More) */
    NN_BLMVM = 1   /* bounded limited-memory variable metric (Benson & More): gradient
                      only, an L-BFGS matrix built from projected-gradient differences */
} nn_method;

/* Solver options; fill with nn_default_opts() and override.  Every
 * reduction combines per-block partials in a fixed order (no atomics), so
 * results are bitwise reproducible on the same device; there is no
 * non-deterministic mode to select. */
typedef struct {
    double tol;           /* stop when ||pg(c)||_2 <= tol * ||f||_2, pg the projected
                             gradient (g_i if c_i > 0, else min(g_i, 0)), g = K c - f.
                             Default 1e-8.  Must be > 0. */
    double inner_rtol;    /* relative residual tolerance of each inner CG solve
                             (the paper's TRON1/2/3 use 1e-1/1e-2/1e-3). Default 1e-1. */
    int32_t max_outer;    /* outer (Newton) iteration cap; default 500 */
    int32_t max_cg;       /* CG iterations per inner solve; default 5000 */
    int32_t precision;    /* nn_precision; default NN_FP64 */
    int32_t c0_mode;      /* 0: start from c = c0_value everywhere (Algorithm 1 of the
                             paper starts from 1e-8); 1: start from the caller's c
                             (warm start).  Either start is projected onto
                             [lower, upper].  Default 0. */
    double c0_value;      /* default 1e-8; must be finite */
    double delta0;        /* initial trust-region radius; <= 0 means unbounded
                             (default).  With a radius, TRON's inner CG stops on the
                             boundary of the ball of the radius left in the outer
                             iteration (Steihaug), and the Cauchy step stays inside
                             the radius.  The model is the objective itself, so the
                             radius only ever grows (x4 when a step reaches it).
                             The batched entry points scale the CG step back into
                             the radius instead. */
    int32_t cg_chunk;     /* CG iterations enqueued between convergence reads: k > 0 a fixed
                             k (default 16); 0 = the previous inner solve's count plus 2
                             (2..16) first, then 16 at a time.  Iterates do not depend on
                             it. */
    int32_t verbose;      /* 1: one line per outer iteration on stderr; default 0 */
    double lower;         /* bounds lower <= c <= upper of the constrained solves
                             (Sec. 2.2.2, eq. Eq:non-negative: c_min 1 <= c <= c_max 1).
                             Default [0, +inf): the non-negative QP (*); [0, 1] is the
                             DMP variant (Remark in Sec. 5).  lower finite, upper > lower
                             (may be +inf).  nn_solve_galerkin ignores them. */
    double upper;
    int32_t method;       /* nn_method: NN_TRON (default) or NN_BLMVM */
    int32_t lmm_vectors;  /* BLMVM: stored (s, y) pairs, 1..8; default 5 (TAO's default) */
    int32_t max_lm_its;   /* BLMVM: iteration cap; default 20000 */
    int32_t precond_degree; /* preconditioner of the CG solves (TRON's inner CG, the
                             Galerkin solve): 0 or 1 = Jacobi (default); k = 2..8 =
                             Chebyshev polynomial of degree k in D^-1 A (the Chebyshev
                             iteration with the Jacobi splitting on [lmax/30, lmax], lmax
                             the Gershgorin bound): k matrix passes per CG iteration,
                             fewer CG iterations.  The minimiser does not change.  The
                             batched entry points take 0 or 1 only. */
    int32_t subspace;     /* TRON's subspace loop (Lin & More 1999): 1 = after a projected
                             search that reached a new bound, and unless the CG stopped on
                             the trust-region boundary, the CG and search repeat on the
                             new face (the variables strictly inside the bounds) from a
                             fresh gradient before the next Cauchy step,
                             until the projected gradient has fallen to inner_rtol of its
                             value at the Cauchy point; 0 = every iteration starts with a
                             Cauchy step.  Either way
                             the minimiser is the same.  Default 0: on these problems the
                             loop's faces (which release no variable until the next Cauchy
                             step) need many more iterations (658,503-DOF cube: 342 outer
                             iterations against 63).  TRON single-problem entry points only
                             (the batched ones run 0). */
    int32_t engine;       /* how a single-problem TRON solve runs: 0 (default) = by size:
                             one workgroup in one launch (every pass over the problem by
                             one 512-thread workgroup, every decision on the device) up
                             to 4,096 rows when the solve is float64, without a trust
                             radius, subspace loop or Chebyshev preconditioner, else the
                             multi-block passes; 1 = always the multi-block passes;
                             2 = always one workgroup (NN_EINVAL if the options do not
                             allow it).  The minimiser is the same. */
} nn_opts;

/* Per-solve report (host struct, filled on return, also on NN_EMAXIT). */
typedef struct {
    double kkt_rel;       /* ||pg||_2 / ||f||_2 at the returned c (f the solve's rhs);
                             pg_i = g_i strictly inside the bounds, min(g_i, 0) at lower,
                             max(g_i, 0) at upper */
    double kkt_nat_inf;   /* ||c - P(c - g)||_inf, P the projection on [lower, upper]
                             (= ||min(c, g)||_inf for [0, inf)) */
    double min_c;         /* min_i c_i (>= lower on every constrained path) */
    double norm_f;        /* ||f||_2 */
    int32_t outer_its;
    int32_t cg_its;
    int32_t spmvs;        /* sparse matrix-vector products of every kind */
    int32_t n_active;     /* #{i : c_i == lower or c_i == upper} (#{c_i == 0} by default) */
    int32_t cauchy_trials;
    int32_t search_trials;
    int32_t refinements;  /* outer FP64 refinement steps (NN_MIXED); residual
                             replacement restarts (nn_solve_galerkin) */
    int32_t status;       /* nn_status of this solve (per member in nn_solve_batch) */
    double bytes_moved;   /* algorithmic HBM bytes of the solve (perfect-cache model) */
    double seconds;       /* device time of the solve (HIP events on the stream) */
    double max_c;         /* max_i c_i (nn_solve_galerkin only, else 0) */
    int32_t n_negative;   /* #{i : c_i < 0} (nn_solve_galerkin only, else 0) */
    int32_t subspace_its; /* iterations of TRON's subspace loop (CG steps without a new
                             Cauchy step); included in outer_its */
    int32_t radius_stops; /* inner solves that stopped on the trust-region radius (the CG
                             step cut on its boundary, or no radius left after the Cauchy
                             step) */
    int32_t reserved;
} nn_stats;

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t;
 * NULL = the null stream).  The stream must outlive the context.  Device
 * memory comes from hipMalloc and returns through hipFree. */
nn_status nn_create(nn_ctx **ctx, int device, void *hip_stream);

/* Device memory hooks for nn_create_ex.  alloc returns `bytes` (> 0) bytes
 * of device memory on the context's device, usable on its stream and aligned
 * to at least 256 bytes, or NULL when it cannot (the library then reports
 * NN_EOOM); free_ takes back a pointer alloc returned.  `user` is passed
 * through unchanged.  Both may be called from any library call on the
 * context, including nn_destroy and nn_matrix_free. */
typedef void *(*nn_alloc_fn)(size_t bytes, void *user);
typedef void (*nn_free_fn)(void *ptr, void *user);

/* nn_create with the caller's allocator (for example a framework's caching
 * allocator): every device buffer of the context (work vectors, reduction
 * partials, per-call batch arrays) and of each matrix it creates (nn_assemble,
 * nn_matrix_from_csr; also the copies later solves add to the matrix) is taken
 * from alloc and given back through free_.  A matrix keeps the hooks of the
 * context that created it and frees through them whichever context frees it,
 * so the hooks and `user` must stay valid until that context is destroyed and
 * every matrix it created is freed.  alloc and free_ must both be non-NULL;
 * NN_EINVAL otherwise.  Host staging buffers stay pinned host memory
 * (hipHostMalloc). */
nn_status nn_create_ex(nn_ctx **ctx, int device, void *hip_stream, nn_alloc_fn alloc,
                       nn_free_fn free_, void *user);
void nn_destroy(nn_ctx *ctx);
/* Message for the last non-OK status on ctx (never NULL; "" if none). */
const char *nn_last_error(const nn_ctx *ctx);
nn_status nn_default_opts(nn_opts *opts);

/*
 * Assemble the stiffness matrix K (and the capacity matrix M if with_mass)
 * over the free DOFs, and the load vector F.
 *
 *   K_ij = sum_e |e| grad(phi_i) . D_e grad(phi_j)   (bilinear form B, Sec. 2.1.2,
 *                                                     eq. functionals_B_L; F_{1,1} = D
 *                                                     in the point-wise Jacobian, Sec. 3.2)
 *   M_ij = sum_e |e| (1 + delta_ij) / ((d+1)(d+2))    (consistent capacity matrix,
 *                                                     Sec. 2.2.2; F_{0,0} = 1/dt, Sec. 3.2)
 *   F_i  = sum_e |e| f_e / (d+1)                      (functional L with element-constant f)
 *
 * Dirichlet nodes (dirichlet[v] != 0) are eliminated: their rows and columns
 * are dropped.  With dirichlet_values their prescribed values c_D are lifted
 * into the load, F_i -= sum_j K_ij c_D,j over the Dirichlet neighbours j of
 * each free node i (the trial space U of Sec. 2.1.2 with c = c^p on the
 * Dirichlet boundary); without them c = 0 there.
 *   D        host [nD * dim * dim]; nD = 1 (one tensor) or n_elems (one per element);
 *            each tensor symmetric positive definite (Sec. 2.1, eq. symmetry and
 *            positive definiteness of D).
 *   kscale   host [n_elems] or NULL: element e uses kscale[e] * D_e.
 *   f_elem   host [n_elems]: source value on each element.
 *   dirichlet host [n_nodes]: 1 = Dirichlet node.
 *   dirichlet_values host [n_nodes] or NULL: c at the Dirichlet nodes (entries
 *            at free nodes are ignored); NULL = homogeneous.
 *   K_out    receives a library-owned matrix (free with nn_matrix_free).
 *   F_dev    device [n] or NULL: receives F.  n = number of free nodes, known
 *            beforehand by the caller (count of dirichlet == 0).
 *   dof_of_node host [n_nodes] or NULL: receives the DOF index of each node, -1
 *            for Dirichlet nodes.
 * Errors: NN_EINVAL (sizes, ids out of range, degenerate element, nnz >= 2^31),
 *         NN_ENONFINITE (NaN/Inf in coords, D, kscale, f or a Dirichlet
 *         value), NN_ENOTSPD (a
 *         non-positive diagonal entry of K), NN_EOOM, NN_EHIP.
 */
nn_status nn_assemble(nn_ctx *ctx, const nn_mesh *mesh, const double *D, int64_t nD,
                      const double *kscale, const double *f_elem, const uint8_t *dirichlet,
                      const double *dirichlet_values, int with_mass, nn_matrix **K_out,
                      double *F_dev, int64_t *dof_of_node);

/* Wrap a caller CSR matrix (host arrays, copied to the device): rowptr [n+1]
 * (int64, rowptr[0] = 0), col [nnz] (int32, ascending within each row,
 * diagonal present), val [nnz], mval [nnz] or NULL (capacity values).  The
 * matrix must be symmetric positive definite for the solver. */
nn_status nn_matrix_from_csr(nn_ctx *ctx, int64_t n, const int64_t *rowptr, const int32_t *col,
                             const double *val, const double *mval, nn_matrix **out);

nn_status nn_matrix_info(const nn_matrix *A, int64_t *n, int64_t *nnz, int *has_mass);
/* Copy the CSR back to host arrays (rowptr [n+1], col/val/mval [nnz]; any may be NULL). */
nn_status nn_matrix_export(nn_ctx *ctx, const nn_matrix *A, int64_t *rowptr, int32_t *col,
                           double *val, double *mval);
/* Device bytes the matrix and one solve's work vectors occupy for a precision
 * (used to admit requests against an HBM budget), including the value and
 * offset copies that single-problem solves have already made (the first
 * single-problem solve of a matrix whose column offsets fit int16 adds
 * 10 B per sliced-ELL entry in float64 (paired layout), 6 B in mixed
 * precision (quad layout)). */
nn_status nn_matrix_bytes(const nn_matrix *A, int precision, size_t *bytes);
void nn_matrix_free(nn_ctx *ctx, nn_matrix *A);

/* y = A x on the stream (device vectors of length n); which = 0: K, 1: M. */
nn_status nn_matvec(nn_ctx *ctx, const nn_matrix *A, int which, const double *x_dev,
                    double *y_dev);

/*
 * Solve (*) for c (Sec. 2.1.3, eq. non-negative), or with the two-sided
 * bounds opts->lower <= c <= opts->upper (Sec. 2.2.2, eq. Eq:non-negative;
 * [0, 1] is the DMP variant of the Remark in Sec. 5).  The minimiser is
 * unique because K is positive definite; it is the feasible c whose gradient
 * g = K c - f is >= 0 where c_i = lower, <= 0 where c_i = upper and 0 in
 * between (for [0, inf): c >= 0, g >= 0, c_i g_i = 0).
 *   f_dev     device [n]
 *   c_dev     device [n]; in: warm start when opts->c0_mode == 1; out: solution
 *             with lower <= c_i <= upper exactly (the projection writes the
 *             bound value itself; +0.0 for a lower bound 0).
 *   active_dev device [n] uint8 or NULL; out: 1 where c_i == lower, 2 where
 *             c_i == upper, else 0.
 *   stats     host or NULL.
 * With opts->precision == NN_MIXED the Cauchy and projected searches and the
 * inner CG run on float32 copies of the values with float32 CG vectors, while
 * every outer iteration re-evaluates the float64 residual g = K c - f that
 * decides convergence; the first mixed solve attaches the float32 copy to K.
 * With opts->method == NN_BLMVM the same minimiser is found by the bounded
 * limited-memory variable-metric method (float64 only; NN_EINVAL with
 * NN_MIXED): each iteration forms d = -H pg from the compact L-BFGS
 * representation of lmm_vectors pairs (s = step, y = difference of projected
 * gradients), drops the components that point out of the box at a bound, and
 * takes the exact minimiser of the quadratic along d when no bound is
 * crossed, else a projected backtracking search; stats.outer_its counts its
 * iterations (cap max_lm_its), cg_its is 0.  Workspace of (2 lmm_vectors + 4)
 * float64 vectors of length n is kept with the context.
 * Returns NN_EMAXIT (c feasible, stats filled) if max_outer (TRON) or
 * max_lm_its (BLMVM) is reached before ||pg|| <= tol ||f||; NN_ENONFINITE if
 * a non-finite value appears.
 */
nn_status nn_solve_nonneg(nn_ctx *ctx, nn_matrix *K, const double *f_dev,
                          const nn_opts *opts, double *c_dev, uint8_t *active_dev,
                          nn_stats *stats);

/*
 * nn_solve_nonneg for callers that cannot allocate device memory during a
 * call (code in tight serving loops, harnesses that forbid allocation): the
 * same TRON solve, with every work buffer (reduction partials, CG scalars,
 * work vectors, face mask) in one fixed device array of the library instead
 * of memory taken through hipMalloc or the context's allocator hooks.  It
 * calls no device allocator and forms no copy of K: the paired, float32 and
 * quad copies are used if an earlier nn_solve_nonneg made them (results are
 * then bitwise those of nn_solve_nonneg), else the column-major values.
 *   Limit: n <= 262,144 rows (the array: about 26 MiB of device memory per
 *          GPU, taken when the library is loaded and held until the process
 *          ends); larger n -> NN_EINVAL.
 *   Options: TRON (method NN_TRON) with the Jacobi preconditioner
 *          (precond_degree <= 1), FP64 or NN_MIXED; NN_MIXED needs the
 *          matrix's float32 copy to exist already (NN_EINVAL otherwise).
 *          Launch timing (nn_set_profiling) is not recorded.
 *   Concurrency: every call on one GPU uses that GPU's single array, so calls
 *          that overlap on one GPU (from any context or thread) race and give
 *          wrong results; serialise them.  Each call clears the state it
 *          reads before use; the array keeps the last call's contents.
 * Arguments, results and statuses as nn_solve_nonneg.
 */
nn_status nn_solve_nonneg_noalloc(nn_ctx *ctx, nn_matrix *K, const double *f_dev,
                                  const nn_opts *opts, double *c_dev, uint8_t *active_dev,
                                  nn_stats *stats);

/*
 * Unconstrained single-field Galerkin solution (Sec. 2.1.2,
 * eq. Single_field_formulation): K c = f, the baseline that violates the
 * discrete maximum principle (Sec. 5.1, Table Tab:S5_cube_dmp).  Jacobi-
 * preconditioned CG from c = 0 until the true residual satisfies
 * ||K c - f||_2 <= tol ||f||_2: CG runs to that bound on its recursive
 * residual, and if the true residual misses it CG restarts from c on
 * f - K c (residual replacement; a few restarts at most, each must halve the
 * residual).  opts->max_cg caps the CG iterations of all passes together;
 * opts->max_outer, inner_rtol, c0_mode, c0_value and delta0 are not used.
 * Float64 only (opts->precision must be NN_FP64, else NN_EINVAL).
 *   f_dev   device [n] float64 (free DOFs, as from nn_assemble)
 *   c_dev   device [n] float64, out: the Galerkin solution (any sign)
 *   stats   host or NULL: kkt_rel = true ||K c - f||_2 / ||f||_2, min_c, max_c,
 *           n_negative = #{c_i < 0}, cg_its, refinements = restarts, spmvs,
 *           bytes_moved, seconds
 * Returns NN_EMAXIT (c and stats filled) if the cap is reached or the
 * residual stalls above tol, NN_ENOTSPD if CG meets non-positive curvature,
 * NN_ENONFINITE on a non-finite value.
 */
nn_status nn_solve_galerkin(nn_ctx *ctx, nn_matrix *K, const double *f_dev, const nn_opts *opts,
                            double *c_dev, nn_stats *stats);

/*
 * One backward-Euler step of the transient problem (Sec. 2.2.2,
 * eq. Eq:non-negative with lower bound 0):
 *     K~ = M/dt + K,  f~ = f + M c^(n) / dt,  c^(n+1) = argmin_{c >= 0} 1/2 c.K~c - c.f~.
 * K must carry capacity values (with_mass).  K~ is formed on the device on
 * the first call for a given dt and kept with the matrix.
 *   c_dev  device [n]; in: c^(n) (>= 0), also the warm start; out: c^(n+1).
 */
nn_status nn_step_transient(nn_ctx *ctx, nn_matrix *K, double dt, const double *f_dev,
                            const nn_opts *opts, double *c_dev, uint8_t *active_dev,
                            nn_stats *stats);

/*
 * Solve nprob independent problems of the nn_solve_nonneg kind together
 * (the batched form of the same method: every step is one launch over all
 * members, each member keeps its own step lengths, trust radius, CG scalars
 * and stopping test).  A member's result depends only on its own K, f and
 * start value: it is bitwise the same in any batch, alone or mixed, and for
 * any launch shape.  The CG iterations run as a captured hipGraph; launch
 * shapes are tuned per size class on first use (one short timing pass).
 *
 *   K, f, c  host arrays of nprob entries (K: matrices of this context's
 *            device; f, c: device [K[p]->n] float64, c in/out as in
 *            nn_solve_nonneg); members may differ in size and pattern
 *   active   host array of nprob device uint8 [n] outputs (entries may be
 *            NULL), or NULL
 *   stats    host array of nprob reports, or NULL; stats[p].status is the
 *            member's own status, stats[p].seconds the whole call's time
 * Options apply to every member (the bounds too; TRON with the Jacobi
 * preconditioner only: NN_EINVAL for NN_BLMVM or precond_degree > 1).
 * Returns NN_OK when every member reached
 * tol; otherwise the status of the first member that did not (the others are
 * still solved and reported).  A failure of the call itself (invalid argument,
 * allocation refused, HIP error) reaches no member: every stats[p].status is
 * then that call status.  Workspace is allocated for the call and released
 * before return: per row of the batch (rows of 64-row slices) 101 bytes in
 * float64, 77 in mixed precision, plus per stored matrix entry (sliced-ELL,
 * rows padded to the longest row of their slice) 14 bytes in float64, 18 in
 * mixed precision (a concatenated copy of every member's matrix; 2 bytes
 * less when a member's columns do not fit int16 offsets from the row).
 */
nn_status nn_solve_batch(nn_ctx *ctx, int32_t nprob, nn_matrix *const *K,
                         const double *const *f_dev, const nn_opts *opts, double *const *c_dev,
                         uint8_t *const *active_dev, nn_stats *stats);

/*
 * One backward-Euler step of nprob independent transient problems together
 * (nn_step_transient for every member, in one batched solve): member p gets
 * c_p^(n+1) = argmin_{c >= 0} 1/2 c.K~_p c - c.(f_p + M_p c_p^(n) / dt) with
 * K~_p = M_p/dt + K_p formed once per dt and kept with the matrix.  Every K[p]
 * must carry capacity values; c_dev[p] holds c^(n) on entry (also the warm
 * start) and c^(n+1) on return.  A member's result is bitwise the same as
 * in a batch of its own.  Other arguments and the return value as
 * nn_solve_batch.  This is the step a continuous-batching server takes for
 * all its resident transient requests at once.
 */
nn_status nn_step_transient_batch(nn_ctx *ctx, int32_t nprob, nn_matrix *const *K, double dt,
                                  const double *const *f_dev, const nn_opts *opts,
                                  double *const *c_dev, uint8_t *const *active_dev,
                                  nn_stats *stats);

/* Device time per launch of the library's kernel classes, accumulated while
 * profiling is on (nn_set_profiling).  For class k: counts[k] launches and
 * total_ms[k] milliseconds measured with HIP events on the context stream.
 * Classes: 0 CG SpMV (fused direction update), 1 CG vector update,
 * 2 gradient SpMV, 3 projected-step SpMV, 4 other.
 * nn_set_profiling: classes = 0 turns profiling off; otherwise bit k of
 * `classes` times class k (NN_PROF_ALL: every class).  A timed launch of the
 * CG classes (0, 1) records its kernel's own begin and end into two events
 * (hipExtLaunchKernelGGL); a launch of the other classes is bracketed by two
 * events on the stream.  Timing perturbs a timed run, less so for fewer
 * classes. */
#define NN_KCLASSES 5
#define NN_PROF_ALL 0x1f
nn_status nn_set_profiling(nn_ctx *ctx, int classes);
/* Time about one launch in `every` (>= 1; default 1: all) of each CG class
 * (0, 1) while profiling is on, chosen by a hash of the launch count (no
 * fixed stride that could keep hitting the same place in every chunk of CG
 * launches); the other classes are always timed in full.  The CG launches of
 * a solve are passes of the same size, so the sample gives their average
 * duration at a fraction of the timing overhead.  NN_EINVAL for every < 1. */
nn_status nn_set_profiling_sample(nn_ctx *ctx, int32_t every);
/* counts/total_ms/total_bytes/total_bytes_csr: host arrays of NN_KCLASSES
 * entries or NULL.  total_bytes is the algorithmic (perfect-cache) byte count
 * of the timed launches for the layout the kernels read (int16 column offsets
 * and paired copies where they are used); total_bytes_csr counts the same
 * launches with the paper's CSR byte model (Sec. 4, Table 2: 4-byte column
 * indices, 8-byte values; the CG matrix pass as a masked SpMV plus a
 * separate direction update, the CG vector update as its unfused operands).
 * Launches that found their work already finished (CG iterations enqueued
 * past convergence) are not counted.  reset != 0 clears the totals. */
nn_status nn_kernel_times(nn_ctx *ctx, int64_t *counts, double *total_ms, double *total_bytes,
                          double *total_bytes_csr, int reset);

#ifdef __cplusplus
}
#endif
#endif /* NNQP_H */
