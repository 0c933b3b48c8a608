/*
 * Plain FP64 CPU oracle for the non-negative diffusion QP.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke entry point and the CPU-baseline
 * leg of the benchmark call this code; the product library never does, and it
 * shares no code with the HIP path.
 *
 * What it computes (arXiv:1506.08435):
 *   - P1 Galerkin stiffness K, capacity (mass) matrix M and load F on a
 *     simplicial mesh (Sec. 2.1.2, bilinear form B and functional L of
 *     eq. functionals_B_L; Sec. 2.1.3 discrete system eq. Helmholtz_discrete;
 *     Sec. 2.2.2 capacity matrix), homogeneous Dirichlet nodes eliminated.
 *   - Dirichlet nodes with given values c_D are eliminated by lifting:
 *     F_F -= K_FD c_D (the Dirichlet part of the space U, Sec. 2.1.2).
 *   - The unique minimiser of 1/2 c.Kc - c.F subject to lo <= c <= hi
 *     (Sec. 2.1.3, eq. non-negative with lo = 0, hi = +inf; Sec. 2.2.2,
 *     eq. Eq:non-negative with c_min <= c <= c_max; the DMP variant of the
 *     Remark in Sec. 5 takes [0, 1]), i.e. the feasible c whose gradient
 *     g = Kc - F satisfies g_i >= 0 where c_i = lo, g_i <= 0 where c_i = hi and
 *     g_i = 0 in between.
 *   - One backward-Euler step of the transient QP (Sec. 2.2.2,
 *     eq. Eq:non-negative with K~ = M/dt + K, f~ = f + M c^(n)/dt).
 *
 * How the minimiser is found: any correct method may be used because the
 * result is unique; this file uses gradient-projection conjugate gradients
 * (More & Toraldo, SIAM J. Optim. 1(1), 1991, the GPCG method the paper names
 * in Sec. 3.1) to identify the active set, then solves K_FF c_F = F_F on that
 * face to the FP64 floor and checks the KKT conditions (the definition of the
 * result) before returning.
 *
 * Style: plain loops, no blocking or fusion; OpenMP only splits independent
 * row loops and sums.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2
#define OR_EDEGEN 3
#define OR_ENOCONV 4

/* Progress lines on stderr for long runs: at most one every g_progress
 * seconds (0: none).  They report, they change nothing. */
static double g_progress = 0.0;
static double g_last_report = 0.0;

static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void report(const char *phase, int64_t k, double r)
{
    if (!(g_progress > 0.0)) return;
    const double now = wall_seconds();
    if (now - g_last_report < g_progress) return;
    g_last_report = now;
    fprintf(stderr, "oracle: %s %lld r %.3e\n", phase, (long long)k, r);
    fflush(stderr);
}

void or_set_progress(double seconds)
{
    g_progress = seconds;
    g_last_report = wall_seconds();
}

/* ------------------------------------------------------------------ */
/* P1 element quantities (Sec. 2.1.3: P^k spaces with k = 1)           */
/* ------------------------------------------------------------------ */

/* Gradients of the dim+1 barycentric basis functions and the volume of a
 * simplex with vertex coordinates X[a*dim + k].
 * With B = [x_1 - x_0, ..., x_d - x_0], grad phi_k (k >= 1) is row k-1 of
 * B^{-1} and grad phi_0 = -sum_k grad phi_k; |e| = |det B| / d!. */
static int p1_geometry(int dim, const double *X, double grad[4][3], double *vol)
{
    double B[3][3], inv[3][3], det;
    for (int r = 0; r < dim; r++)
        for (int k = 0; k < dim; k++)
            B[r][k] = X[(k + 1) * dim + r] - X[r]; /* column k = x_{k+1} - x_0 */
    if (dim == 2) {
        det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
        if (det == 0.0) return OR_EDEGEN;
        inv[0][0] = B[1][1] / det;
        inv[0][1] = -B[0][1] / det;
        inv[1][0] = -B[1][0] / det;
        inv[1][1] = B[0][0] / det;
        *vol = fabs(det) / 2.0;
    } else {
        double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
        double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
        double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
        det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
        if (det == 0.0) return OR_EDEGEN;
        /* inverse = adjugate / det; adj[i][j] = cofactor[j][i] */
        inv[0][0] = c00 / det;
        inv[1][0] = c01 / det;
        inv[2][0] = c02 / det;
        inv[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) / det;
        inv[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) / det;
        inv[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) / det;
        inv[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) / det;
        inv[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) / det;
        inv[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) / det;
        *vol = fabs(det) / 6.0;
    }
    for (int k = 0; k < dim; k++) grad[0][k] = 0.0;
    for (int a = 1; a <= dim; a++)
        for (int k = 0; k < dim; k++) {
            grad[a][k] = inv[a - 1][k];
            grad[0][k] -= inv[a - 1][k];
        }
    return OR_OK;
}

/* Element stiffness K^e_ab = |e| grad phi_a . D grad phi_b (exact for an
 * element-constant D); upper triangle computed, lower mirrored. */
static void p1_stiffness(int dim, double grad[4][3], double vol, const double *D,
                         double Ke[4][4])
{
    int nv = dim + 1;
    for (int b = 0; b < nv; b++) {
        double Dg[3];
        for (int r = 0; r < dim; r++) {
            Dg[r] = 0.0;
            for (int k = 0; k < dim; k++) Dg[r] += D[r * dim + k] * grad[b][k];
        }
        for (int a = 0; a <= b; a++) {
            double s = 0.0;
            for (int r = 0; r < dim; r++) s += grad[a][r] * Dg[r];
            Ke[a][b] = vol * s;
            Ke[b][a] = Ke[a][b];
        }
    }
}

/* Consistent P1 mass: M^e_ab = |e| (1 + delta_ab) / ((d+1)(d+2)). */
static double p1_mass(int dim, double vol, int a, int b)
{
    double den = (double)((dim + 1) * (dim + 2));
    return vol * (a == b ? 2.0 : 1.0) / den;
}

/* ------------------------------------------------------------------ */
/* Assembly (Sec. 3.2: the assembly operator over elements)            */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;       /* free DOFs */
    int64_t nnz;
    int64_t *rowptr; /* n+1 */
    int32_t *col;    /* nnz, ascending within a row */
    double *K;       /* nnz */
    double *M;       /* nnz or NULL */
    double *F;       /* n */
    int64_t *dof;    /* n_nodes: free DOF index or -1 */
    int64_t n_nodes;
} or_problem;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int64_t find_slot(const or_problem *P, int64_t row, int32_t c)
{
    int64_t lo = P->rowptr[row], hi = P->rowptr[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (P->col[mid] == c) return mid;
        if (P->col[mid] < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

void or_free(or_problem *P)
{
    if (!P) return;
    free(P->rowptr);
    free(P->col);
    free(P->K);
    free(P->M);
    free(P->F);
    free(P->dof);
    free(P);
}

/*
 * Assemble K (and M if with_mass) over the free DOFs.
 *   coords  [nn*dim], elems [ne*(dim+1)]
 *   D       [nD*dim*dim], nD = 1 (shared) or ne (per element)
 *   kscale  [ne] or NULL: D_e = kscale[e] * D
 *   f_elem  [ne]: element-constant source; the load uses the one-point rule
 *           F^e_a = |e| f_e / (d+1), exact for element-constant f.
 *   dirichlet [nn]: 1 = Dirichlet node, eliminated.
 *   dvals   [nn] or NULL: the value of c at each Dirichlet node (NULL: 0);
 *           F_r -= K_rj c_j for every Dirichlet neighbour j of a free row r.
 */
or_problem *or_assemble(int dim, int64_t nn, int64_t ne, const double *coords,
                        const int32_t *elems, const double *D, int64_t nD,
                        const double *kscale, const double *f_elem,
                        const uint8_t *dirichlet, const double *dvals, int with_mass,
                        int *status)
{
    *status = OR_EINVAL;
    if ((dim != 2 && dim != 3) || nn < 0 || ne < 0 || (nD != 1 && nD != ne)) return NULL;
    int nv = dim + 1;
    or_problem *P = (or_problem *)calloc(1, sizeof(or_problem));
    if (!P) { *status = OR_ENOMEM; return NULL; }
    P->n_nodes = nn;
    P->dof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nn > 0 ? nn : 1));
    int64_t n = 0;
    for (int64_t i = 0; i < nn; i++) P->dof[i] = dirichlet[i] ? -1 : n++;
    P->n = n;

    /* node -> element incidence */
    int64_t *ip = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
    int64_t *ie = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ne * nv > 0 ? ne * nv : 1));
    for (int64_t e = 0; e < ne; e++)
        for (int a = 0; a < nv; a++) {
            int32_t v = elems[e * nv + a];
            if (v < 0 || v >= nn) { free(ip); free(ie); or_free(P); return NULL; }
            ip[v + 1]++;
        }
    for (int64_t i = 0; i < nn; i++) ip[i + 1] += ip[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nn > 0 ? nn : 1));
    for (int64_t i = 0; i < nn; i++) fill[i] = ip[i];
    for (int64_t e = 0; e < ne; e++)
        for (int a = 0; a < nv; a++) ie[fill[elems[e * nv + a]]++] = e;
    free(fill);

    /* sparsity: row i holds every free DOF sharing an element with node i */
    P->rowptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t **rows = (int32_t **)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t *));
    int64_t *rlen = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nn; i++) {
        int64_t r = P->dof[i];
        if (r < 0) continue;
        int64_t cap = (ip[i + 1] - ip[i]) * nv;
        int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
        int64_t m = 0;
        for (int64_t t = ip[i]; t < ip[i + 1]; t++) {
            int64_t e = ie[t];
            for (int b = 0; b < nv; b++) {
                int64_t dj = P->dof[elems[e * nv + b]];
                if (dj >= 0) buf[m++] = (int32_t)dj;
            }
        }
        qsort(buf, (size_t)m, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t t = 0; t < m; t++)
            if (u == 0 || buf[t] != buf[u - 1]) buf[u++] = buf[t];
        rows[r] = buf;
        rlen[r] = u;
    }
    for (int64_t r = 0; r < n; r++) P->rowptr[r + 1] = P->rowptr[r] + rlen[r];
    P->nnz = P->rowptr[n];
    P->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(P->nnz > 0 ? P->nnz : 1));
    for (int64_t r = 0; r < n; r++) {
        memcpy(P->col + P->rowptr[r], rows[r], sizeof(int32_t) * (size_t)rlen[r]);
        free(rows[r]);
    }
    free(rows);
    free(rlen);
    free(ip);
    free(ie);

    P->K = (double *)calloc((size_t)(P->nnz > 0 ? P->nnz : 1), sizeof(double));
    P->F = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (with_mass) P->M = (double *)calloc((size_t)(P->nnz > 0 ? P->nnz : 1), sizeof(double));

    /* element loop: compute each element matrix and add it into the global rows */
    for (int64_t e = 0; e < ne; e++) {
        double X[12], grad[4][3], vol, Ke[4][4], De[9];
        for (int a = 0; a < nv; a++)
            for (int k = 0; k < dim; k++) X[a * dim + k] = coords[(int64_t)elems[e * nv + a] * dim + k];
        if (p1_geometry(dim, X, grad, &vol) != OR_OK) { or_free(P); *status = OR_EDEGEN; return NULL; }
        const double *Dsrc = D + (nD == 1 ? 0 : e * dim * dim);
        double ks = kscale ? kscale[e] : 1.0;
        for (int t = 0; t < dim * dim; t++) De[t] = ks * Dsrc[t];
        p1_stiffness(dim, grad, vol, De, Ke);
        for (int a = 0; a < nv; a++) {
            int64_t r = P->dof[elems[e * nv + a]];
            if (r < 0) continue;
            P->F[r] += vol * f_elem[e] / (double)nv;
            for (int b = 0; b < nv; b++) {
                int64_t c = P->dof[elems[e * nv + b]];
                if (c < 0) {
                    if (dvals) P->F[r] -= Ke[a][b] * dvals[elems[e * nv + b]];
                    continue;
                }
                int64_t s = find_slot(P, r, (int32_t)c);
                P->K[s] += Ke[a][b];
                if (with_mass) P->M[s] += p1_mass(dim, vol, a, b);
            }
        }
    }
    *status = OR_OK;
    return P;
}

void or_problem_sizes(const or_problem *P, int64_t *n, int64_t *nnz)
{
    *n = P->n;
    *nnz = P->nnz;
}

void or_problem_export(const or_problem *P, int64_t *rowptr, int32_t *col, double *K,
                       double *M, double *F, int64_t *dof)
{
    memcpy(rowptr, P->rowptr, sizeof(int64_t) * (size_t)(P->n + 1));
    if (P->nnz) {
        memcpy(col, P->col, sizeof(int32_t) * (size_t)P->nnz);
        memcpy(K, P->K, sizeof(double) * (size_t)P->nnz);
        if (M && P->M) memcpy(M, P->M, sizeof(double) * (size_t)P->nnz);
    }
    if (P->n) memcpy(F, P->F, sizeof(double) * (size_t)P->n);
    memcpy(dof, P->dof, sizeof(int64_t) * (size_t)P->n_nodes);
}

/* ------------------------------------------------------------------ */
/* Vector helpers                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const int64_t *rp;
    const int32_t *ci;
    const double *v;
    const double *F;
    double lo, hi;   /* bounds lo <= c <= hi (hi may be +inf) */
} qp_t;

void or_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
             const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) s += v[k] * x[ci[k]];
        y[i] = s;
    }
}

static void spmv(const qp_t *Q, const double *x, double *y) { or_spmv(Q->n, Q->rp, Q->ci, Q->v, x, y); }

/* Sums are taken in a fixed order (fixed-size chunks, chunk totals added
 * serially), so results do not depend on the thread count or schedule. */
#define OR_CHUNK 4096

static double dot(int64_t n, const double *a, const double *b)
{
    int64_t nc = (n + OR_CHUNK - 1) / OR_CHUNK;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nc; t++) {
        double s = 0.0;
        int64_t hi = (t + 1) * OR_CHUNK < n ? (t + 1) * OR_CHUNK : n;
        for (int64_t i = t * OR_CHUNK; i < hi; i++) s += a[i] * b[i];
        part[t] = s;
    }
    double s = 0.0;
    for (int64_t t = 0; t < nc; t++) s += part[t];
    free(part);
    return s;
}

/* Projection onto [lo, hi] (NaN maps to lo; callers count non-finite values
 * separately; with lo = 0 the result is a canonical +0.0). */
static inline double proj(const qp_t *Q, double x)
{
    double y = x > Q->lo ? x : Q->lo;
    return y < Q->hi ? y : Q->hi;
}

/* Projected gradient: g_i strictly between the bounds, min(g_i, 0) at the
 * lower bound, max(g_i, 0) at the upper bound. */
static inline double pgrad(const qp_t *Q, double c, double g)
{
    if (c <= Q->lo) return g < 0.0 ? g : 0.0;
    if (c >= Q->hi) return g > 0.0 ? g : 0.0;
    return g;
}

static double pg_norm(const qp_t *Q, const double *c, const double *g)
{
    int64_t n = Q->n;
    int64_t nc = (n + OR_CHUNK - 1) / OR_CHUNK;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nc; t++) {
        double s = 0.0;
        int64_t hi = (t + 1) * OR_CHUNK < n ? (t + 1) * OR_CHUNK : n;
        for (int64_t i = t * OR_CHUNK; i < hi; i++) {
            double p = pgrad(Q, c[i], g[i]);
            s += p * p;
        }
        part[t] = s;
    }
    double s = 0.0;
    for (int64_t t = 0; t < nc; t++) s += part[t];
    free(part);
    return sqrt(s);
}

/* Rounding floor of ||Kc - F||_2 / ||F||_2: each residual entry carries an
 * error of a few units of roundoff times sum_j |K_ij c_j| + |F_i|; the
 * factor 32 covers rows of up to 32 entries. */
static double residual_floor(const qp_t *Q, const double *c, double nf)
{
    const double u = 1.1102230246251565e-16;
    double s = 0.0;
    for (int64_t i = 0; i < Q->n; i++) {
        double a = fabs(Q->F[i]);
        for (int64_t k = Q->rp[i]; k < Q->rp[i + 1]; k++) a += fabs(Q->v[k] * c[Q->ci[k]]);
        s += a * a;
    }
    return 32.0 * u * sqrt(s) / nf;
}

static void gradient(const qp_t *Q, const double *c, double *g)
{
    spmv(Q, c, g);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < Q->n; i++) g[i] -= Q->F[i];
}

/* binding: at the lower bound with g_i >= 0, or at the upper bound with
 * g_i <= 0 (a zero gradient counts as binding) */
static inline int binding(const qp_t *Q, double c, double g)
{
    return (c == Q->lo && g >= 0.0) || (c == Q->hi && g <= 0.0);
}

/*
 * KKT report for c under lo <= c <= hi (used as the certificate):
 *   out[0]  = ||pg||_2 / ||F||_2  (||pg||_2 when F = 0)
 *   out[1]  = ||c - P(c - g)||_inf  (natural residual; ||min(c, g)||_inf for [0, inf))
 *   out[2]  = min_i c_i
 *   out[3]  = max_i min(c_i - lo, hi - c_i) |g_i|  (complementarity)
 *   out[4]  = ||F||_2
 *   out[5]  = number of non-finite entries of c or g
 *   out[6]  = min_i g_i over {c_i = lo}  (+inf if none)
 *   out[7]  = number of i with c_i == lo
 *   out[8]  = max_i c_i
 *   out[9]  = max_i g_i over {c_i = hi}  (-inf if none)
 *   out[10] = number of i with c_i == hi
 */
void or_kkt(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
            const double *F, double lo, double hi, const double *c, double *out)
{
    qp_t Q = {n, rp, ci, v, F, lo, hi};
    double *g = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    gradient(&Q, c, g);
    double pg2 = 0, nat = 0, minc = INFINITY, maxc = -INFINITY, comp = 0, ff = 0, nonfin = 0;
    double ming = INFINITY, nlo = 0, maxg = -INFINITY, nhi = 0;
    for (int64_t i = 0; i < n; i++) {
        double p = pgrad(&Q, c[i], g[i]);
        pg2 += p * p;
        double m = fabs(c[i] - proj(&Q, c[i] - g[i]));
        if (m > nat) nat = m;
        if (c[i] < minc) minc = c[i];
        if (c[i] > maxc) maxc = c[i];
        double dist = fmin(c[i] - lo, hi - c[i]);
        double cg = dist * fabs(g[i]);
        if (cg > comp) comp = cg;
        ff += F[i] * F[i];
        if (!isfinite(c[i]) || !isfinite(g[i])) nonfin += 1;
        if (c[i] == lo) {
            nlo += 1;
            if (g[i] < ming) ming = g[i];
        }
        if (c[i] == hi) {
            nhi += 1;
            if (g[i] > maxg) maxg = g[i];
        }
    }
    double nf = sqrt(ff);
    out[0] = nf > 0 ? sqrt(pg2) / nf : sqrt(pg2);
    out[1] = nat;
    out[2] = n > 0 ? minc : 0.0;
    out[3] = comp;
    out[4] = nf;
    out[5] = nonfin;
    out[6] = ming;
    out[7] = nlo;
    out[8] = n > 0 ? maxc : 0.0;
    out[9] = maxg;
    out[10] = nhi;
    free(g);
}

/* ------------------------------------------------------------------ */
/* Jacobi-preconditioned CG on the free rows (mask[i] = 1)             */
/* ------------------------------------------------------------------ */

/* Solves K_FF x_F = b_F with x_A held fixed at its input value (0 on the
 * active set in every use here).  Restarts from the true residual every
 * `restart` iterations; stops at ||r|| <= atol or after stagnation.
 * Returns the iteration count. */
static int64_t pcg_face(const qp_t *Q, const uint8_t *mask, const double *b, double *x,
                        double atol, int64_t maxit, double *work)
{
    int64_t n = Q->n;
    double *r = work, *z = work + n, *p = work + 2 * n, *q = work + 3 * n, *dinv = work + 4 * n;
    for (int64_t i = 0; i < n; i++) {
        dinv[i] = 0.0;
        if (mask[i])
            for (int64_t k = Q->rp[i]; k < Q->rp[i + 1]; k++)
                if (Q->ci[k] == i) dinv[i] = 1.0 / Q->v[k];
    }
    int64_t it = 0;
    double best = INFINITY;
    int64_t since_best = 0;
    const int64_t restart = 200;
    while (it < maxit) {
        spmv(Q, x, q);
        for (int64_t i = 0; i < n; i++) r[i] = mask[i] ? b[i] - q[i] : 0.0;
        double rn = sqrt(dot(n, r, r));
        if (rn < best * 0.999) { best = rn; since_best = 0; }
        else if (++since_best >= 3) break;
        if (rn <= atol) break;
        report("face solve iteration", it, rn);
        for (int64_t i = 0; i < n; i++) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
        double rz = dot(n, r, z);
        for (int64_t j = 0; j < restart && it < maxit; j++, it++) {
            spmv(Q, p, q);
            for (int64_t i = 0; i < n; i++) if (!mask[i]) q[i] = 0.0;
            double pq = dot(n, p, q);
            if (!(pq > 0.0)) break;
            double alpha = rz / pq;
            for (int64_t i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            if (sqrt(dot(n, r, r)) <= 0.5 * atol) { it++; break; }
            for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
            double rz2 = dot(n, r, z);
            double beta = rz2 / rz;
            rz = rz2;
            for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
    }
    return it;
}

/* Unconstrained Galerkin solve K c = F by Jacobi-PCG (Sec. 2.1.3,
 * eq. Helmholtz_discrete), to ||r|| <= rtol ||F||. */
int64_t or_galerkin(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                    const double *F, double rtol, double *c)
{
    qp_t Q = {n, rp, ci, v, F, -INFINITY, INFINITY};
    uint8_t *mask = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    double *work = (double *)malloc(sizeof(double) * 5 * (size_t)(n > 0 ? n : 1));
    memset(mask, 1, (size_t)n);
    double nf = sqrt(dot(n, F, F));
    int64_t it = pcg_face(&Q, mask, F, c, rtol * nf, 100 * n + 1000, work);
    free(mask);
    free(work);
    return it;
}

/* ------------------------------------------------------------------ */
/* GPCG (More & Toraldo 1991) + face solve + KKT certificate            */
/* ------------------------------------------------------------------ */

typedef struct {
    double r;        /* final ||pg||/||F|| */
    int64_t outer;   /* GPCG major iterations */
    int64_t gp_steps;
    int64_t cg_its;
    int64_t face_its;
    int64_t polishes;
    int64_t certified;
    double floor;    /* rounding floor of r at the returned point */
} or_stats;

/* Projected search along direction d from x: y(t) = P(x + t d), t halved
 * from t0 until q(y) - q(x) <= mu g.(y - x).  On return x = y, g is updated
 * through K s, and the decrease q(x_old) - q(x_new) is returned. */
static double projected_search(const qp_t *Q, double *x, double *g, const double *d, double t0,
                               double mu, double *y, double *s, double *Ks, int *spmvs)
{
    int64_t n = Q->n;
    double t = t0, dq = 0.0;
    for (int trial = 0; trial < 80; trial++) {
        for (int64_t i = 0; i < n; i++) { y[i] = proj(Q, x[i] + t * d[i]); s[i] = y[i] - x[i]; }
        spmv(Q, s, Ks);
        (*spmvs)++;
        double gs = dot(n, g, s), sKs = dot(n, s, Ks);
        dq = gs + 0.5 * sKs;
        if (dq <= mu * gs) break;
        t *= 0.5;
    }
    if (!(dq <= 0.0)) return 0.0; /* no decrease found: keep x */
    for (int64_t i = 0; i < n; i++) { x[i] = y[i]; g[i] += Ks[i]; }
    return -dq;
}

int or_solve(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *F,
             double lo, double hi, double tol, int64_t max_outer, double *c, or_stats *st)
{
    const double mu = 0.01, eta1 = 0.1, eta2 = 0.1;
    qp_t Q = {n, rp, ci, v, F, lo, hi};
    if (!(lo < hi) || !isfinite(lo)) return OR_EINVAL;
    memset(st, 0, sizeof(*st));
    if (n == 0) { st->certified = 1; return OR_OK; }
    size_t sz = sizeof(double) * (size_t)n;
    double *g = malloc(sz), *d = malloc(sz), *y = malloc(sz), *s = malloc(sz), *Ks = malloc(sz);
    double *w = malloc(sz), *r = malloc(sz), *z = malloc(sz), *p = malloc(sz), *q = malloc(sz);
    double *dinv = malloc(sz), *work = malloc(5 * sz), *rhs = malloc(sz);
    uint8_t *b_old = malloc((size_t)n), *mask = malloc((size_t)n);
    int spmvs = 0;
    double nf = sqrt(dot(n, F, F));
    double fmax = -INFINITY;
    for (int64_t i = 0; i < n; i++) if (F[i] > fmax) fmax = F[i];
    for (int64_t i = 0; i < n; i++) {
        dinv[i] = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++)
            if (ci[k] == i && v[k] > 0.0) dinv[i] = 1.0 / v[k];
    }
    int rc = OR_ENOCONV;
    if (lo == 0.0 && !(fmax > 0.0)) {
        /* F <= 0 with lower bound 0: c = 0 gives g = -F >= 0, so c = 0 is the
         * minimiser. */
        memset(c, 0, sz);
        st->certified = 1;
        rc = OR_OK;
        goto done;
    }
    for (int64_t i = 0; i < n; i++) c[i] = proj(&Q, c[i]);
    gradient(&Q, c, g);
    double inner_tol = tol;
    double best_rel = INFINITY;
    int64_t since_best = 0;
    for (int64_t outer = 0; outer < max_outer; outer++) {
        st->outer = outer + 1;
        double rel = pg_norm(&Q, c, g) / nf;
        st->r = rel;
        report("outer iteration", outer, rel);
        /* Near the rounding floor of the residual the iteration stops
         * gaining: once r is below that floor and has not halved for thirty
         * iterations, the face solve and certificate take over (they accept
         * r at max(tol, floor)). */
        if (rel < 0.5 * best_rel) {
            best_rel = rel;
            since_best = 0;
        } else {
            since_best++;
        }
        if (rel <= inner_tol || (since_best >= 30 && rel <= residual_floor(&Q, c, nf))) {
            /* Face solve on the binding set of c, then check the KKT conditions. */
            st->polishes++;
            /* binding variables stay at their bound value */
            for (int64_t i = 0; i < n; i++) {
                mask[i] = binding(&Q, c[i], g[i]) ? 0 : 1;
                y[i] = c[i];
            }
            st->face_its += pcg_face(&Q, mask, F, y, 1e-15 * nf, 20 * n + 2000, work);
            /* how far the face solution left the box, relative to its size */
            double yabs = 0.0, outside = 0.0;
            for (int64_t i = 0; i < n; i++) {
                if (fabs(y[i]) > yabs) yabs = fabs(y[i]);
                if (lo - y[i] > outside) outside = lo - y[i];
                if (y[i] - hi > outside) outside = y[i] - hi;
            }
            for (int64_t i = 0; i < n; i++) y[i] = proj(&Q, y[i]);
            gradient(&Q, y, d);
            double rel_y = pg_norm(&Q, y, d) / nf;
            double floor_y = residual_floor(&Q, y, nf);
            st->floor = floor_y;
            if (outside <= 1e-10 * yabs && rel_y <= (tol > floor_y ? tol : floor_y)) {
                memcpy(c, y, sz);
                memcpy(g, d, sz);
                st->r = rel_y;
                st->certified = 1;
                rc = OR_OK;
                break;
            }
            /* Wrong face (a free value went negative) or not yet accurate:
             * continue from the better of the two points, tighter. */
            if (rel_y < rel) { memcpy(c, y, sz); memcpy(g, d, sz); }
            inner_tol *= 0.1;
            if (inner_tol < floor_y) inner_tol = floor_y;
            if (st->polishes > 60) break;
            continue;
        }

        /* Gradient-projection phase: projected searches along -g until the
         * binding set settles or the decrease stalls. */
        double dmax = 0.0;
        for (int j = 0; j < 50; j++) {
            for (int64_t i = 0; i < n; i++) {
                b_old[i] = (uint8_t)binding(&Q, c[i], g[i]);
                d[i] = b_old[i] ? 0.0 : -g[i];
            }
            double dd = dot(n, d, d);
            if (dd == 0.0) break;
            spmv(&Q, d, Ks);
            spmvs++;
            double dKd = dot(n, d, Ks);
            double t0 = dKd > 0.0 ? dd / dKd : 1.0;
            double dec = projected_search(&Q, c, g, d, t0, mu, y, s, Ks, &spmvs);
            st->gp_steps++;
            if (dec > dmax) dmax = dec;
            int same = 1;
            for (int64_t i = 0; i < n && same; i++)
                if ((uint8_t)binding(&Q, c[i], g[i]) != b_old[i]) same = 0;
            if (same || dec <= eta1 * dmax) break;
        }

        /* Conjugate-gradient phase on the face of c (variables at a bound held fixed). */
        for (int face = 0; face < 50; face++) {
            for (int64_t i = 0; i < n; i++) {
                mask[i] = c[i] > lo && c[i] < hi;
                r[i] = mask[i] ? -g[i] : 0.0;
                z[i] = mask[i] ? dinv[i] * r[i] : 0.0;
                p[i] = z[i];
                w[i] = 0.0;
            }
            double rz = dot(n, r, z);
            if (!(rz > 0.0)) break;
            double maxdec = 0.0;
            for (int64_t it = 0; it < n + 100; it++) {
                spmv(&Q, p, q);
                spmvs++;
                for (int64_t i = 0; i < n; i++) if (!mask[i]) q[i] = 0.0;
                double pq = dot(n, p, q);
                if (!(pq > 0.0)) break;
                double alpha = rz / pq;
                for (int64_t i = 0; i < n; i++) { w[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
                st->cg_its++;
                double dec = 0.5 * alpha * rz; /* q(w_j) - q(w_{j+1}) for CG from w = 0 */
                if (dec > maxdec) maxdec = dec;
                for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
                double rz2 = dot(n, r, z);
                if (dec <= eta2 * maxdec || rz2 <= 0.0) break;
                double beta = rz2 / rz;
                rz = rz2;
                for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
            }
            projected_search(&Q, c, g, w, 1.0, mu, y, s, Ks, &spmvs);
            if (pg_norm(&Q, c, g) / nf <= inner_tol) break;
            /* stay on the face while every variable at a bound is binding */
            int same = 1;
            for (int64_t i = 0; i < n && same; i++)
                if ((c[i] == lo || c[i] == hi) && !binding(&Q, c[i], g[i])) same = 0;
            if (!same) break;
        }
    }
done:
    free(g); free(d); free(y); free(s); free(Ks); free(w); free(r); free(z); free(p); free(q);
    free(dinv); free(work); free(rhs); free(b_old); free(mask);
    return rc;
}

/* One backward-Euler step (Sec. 2.2.2): K~ = M/dt + K, f~ = F + M c^n / dt,
 * solve the bound-constrained QP warm-started from c^n. c_out may alias nothing. */
int or_transient_step(int64_t n, const int64_t *rp, const int32_t *ci, const double *Kv,
                      const double *Mv, double dt, const double *F, const double *cn,
                      double lo, double hi, double tol, int64_t max_outer, double *c_out,
                      or_stats *st)
{
    int64_t nnz = rp[n];
    double *Kt = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *ft = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t k = 0; k < nnz; k++) Kt[k] = Mv[k] / dt + Kv[k];
    or_spmv(n, rp, ci, Mv, cn, ft);
    for (int64_t i = 0; i < n; i++) ft[i] = F[i] + ft[i] / dt;
    memcpy(c_out, cn, sizeof(double) * (size_t)n);
    int rc = or_solve(n, rp, ci, Kt, ft, lo, hi, tol, max_outer, c_out, st);
    free(Kt);
    free(ft);
    return rc;
}

/* Builds K~ values and f~ for one backward-Euler step (exported for checks). */
void or_transient_system(int64_t n, const int64_t *rp, const int32_t *ci, const double *Kv,
                         const double *Mv, double dt, const double *F, const double *cn,
                         double *Kt, double *ft)
{
    int64_t nnz = rp[n];
    for (int64_t k = 0; k < nnz; k++) Kt[k] = Mv[k] / dt + Kv[k];
    or_spmv(n, rp, ci, Mv, cn, ft);
    for (int64_t i = 0; i < n; i++) ft[i] = F[i] + ft[i] / dt;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
