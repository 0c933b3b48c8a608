/*
 * Memory and undefined-behaviour check of the oracle (test infrastructure,
 * like oracle.c itself): a standalone program that runs every entry point of
 * oracle.c on small meshes, to be built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py builds and runs
 * it).  It checks the oracle's own certificates, not GPU results.
 *
 * Meshes: a 2D square split along each cell's v00-v11 diagonal and a 3D cube
 * of six Kuhn tets per cell (the simplices of the workloads), anisotropic D,
 * f = 1 on a central block of cells, homogeneous Dirichlet on the boundary
 * (and a non-homogeneous lift in one case).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n, nnz;
    int64_t *rowptr;
    int32_t *col;
    double *K, *M, *F;
    int64_t *dof;
    int64_t n_nodes;
} or_problem;
typedef struct {
    double r;
    int64_t outer, gp_steps, cg_its, face_its, polishes, certified;
    double floor;
} or_stats;

or_problem *or_assemble(int dim, int64_t nn, int64_t ne, const double *coords,
                        const int32_t *elems, const double *D, int64_t nD,
                        const double *kscale, const double *f_elem,
                        const uint8_t *dirichlet, const double *dvals, int with_mass,
                        int *status);
void or_free(or_problem *P);
int or_solve(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *F,
             double lo, double hi, double tol, int64_t max_outer, double *c, or_stats *st);
void or_kkt(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *F,
            double lo, double hi, const double *c, double *out);
int64_t or_galerkin(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                    const double *F, double rtol, double *c);
int or_transient_step(int64_t n, const int64_t *rp, const int32_t *ci, const double *Kv,
                      const double *Mv, double dt, const double *F, const double *cn,
                      double lo, double hi, double tol, int64_t max_outer, double *c,
                      or_stats *st);

static int failures = 0;

static void expect(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        failures++;
    }
}

/* structured mesh of n^dim cells on [0,1]^dim: 2 triangles or 6 Kuhn tets per cell */
static void mesh(int dim, int n, int64_t *nn, int64_t *ne, double **X, int32_t **E, uint8_t **bnd)
{
    const int m = n + 1;
    *nn = dim == 2 ? (int64_t)m * m : (int64_t)m * m * m;
    *ne = dim == 2 ? 2LL * n * n : 6LL * n * n * n;
    *X = (double *)malloc(sizeof(double) * dim * (size_t)*nn);
    *E = (int32_t *)malloc(sizeof(int32_t) * (dim + 1) * (size_t)*ne);
    *bnd = (uint8_t *)malloc((size_t)*nn);
    for (int64_t v = 0; v < *nn; v++) {
        int64_t i = v % m, j = (v / m) % m, k = dim == 3 ? v / ((int64_t)m * m) : 0;
        (*X)[dim * v] = (double)i / n;
        (*X)[dim * v + 1] = (double)j / n;
        if (dim == 3) (*X)[dim * v + 2] = (double)k / n;
        (*bnd)[v] = i == 0 || i == n || j == 0 || j == n || (dim == 3 && (k == 0 || k == n));
    }
    int64_t e = 0;
    if (dim == 2) {
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                int32_t v00 = i + m * j, v10 = v00 + 1, v01 = v00 + m, v11 = v01 + 1;
                int32_t t[6] = {v00, v10, v11, v00, v11, v01};
                memcpy(*E + 3 * e, t, sizeof(t));
                e += 2;
            }
    } else {
        static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                       {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        const int64_t stride[3] = {1, m, (int64_t)m * m};
        for (int k = 0; k < n; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    const int32_t v0 = (int32_t)(i + (int64_t)m * j + (int64_t)m * m * k);
                    for (int p = 0; p < 6; p++) {
                        int32_t v = v0;
                        (*E)[4 * e] = v;
                        for (int s = 0; s < 3; s++) {
                            v += (int32_t)stride[perm[p][s]];
                            (*E)[4 * e + 1 + s] = v;
                        }
                        e++;
                    }
                }
    }
}

static void run_case(int dim, int n, int lift, double hi)
{
    int64_t nn, ne;
    double *X;
    int32_t *E;
    uint8_t *bnd;
    mesh(dim, n, &nn, &ne, &X, &E, &bnd);
    double D[9];
    if (dim == 2) {
        const double c = cos(M_PI / 6), s = sin(M_PI / 6), a = 1.0, b = 1e-3;
        D[0] = a * c * c + b * s * s;
        D[1] = D[2] = (a - b) * c * s;
        D[3] = a * s * s + b * c * c;
    } else {
        memset(D, 0, sizeof(D));
        D[0] = 1.0;
        D[4] = 1e-2;
        D[8] = 1e-4;
        D[1] = D[3] = 2e-3;   /* a small coupling keeps D SPD and anisotropic */
    }
    double *f = (double *)malloc(sizeof(double) * (size_t)ne);
    double *ks = (double *)malloc(sizeof(double) * (size_t)ne);
    for (int64_t e = 0; e < ne; e++) {
        f[e] = (e % 7 == 3) ? 1.0 : 0.0;
        ks[e] = 1.0 + 0.5 * (double)(e % 5);
    }
    double *dv = NULL;
    if (lift) {
        dv = (double *)malloc(sizeof(double) * (size_t)nn);
        for (int64_t v = 0; v < nn; v++) dv[v] = X[dim * v] > 0.5 ? 0.25 : 0.0;
    }
    int st = -1;
    or_problem *P = or_assemble(dim, nn, ne, X, E, D, 1, ks, f, bnd, dv, 1, &st);
    expect(P != NULL && st == 0, "assembly");
    if (P) {
        const int64_t N = P->n;
        double *c = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
        double *c2 = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
        or_stats S;
        int rc = or_solve(N, P->rowptr, P->col, P->K, P->F, 0.0, hi, 1e-12, 20000, c, &S);
        expect(rc == 0 && S.certified, "bound-constrained solve certified");
        double kkt[16] = {0};   /* or_kkt writes 11 values */
        or_kkt(N, P->rowptr, P->col, P->K, P->F, 0.0, hi, c, kkt);
        expect(kkt[0] <= 1e-10, "KKT residual of the returned point");
        or_galerkin(N, P->rowptr, P->col, P->K, P->F, 1e-12, c2);
        rc = or_transient_step(N, P->rowptr, P->col, P->K, P->M, 1e-3, P->F, c, 0.0, hi, 1e-12,
                               20000, c2, &S);
        expect(rc == 0 && S.certified, "backward-Euler step certified");
        free(c);
        free(c2);
        or_free(P);
    }
    free(X);
    free(E);
    free(bnd);
    free(f);
    free(ks);
    free(dv);
}

int main(void)
{
    run_case(2, 24, 0, INFINITY);
    run_case(2, 17, 1, 0.02);   /* lifted Dirichlet data, both bounds */
    run_case(3, 7, 0, INFINITY);
    run_case(3, 8, 1, INFINITY);
    if (failures) return 1;
    printf("sanitized oracle ok\n");
    return 0;
}
