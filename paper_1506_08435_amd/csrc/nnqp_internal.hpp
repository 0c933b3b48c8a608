// Internal declarations of the MI355X non-negative QP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "nnqp.h"

namespace nnqp {

// ---------------------------------------------------------------- launch geometry
// Every row-parallel kernel of a solve uses the same partition of the rows:
// `nb` blocks of 256 threads, block b owning rows [lb*chunk, (lb+1)*chunk) where
// lb = xcd_block(b).  The hardware deals workgroups round-robin to the 8 XCDs,
// so lb maps the blocks of one XCD onto one contiguous eighth of the rows: each
// XCD's L2 then sees one slab of the vectors instead of all of them, and a row
// is touched by the same XCD in every kernel of the solve.
constexpr int kBlock = 256;
constexpr int kXcds = 8;
constexpr int kMaxBlocks = 2048;   // 8 workgroups per CU on 256 CUs
constexpr int kMaxRed = 8;         // values per reduction

struct Part {
    int n = 0;       // rows
    int nb = 0;      // blocks (multiple of kXcds)
    int chunk = 0;   // rows per block (multiple of kBlock)
};

Part make_part(int64_t n, int max_blocks = kMaxBlocks);

__device__ __forceinline__ int xcd_block(int b, int nb)
{
    return (b % kXcds) * (nb / kXcds) + (b / kXcds);
}

// ---------------------------------------------------------------- device scalars
// Scalars the kernels hand to each other without a host round trip.
struct DevScalars {
    double red[kMaxRed];   // output of the last reduction kernel
    double rz;             // CG: r.z
    double rr;             // CG: r.r
    double rr_stop;        // CG: stop when r.r <= rr_stop
    double alpha, beta, pq;
    double nnz_free;       // nonzeros in the free rows (byte model)
    double n_free;
    int done;              // CG: 0 running, 1 converged/capped, 3 breakdown, 4 non-finite
    int it;                // CG iterations done
    int max_it;
    int pad;
};

// ---------------------------------------------------------------- objects
struct Workspace {
    int64_t cap = 0;
    double *g = nullptr, *w = nullptr, *r = nullptr, *z = nullptr, *q = nullptr;
    double *p0 = nullptr, *p1 = nullptr, *ks0 = nullptr, *ks1 = nullptr, *dm = nullptr;
    double *ft = nullptr;  // transient right-hand side
    uint8_t *mask = nullptr;
};

struct ProfEntry {
    int cls;
    hipEvent_t a, b;
    double bytes;
    int valid;
};

}  // namespace nnqp

struct nn_matrix {
    int64_t n = 0, nnz = 0;
    int *rowptr = nullptr;     // [n+1]
    int *col = nullptr;        // [nnz]
    double *val = nullptr;     // K values
    double *mval = nullptr;    // M values (or null)
    double *diag = nullptr;    // diag(K)
    double *kt = nullptr;      // M/dt + K values (transient), lazily formed
    double *kt_diag = nullptr;
    double kt_dt = 0.0;
    int lanes = 16;            // lanes per row of the SpMV kernels
    int max_row = 0;
};

struct nn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    double *partials = nullptr;      // [kMaxBlocks * kMaxRed]
    unsigned *ticket = nullptr;
    nnqp::DevScalars *scal = nullptr;
    nnqp::DevScalars *h_scal = nullptr;  // pinned mirror
    nnqp::Workspace ws;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool prof = false;
    std::vector<nnqp::ProfEntry> prof_live;
    std::vector<hipEvent_t> ev_pool;
    int64_t prof_count[NN_KCLASSES] = {0};
    double prof_ms[NN_KCLASSES] = {0};
    double prof_bytes[NN_KCLASSES] = {0};
};

namespace nnqp {

// status helpers
nn_status fail(nn_ctx *ctx, nn_status st, const std::string &msg);
#define NN_HIP_TRY(ctx, call)                                                        \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::nnqp::fail((ctx), NN_EHIP,                                      \
                                std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

nn_status ensure_workspace(nn_ctx *ctx, int64_t n);
nn_status read_scalars(nn_ctx *ctx);

// profiling around launches of a kernel class
void prof_begin(nn_ctx *ctx, int cls, double bytes);
void prof_end(nn_ctx *ctx);
void prof_collect(nn_ctx *ctx);

// ---------------------------------------------------------------- kernel launchers
// (kernels.hip).  All launch on ctx->stream with the partition of the matrix.
enum { KC_CG_SPMV = 0, KC_CG_UPDATE = 1, KC_GRAD = 2, KC_TRIAL = 3, KC_OTHER = 4 };

void launch_matvec(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *x, double *y);
// c: init (mode 0: c = c0v; mode 1: c = P(c)); reduce over f: |f|^2, max f, #nonfinite(f), #nonfinite(c)
void launch_init(nn_ctx *ctx, int64_t n, double *c, const double *f, int mode, double c0v);
// g = A c - f; reduce |pg|^2, #nonfinite, ||min(c,g)||_inf, min c, #zero
void launch_grad(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *c,
                 const double *f, double *g);
// s = P(c + t d) - c gathered; ks = A s; reduce g.s, s.As, s.s (rows with mask == 0 skipped if mask)
void launch_trial(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *c,
                  const double *d, double t, const double *g, const uint8_t *mask, double *ks);
// c = P(c + t d)
void launch_apply(nn_ctx *ctx, int64_t n, double *c, const double *d, double t);
// CG set-up on the free set of (c, g + ks): see kernels.hip
void launch_cg_setup(nn_ctx *ctx, const nn_matrix *A, const double *diag, const double *c,
                     double *g, const double *ks, double rtol, int max_it);
void launch_cg_spmv(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *p_old,
                    double *p_new);
void launch_cg_update(nn_ctx *ctx, int64_t n, const double *p);
// reduce over free rows: min_{w<0} c/(-w), g.w, w.w
void launch_breakpoint(nn_ctx *ctx, int64_t n, const double *c, const double *w, const double *g);
// active = (c == 0)
void launch_active(nn_ctx *ctx, int64_t n, const double *c, uint8_t *active);
// out = m/dt + k
void launch_axpby_vals(nn_ctx *ctx, int64_t nnz, const double *m, double dt, const double *k,
                       double *out);
void launch_diag(nn_ctx *ctx, const nn_matrix *A, const double *vals, double *diag);
// ft = f + (M c)/dt, fused SpMV
void launch_transient_rhs(nn_ctx *ctx, const nn_matrix *A, const double *c, const double *f,
                          double dt, double *ft);

// ---------------------------------------------------------------- assembly (assemble.hip)
nn_status assemble_impl(nn_ctx *ctx, const nn_mesh *mesh, const double *D, int64_t nD,
                        const double *kscale, const double *f_elem, const uint8_t *dirichlet,
                        int with_mass, nn_matrix **K_out, double *F_dev, int64_t *dof_of_node);

// ---------------------------------------------------------------- solver (solver.hip)
nn_status solve_impl(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *diag,
                     const double *f, const nn_opts *o, double *c, uint8_t *active, nn_stats *st);

int choose_lanes(double avg_row);
nn_status finish_matrix(nn_ctx *ctx, nn_matrix *A);

}  // namespace nnqp
