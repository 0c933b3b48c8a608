// Internal declarations of the MI355X non-negative QP library (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "nnqp.h"

namespace nnqp {

// ---------------------------------------------------------------- launch geometry
// The solver stores K in sliced-ELL form: rows are grouped in slices of 64
// (one wavefront), each slice padded to the longest row in it and stored
// column-major, so lane l of the wavefront owns row 64 s + l and every
// value/index load of the wavefront is one contiguous 512/256-byte segment.
// Every row-parallel kernel walks the slices grid-stride, one slice per
// wavefront at a time, with the same slice -> wavefront assignment, so the
// vectors a kernel writes are read back by the same wavefront (and XCD) in
// the next kernel.  Two 1024-thread blocks per CU fill its 32 wave slots.
constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / 64;
constexpr int kSlice = 64;
constexpr int kMaxBlocks = 512;    // 2 workgroups per CU on 256 CUs
constexpr int kMaxRed = 8;         // values per reduction
constexpr int kLadder = 3;         // step lengths of one Cauchy ladder pass (odd)
constexpr int kLadderBlocks = 256; // blocks of a ladder pass

struct Part {
    int n = 0;        // rows
    int nslices = 0;  // ceil(n / 64)
    int nb = 0;       // blocks
};

Part make_part(int64_t n, int max_blocks = kMaxBlocks);

// ---------------------------------------------------------------- reductions
// A reduction kernel leaves one partial per block and value in a slot of
// ctx->partials ([slot][value][block]); nothing is combined with atomics.
// Results the host needs are combined on the host in block order; results the
// next kernel needs (CG scalars) are combined by every block of that kernel in
// the same fixed order, so all blocks hold bitwise identical values.
enum { SLOT_HOST = 0, SLOT_U0 = 1, SLOT_U1 = 2, SLOT_Q = 3, kSlots = 4 };
enum : int { OP_SUM = 0, OP_MIN = 1, OP_MAX = 2 };

// ---------------------------------------------------------------- device scalars
// Scalars the CG kernels hand to each other without a host round trip.  Only
// block 0 of a kernel writes them; the next kernel on the stream reads them.
struct DevScalars {
    double rzh[2];         // r.z of CG iteration j, stored at j % 2
    double rr_stop;        // stop when r.r <= rr_stop
    double n_free;         // free rows of the current face
    double nnz_free;       // nonzeros in the free rows (byte model)
    double ww[2];          // |w_j|^2 of the CG iterate (trust-region solves), at j % 2
    int done;              // CG: 0 running, 1 converged/capped, 2 trust-region boundary,
                           // 3 breakdown, 4 non-finite
    int it;                // CG iterations done
    int tr_hit;            // the last update stopped w on the trust-region boundary
};

// ---------------------------------------------------------------- objects
struct Workspace {
    int64_t cap = 0;
    double *g = nullptr, *w = nullptr, *r = nullptr, *z = nullptr, *q = nullptr;
    double *p0 = nullptr, *p1 = nullptr, *ks0 = nullptr, *ks1 = nullptr, *dm = nullptr;
    double *ft = nullptr;  // transient right-hand side
    double *ks2 = nullptr;   // third Cauchy ladder product (with ks0, ks1)
    // float32 CG vectors of the mixed-precision inner solve
    float *w32 = nullptr, *r32 = nullptr, *z32 = nullptr, *q32 = nullptr, *p32 = nullptr,
          *dm32 = nullptr;
    uint8_t *mask = nullptr;
    // Chebyshev preconditioner vectors (allocated on first use): residual of
    // the inner Chebyshev iteration and its two increments (ping-pong)
    int64_t cheb_cap = 0;
    double *cres = nullptr, *cdz[2] = {nullptr, nullptr};
    float *cres32 = nullptr, *cdz32[2] = {nullptr, nullptr};
};

// Chebyshev polynomial preconditioner of degree `degree` for the inner CG:
// z = q(D^-1 A) D^-1 r, the Chebyshev iteration for A z = r from z = 0 with
// the Jacobi splitting on the interval [lmax / ratio, lmax], lmax the
// Gershgorin bound of D^-1 A.  theta, delta: centre and half-width of the
// interval; step i >= 1 forms dz_i = ca[i] dz_{i-1} + cb[i] D^-1 res_i.
struct Cheb {
    int degree = 1;
    double theta = 1.0, delta = 0.0;
    double ca[16] = {0}, cb[16] = {0};
};

// Buffers of the BLMVM solver (blmvm.hip), kept with the context.
struct LmWork {
    int64_t cap = 0;   // length of every vector
    int m = 0;         // pair slots
    double *S = nullptr, *Y = nullptr;   // [m][cap]: steps s and projected-gradient differences y
    double *pg = nullptr, *d = nullptr, *gn = nullptr;
    double *part = nullptr;              // [value][kMaxBlocks] partials of the pair pass
    void *state = nullptr, *h_state = nullptr;   // device state and its pinned mirror
};

// Matrix values used by a kernel: float32 when v32 is set, else float64.
struct Vals {
    const double *v64 = nullptr;
    const float *v32 = nullptr;
    const float *v32q = nullptr;   // v32 in the quad layout (with A->d16q), or null
    const double *v64p = nullptr;  // v64 in the paired layout (with A->d16p), or null
};

// Bounds lo <= c <= hi of a constrained solve (hi may be +inf; lo finite).
// Default: the non-negative QP.  Projection P(x) = min(max(x, lo), hi), with
// NaN mapped to lo.
struct Box {
    double lo = 0.0;
    double hi = __builtin_inf();
};

// A search direction in float64 or float32 (exactly one is set).
struct Dir {
    const double *f64 = nullptr;
    const float *f32 = nullptr;
};

struct ProfEntry {
    int cls;
    hipEvent_t a, b;                 // markers recorded before and after the launch
    hipEvent_t ka = nullptr, kb = nullptr;   // or the kernel's own begin and end
    int seq = -1;                    // CG launches: index within their chunk
    double bytes;       // algorithmic bytes of the layout the kernel reads
    double bytes_csr;   // the same launch under the paper's CSR byte model
    int valid;
};

// Device memory through the caller's hooks (nn_create_ex) or, without
// hooks, hipMalloc / hipFree.  Contexts and matrices each carry the hooks
// their buffers came from.
struct DevAlloc {
    nn_alloc_fn alloc = nullptr;
    nn_free_fn free_ = nullptr;
    void *user = nullptr;
};
hipError_t dev_malloc_raw(const DevAlloc &a, void **p, size_t bytes);
void dev_free(const DevAlloc &a, void *p);   // p may be null
template <class T>
inline hipError_t dev_malloc(const DevAlloc &a, T **p, size_t bytes)
{
    void *v = nullptr;
    const hipError_t e = dev_malloc_raw(a, &v, bytes);
    *p = static_cast<T *>(v);
    return e;
}

}  // namespace nnqp

struct nn_matrix {
    nnqp::DevAlloc al;         // hooks of the creating context (frees go through them)
    int64_t n = 0, nnz = 0;
    int *rowptr = nullptr;     // CSR pattern [n+1] (boundary format, export)
    int *col = nullptr;        // [nnz]
    int64_t nslices = 0, nsell = 0;
    int *sl_off = nullptr;     // [nslices+1] first entry of each 64-row slice
    int *sl_col = nullptr;     // [nsell] column of each sliced-ELL entry (padding: own row)
    short *sl_d16 = nullptr;   // [nsell] col - row as int16 when every offset fits, else null
    // Paired copies for the CG and search passes of the single-problem solver
    // (made when sl_d16 exists): within each slice, entries 2k and 2k+1 of a
    // row sit side by side (one 8- or 16-byte value load and one 4-byte offset
    // load per pair); an odd last column keeps its place.
    short *d16p = nullptr;
    double *val64p = nullptr;
    double *kt64p = nullptr;
    // Quad copies for the float32 CG and search passes (made when sl_d16
    // exists): entries 4k .. 4k+3 of a row side by side (one 16-byte value
    // load, one 8-byte offset load), two left-over entries as a pair, an odd
    // last one in place.
    short *d16q = nullptr;
    float *val32q = nullptr;
    float *kt32q = nullptr;
    double *val = nullptr;     // K values, sliced-ELL order [nsell]
    double *mval = nullptr;    // M values, sliced-ELL order (or null)
    double *diag = nullptr;    // diag(K)
    double *kt = nullptr;      // M/dt + K values (transient), lazily formed
    double *kt_diag = nullptr;
    double kt_dt = 0.0;
    float *val32 = nullptr;    // float32 K values (mixed precision), lazily formed
    float *kt32 = nullptr;     // float32 M/dt + K values, formed with kt
    int wmax = 0;              // widest slice
    int max_row = 0;
};

struct nn_ctx {
    nnqp::DevAlloc al;         // device memory hooks (default: hipMalloc / hipFree)
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream for graph capture (batched CG)
    std::string err;
    double *partials = nullptr;      // [kSlots][kMaxBlocks][kMaxRed]
    double *h_part = nullptr;        // pinned host copy of one slot
    double *h_multi = nullptr;       // pinned host copy of the gradient + Cauchy ladder partials
    nnqp::DevScalars *scal = nullptr;
    nnqp::DevScalars *h_scal = nullptr;  // pinned mirror
    nnqp::Workspace ws;
    nnqp::LmWork lm;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool prof = false;
    int prof_mask = 0;         // classes timed while prof is on
    bool prof_open = false;    // a begin event was recorded and awaits its end
    bool prof_attach = false;  // the next row-kernel launch takes the open entry's kernel events
    int prof_every = 1;        // time one CG-class launch in prof_every
    int prof_seq = -1;         // chunk index the next CG-class entry is tagged with
    int64_t prof_calls[NN_KCLASSES] = {0};   // CG-class launches seen (sampling)
    std::vector<nnqp::ProfEntry> prof_live;
    std::vector<hipEvent_t> ev_pool;
    int64_t prof_count[NN_KCLASSES] = {0};
    double prof_ms[NN_KCLASSES] = {0};
    double prof_bytes[NN_KCLASSES] = {0};
    double prof_bytes_csr[NN_KCLASSES] = {0};
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
// Option checks shared by the solve entry points (api.hip).
nn_status check_opts(nn_ctx *ctx, const nn_opts *o);

// Single-problem solves up to this many rows run in one workgroup and one
// launch (solo.hip) when the options allow it (nn_opts.engine).
constexpr int64_t kSoloMaxRows = 4096;
// whether the solve of A with options o can run in one workgroup
bool solo_eligible(const nn_matrix *A, const nn_opts *o);
// the TRON solve of solver.hip in one workgroup (float64 values `vals`)
nn_status solo_solve_impl(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *diag,
                          const double *f, const nn_opts *o, double *c, uint8_t *active,
                          nn_stats *st);

// Rows the fixed work array of nn_solve_nonneg_noalloc holds (noalloc.hip).
constexpr int64_t kNoAllocMaxRows = 262144;
// Take the current device's address of that array (once per device; called
// by nn_create with the device current).
void noalloc_attach(int device);

// Sliced-ELL offsets of a CSR pattern: off[s] for s = 0..nslices, widest slice.
void sell_offsets(const int64_t *rowptr, int64_t n, std::vector<int64_t> &off, int &wmax);
// Device CSR values (ordered by rowptr) -> sliced-ELL arrays of A (col, vals, diag).
nn_status sell_build(nn_ctx *ctx, nn_matrix *A, const int64_t *rowptr_host, const double *csr_val,
                     const double *csr_mval);
nn_status read_scalars(nn_ctx *ctx);
// Combine the host-slot partials of the last reduction kernel over n rows;
// ops[k] is OP_SUM / OP_MIN / OP_MAX for value k.
nn_status host_reduce(nn_ctx *ctx, int64_t n, int nv, const int *ops, double *out);

// profiling around launches of a kernel class.  bytes: algorithmic bytes of
// the layout the kernel reads (index width, paired copies); bytes_csr: the
// same launch under the paper's CSR model (Sec. 4, Table 2: 4-byte column
// indices, every vector operand of the unfused operations counted), NaN for
// "the same as bytes"
void prof_begin(nn_ctx *ctx, int cls, double bytes, double bytes_csr = __builtin_nan(""));
void prof_end(nn_ctx *ctx);
void prof_collect(nn_ctx *ctx);
// For the CG classes (one kernel per bracket): the open entry's kernel
// events, which the launch passes to hipExtLaunchKernelGGL so that they
// record the kernel's own begin and end instead of markers around it.
// False (a, b untouched) when no such entry is waiting.
bool prof_kernel_events(nn_ctx *ctx, hipEvent_t *a, hipEvent_t *b);
// add one timed launch of class cls (ms, algorithmic bytes) to the totals
void prof_add(nn_ctx *ctx, int cls, double ms, double bytes, double bytes_csr = __builtin_nan(""));

// ---------------------------------------------------------------- kernel launchers
// (kernels.hip).  All launch on ctx->stream with the partition of the rows.
// Kernels marked [host] leave partials for host_reduce; their value lists
// are given in order.
enum { KC_CG_SPMV = 0, KC_CG_UPDATE = 1, KC_GRAD = 2, KC_TRIAL = 3, KC_OTHER = 4 };
// CG faces: the complement of the binding set (the Cauchy point's face), every
// row (unconstrained solve), the rows strictly inside the bounds (a subspace
// step: variables at a bound stay there until the next Cauchy step)
enum { FACE_BINDING = 0, FACE_ALL = 1, FACE_INTERIOR = 2 };

void launch_matvec(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *x, double *y);
// [host] c = c0v (mode 0) or P(c) (mode 1); |f|^2 sum, max f, #nonfinite f sum, #nonfinite c sum
void launch_init(nn_ctx *ctx, int64_t n, double *c, const double *f, int mode, double c0v, Box B);
// [host] g = A c - f; |pg|^2 sum, #nonfinite sum, ||c - P(c - g)||_inf max, min c min,
// #(c at a bound) sum
void launch_grad(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *vals_p,
                 const double *c, const double *f, double *g, Box B);
// [host] s = P(c + t d) - c gathered, ks = A s; g.s, s.As, s.s (sums); rows with mask == 0 skipped
void launch_trial(nn_ctx *ctx, const nn_matrix *A, const Vals &V, const double *c, Dir d,
                  double t, const double *g, const uint8_t *mask, double *ks, Box B);
// [SLOT_U0..U1, 15 values] Cauchy ladder: for k < kLadder, s_k = P(c - t[k] g) - c,
// ks[k] = A s_k; g.s_k, s_k.A s_k, s_k.s_k as values 3k..3k+2
void launch_ladder(nn_ctx *ctx, const nn_matrix *A, const Vals &V, const double *c,
                   const double *g, const double *t, double *const *ks, Box B);
// c = P(c + t d)
void launch_apply(nn_ctx *ctx, int64_t n, double *c, Dir d, double t, Box B);
// CG set-up on the face of (c, g + ks) (every row not binding: not at lo with
// g >= 0, not at hi with g <= 0: FACE_BINDING; every row: FACE_ALL; every row
// strictly inside the bounds: FACE_INTERIOR); partials of r.z,
// r.r, #free, nnz(free) in SLOT_U0; f32 selects the float32 CG vectors
void launch_cg_setup(nn_ctx *ctx, const nn_matrix *A, const double *diag, const double *c,
                     double *g, const double *ks, bool f32, Box B, int face,
                     const Cheb *ch = nullptr);
// Chebyshev step `step` (1..degree-1) on the free rows; the last one writes
// r.z into value 0 of partial slot `slot`
void launch_cheb(nn_ctx *ctx, const nn_matrix *A, const Vals &V, const Cheb &ch, int step,
                 int slot);
// [host] Gershgorin bound of D^-1 A (max)
void launch_gersh(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *diag);
// Chebyshev coefficients for `degree` on [lmax / ratio, lmax], and the vectors
// it needs; degree <= 1 leaves ch->degree = 1 (plain Jacobi)
nn_status cheb_prepare(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *diag,
                       int degree, Cheb *ch);
// [host] r = A c - f (not stored): |r|^2 sum, #nonfinite sum, max c max, min c min, #(c<0) sum
void launch_resid(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *c,
                  const double *f);
// c += w (float64 CG solution vector)
void launch_add(nn_ctx *ctx, int64_t n, double *c, const double *w);
// CG iteration j: direction update + matrix pass (prologue: scalars from the
// previous kernel's partials); float32 values and vectors when V.v32 is set.
// tr: a trust-region solve (the pass also reduces p.p and w.p for the update)
void launch_cg_spmv(nn_ctx *ctx, const nn_matrix *A, const Vals &V, int j, int max_it, double rtol,
                    bool tr = false);
// CG iteration j: vector update (Chebyshev start terms when ch is given).
// delta2 finite: the iterate w stays in the ball |w| <= sqrt(delta2); a step
// that would leave it stops on the boundary (Steihaug) and ends the CG.
void launch_cg_update(nn_ctx *ctx, int64_t n, int j, bool f32, const Cheb *ch = nullptr,
                      double delta2 = __builtin_inf());
// [host] first bound crossing along w: min over w<0 of (c-lo)/(-w) and over
// w>0 of (hi-c)/w, min; g.w sum, w.w sum
void launch_breakpoint(nn_ctx *ctx, int64_t n, const double *c, Dir w, const double *g, Box B);
// b = (float)a
void launch_to_f32(nn_ctx *ctx, int64_t m, const double *a, float *b);
// paired copies of a sliced-ELL array of A (layout of nn_matrix::d16p)
void launch_pair_d16(nn_ctx *ctx, const nn_matrix *A, const short *src, short *dst);
void launch_pair_f64(nn_ctx *ctx, const nn_matrix *A, const double *src, double *dst);
// quad copies (layout of nn_matrix::d16q)
void launch_quad_f32(nn_ctx *ctx, const nn_matrix *A, const float *src, float *dst);
void launch_quad_d16(nn_ctx *ctx, const nn_matrix *A, const short *src, short *dst);
// active = 1 where c == lo, 2 where c == hi, else 0
void launch_active(nn_ctx *ctx, int64_t n, const double *c, uint8_t *active, Box B);
// out = m/dt + k
void launch_axpby_vals(nn_ctx *ctx, int64_t nnz, const double *m, double dt, const double *k,
                       double *out);
// [host] int16 offsets col - row into sd; max |col - row| over real rows (max)
void launch_sell_d16(nn_ctx *ctx, const nn_matrix *A, short *sd);
void launch_diag(nn_ctx *ctx, const nn_matrix *A, const double *vals, double *diag);
// csr -> sliced-ELL: col, values (and capacity values), diag
void launch_csr_to_sell(nn_ctx *ctx, nn_matrix *A, const double *csr_val, const double *csr_mval);
// ft = f + (M c)/dt, fused SpMV
void launch_transient_rhs(nn_ctx *ctx, const nn_matrix *A, const double *c, const double *f,
                          double dt, double *ft);

// ---------------------------------------------------------------- assembly (assemble.hip)
nn_status assemble_impl(nn_ctx *ctx, const nn_mesh *mesh, const double *D, int64_t nD,
                        const double *kscale, const double *f_elem, const uint8_t *dirichlet,
                        const double *dvals, int with_mass, nn_matrix **K_out, double *F_dev,
                        int64_t *dof_of_node);

// ---------------------------------------------------------------- solver (solver.hip)
// vals: float64 values (gradient, always); vals32: float32 values for the
// searches and the inner CG (mixed precision) or null; vals32q: the same in
// the quad layout, or null; vals64p: vals in the paired layout, or null.
nn_status solve_impl(nn_ctx *ctx, const nn_matrix *A, const double *vals, const float *vals32,
                     const float *vals32q, const double *vals64p, const double *diag,
                     const double *f, const nn_opts *o, double *c, uint8_t *active, nn_stats *st);

nn_status finish_matrix(nn_ctx *ctx, nn_matrix *A);

// The same problem by BLMVM (blmvm.hip); vals are float64 values of A.
nn_status blmvm_impl(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *f,
                     const nn_opts *o, double *c, uint8_t *active, nn_stats *st);
void lm_release(nn_ctx *ctx);

// Unconstrained Galerkin solve K c = f by Jacobi-PCG from c = 0 (solver.hip).
nn_status galerkin_impl(nn_ctx *ctx, const nn_matrix *A, const double *f, const nn_opts *o,
                        double *c, nn_stats *st);

// ---------------------------------------------------------------- batched solver (batch.hip)
// P problems solved together; arrays are host arrays of P entries (see
// nn_solve_batch).  Arguments are validated by the caller.  dt > 0: one
// backward-Euler step of every member (its M/dt + K values must have been
// formed by ensure_transient; f is the load, c = c^n in and c^(n+1) out).
nn_status solve_batch_impl(nn_ctx *ctx, int P, nn_matrix *const *K, const double *const *f,
                           const nn_opts *o, double *const *c, uint8_t *const *active,
                           nn_stats *stats, double dt);
// Form (once per dt) the M/dt + K values, their diagonal and, for mixed
// precision, their float32 copy; with `paired`, also the copy the
// single-problem solver reads at this precision (paired float64 or quad
// float32, with their int16 offsets).
nn_status ensure_transient(nn_ctx *ctx, nn_matrix *K, double dt, bool mixed, bool paired);

}  // namespace nnqp
