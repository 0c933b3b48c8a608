// Row-parallel kernels of the non-negative QP solver for gfx950.
//
// Every kernel here is bound by HBM bandwidth (sparse matrix-vector products
// at ~0.14 flop/byte and vector streams), so the design goal is bytes, not
// flops: CSR rows are processed by groups of G lanes of a 64-wide wavefront
// (G = 4..64 chosen from the mean row length), the column/value stream of
// consecutive rows is read contiguously by consecutive lanes, vector updates
// and dot products are fused into the SpMV passes that touch the same rows,
// and every reduction is one pass with a deterministic, ticketed last-block
// combine (no floating-point atomics).
#include <cmath>

#include "nnqp_internal.hpp"

namespace nnqp {

Part make_part(int64_t n, int max_blocks)
{
    Part p;
    p.n = (int)n;
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    if (nb > max_blocks) nb = max_blocks;
    nb = ((nb + kXcds - 1) / kXcds) * kXcds;
    int64_t chunk = (n + nb - 1) / nb;
    chunk = ((chunk + kBlock - 1) / kBlock) * kBlock;
    if (chunk < kBlock) chunk = kBlock;
    p.nb = (int)nb;
    p.chunk = (int)chunk;
    return p;
}

int choose_lanes(double avg_row)
{
    if (avg_row <= 4.0) return 4;
    if (avg_row <= 8.0) return 8;
    if (avg_row <= 16.0) return 16;
    if (avg_row <= 32.0) return 32;
    return 64;
}

// ---------------------------------------------------------------- reductions
enum : int { OP_SUM = 0, OP_MIN = 1, OP_MAX = 2 };

template <uint32_t OPS>
__device__ __forceinline__ constexpr int op_of(int k)
{
    return (int)((OPS >> (2 * k)) & 3u);
}

#define OPS2(a, b) ((uint32_t)(a) | ((uint32_t)(b) << 2))
#define OPS3(a, b, c) (OPS2(a, b) | ((uint32_t)(c) << 4))
#define OPS4(a, b, c, d) (OPS3(a, b, c) | ((uint32_t)(d) << 6))
#define OPS5(a, b, c, d, e) (OPS4(a, b, c, d) | ((uint32_t)(e) << 8))

__device__ __forceinline__ double red_comb(int op, double a, double b)
{
    return op == OP_SUM ? a + b : (op == OP_MIN ? fmin(a, b) : fmax(a, b));
}

template <uint32_t OPS, int NV>
__device__ __forceinline__ void red_init(double (&a)[NV])
{
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const int op = op_of<OPS>(k);
        a[k] = op == OP_SUM ? 0.0 : (op == OP_MIN ? INFINITY : -INFINITY);
    }
}

template <uint32_t OPS, int NV>
__device__ __forceinline__ void wave_red(double (&a)[NV])
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int k = 0; k < NV; k++) a[k] = red_comb(op_of<OPS>(k), a[k], __shfl_xor(a[k], o, 64));
}

// Block-wide reduction of a[]; the last block to finish combines the partials
// of all blocks in block order and returns true with the grid-wide result in
// a[] of every thread of that block.  The combination order is fixed for a
// given grid, so results are bitwise reproducible.  Partials go through
// device-scope atomic stores/loads so that blocks on different XCDs (separate
// L2s) see each other's values.
template <uint32_t OPS, int NV>
__device__ bool grid_reduce(double (&a)[NV], double *partials, unsigned *ticket)
{
    constexpr int W = kBlock / 64;
    __shared__ double sh[W][NV];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_red<OPS, NV>(a);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wid][k] = a[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double b[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) {
            b[k] = sh[0][k];
            for (int w = 1; w < W; w++) b[k] = red_comb(op_of<OPS>(k), b[k], sh[w][k]);
            __hip_atomic_store(&partials[blockIdx.x * NV + k], b[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        unsigned t = atomicAdd(ticket, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    red_init<OPS, NV>(a);
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock)
#pragma unroll
        for (int k = 0; k < NV; k++)
            a[k] = red_comb(op_of<OPS>(k), a[k],
                            __hip_atomic_load(&partials[b * NV + k], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT));
    wave_red<OPS, NV>(a);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wid][k] = a[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double v = sh[0][k];
        for (int w = 1; w < W; w++) v = red_comb(op_of<OPS>(k), v, sh[w][k]);
        a[k] = v;
    }
    if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// ---------------------------------------------------------------- row helpers
// Rows [r0, r1) of this block under the solve's partition.
struct RowRange {
    int r0, r1;
};

__device__ __forceinline__ RowRange block_rows(const Part &P)
{
    const int lb = xcd_block(blockIdx.x, P.nb);
    const long long r0 = (long long)lb * P.chunk;
    long long r1 = r0 + P.chunk;
    if (r1 > P.n) r1 = P.n;
    RowRange rr;
    rr.r0 = (int)(r0 < P.n ? r0 : P.n);
    rr.r1 = (int)(r1 > rr.r0 ? r1 : rr.r0);
    return rr;
}

// Sum over row i of v[k] * x(col[k]) by a group of G lanes: lane l takes
// entries l, l+G, ... and the group combines with a fixed butterfly.  Every
// lane of the group must call this (the shuffles are group-wide).
template <int G, class X>
__device__ __forceinline__ double row_dot(const int *__restrict__ rp, const int *__restrict__ ci,
                                          const double *__restrict__ v, int i, int lane, bool act,
                                          X x)
{
    double s = 0.0;
    if (act) {
        const int k1 = rp[i + 1];
        for (int k = rp[i] + lane; k < k1; k += G) s += v[k] * x(ci[k]);
    }
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, G);
    return s;
}

__device__ __forceinline__ double proj0(double x) { return x > 0.0 ? x : 0.0; }

// ---------------------------------------------------------------- kernels
template <int G>
__global__ __launch_bounds__(kBlock) void k_matvec(Part P, const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ x, double *__restrict__ y)
{
    constexpr int R = kBlock / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const RowRange rr = block_rows(P);
    for (int base = rr.r0; base < rr.r1; base += R) {
        const int i = base + grp;
        const bool act = i < rr.r1;
        const double s = row_dot<G>(rp, ci, v, i, lane, act, [&](int j) { return x[j]; });
        if (act && lane == 0) y[i] = s;
    }
}

// ft = f + (M c) / dt
template <int G>
__global__ __launch_bounds__(kBlock) void k_transient_rhs(Part P, const int *__restrict__ rp,
                                                          const int *__restrict__ ci,
                                                          const double *__restrict__ m,
                                                          const double *__restrict__ c,
                                                          const double *__restrict__ f, double dt,
                                                          double *__restrict__ ft)
{
    constexpr int R = kBlock / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const RowRange rr = block_rows(P);
    for (int base = rr.r0; base < rr.r1; base += R) {
        const int i = base + grp;
        const bool act = i < rr.r1;
        const double s = row_dot<G>(rp, ci, m, i, lane, act, [&](int j) { return c[j]; });
        if (act && lane == 0) ft[i] = f[i] + s / dt;
    }
}

// g = K c - f with the projected-gradient report.
// red: |pg|^2, #non-finite, ||min(c,g)||_inf, min c, #(c == 0)
constexpr uint32_t kOpsGrad = OPS5(OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM);

template <int G>
__global__ __launch_bounds__(kBlock) void k_grad(Part P, const int *__restrict__ rp,
                                                 const int *__restrict__ ci,
                                                 const double *__restrict__ v,
                                                 const double *__restrict__ c,
                                                 const double *__restrict__ f,
                                                 double *__restrict__ g, double *partials,
                                                 unsigned *ticket, DevScalars *S)
{
    constexpr int R = kBlock / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const RowRange rr = block_rows(P);
    double a[5];
    red_init<kOpsGrad, 5>(a);
    for (int base = rr.r0; base < rr.r1; base += R) {
        const int i = base + grp;
        const bool act = i < rr.r1;
        const double s = row_dot<G>(rp, ci, v, i, lane, act, [&](int j) { return c[j]; });
        if (act && lane == 0) {
            const double gi = s - f[i];
            const double cv = c[i];
            g[i] = gi;
            const double pg = cv > 0.0 ? gi : (gi < 0.0 ? gi : 0.0);
            a[0] += pg * pg;
            a[1] += (isfinite(gi) && isfinite(cv)) ? 0.0 : 1.0;
            a[2] = fmax(a[2], fabs(fmin(cv, gi)));
            a[3] = fmin(a[3], cv);
            a[4] += cv == 0.0 ? 1.0 : 0.0;
        }
    }
    if (grid_reduce<kOpsGrad, 5>(a, partials, ticket) && threadIdx.x == 0)
        for (int k = 0; k < 5; k++) S->red[k] = a[k];
}

// Trial point of a projected search: s = P(c + t d) - c, formed for every
// gathered column; ks = K s.  red: g.s, s.Ks, s.s.  Rows with mask == 0 are
// skipped when a mask is given (there d = 0, so s = 0 and they add nothing).
constexpr uint32_t kOpsTrial = OPS3(OP_SUM, OP_SUM, OP_SUM);

template <int G>
__global__ __launch_bounds__(kBlock) void k_trial(Part P, const int *__restrict__ rp,
                                                  const int *__restrict__ ci,
                                                  const double *__restrict__ v,
                                                  const double *__restrict__ c,
                                                  const double *__restrict__ d, double t,
                                                  const double *__restrict__ g,
                                                  const uint8_t *__restrict__ mask,
                                                  double *__restrict__ ks, double *partials,
                                                  unsigned *ticket, DevScalars *S)
{
    constexpr int R = kBlock / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const RowRange rr = block_rows(P);
    auto sv = [&](int j) {
        const double cj = c[j];
        return proj0(cj + t * d[j]) - cj;
    };
    double a[3];
    red_init<kOpsTrial, 3>(a);
    for (int base = rr.r0; base < rr.r1; base += R) {
        const int i = base + grp;
        const bool act = i < rr.r1 && (mask == nullptr || mask[i] != 0);
        const double s = row_dot<G>(rp, ci, v, i, lane, act, sv);
        if (act && lane == 0) {
            if (ks) ks[i] = s;
            const double si = sv(i);
            a[0] += g[i] * si;
            a[1] += si * s;
            a[2] += si * si;
        }
    }
    if (grid_reduce<kOpsTrial, 3>(a, partials, ticket) && threadIdx.x == 0)
        for (int k = 0; k < 3; k++) S->red[k] = a[k];
}

// c = P(c + t d)
__global__ __launch_bounds__(kBlock) void k_apply(Part P, double *__restrict__ c,
                                                  const double *__restrict__ d, double t)
{
    const RowRange rr = block_rows(P);
    for (int i = rr.r0 + threadIdx.x; i < rr.r1; i += kBlock) c[i] = proj0(c[i] + t * d[i]);
}

// c = c0v (mode 0) or c = P(c) (mode 1); report over f and c:
// |f|^2, max f, #non-finite f, #non-finite c (before projection)
constexpr uint32_t kOpsInit = OPS4(OP_SUM, OP_MAX, OP_SUM, OP_SUM);

__global__ __launch_bounds__(kBlock) void k_init(Part P, double *__restrict__ c,
                                                 const double *__restrict__ f, int mode, double c0v,
                                                 double *partials, unsigned *ticket, DevScalars *S)
{
    const RowRange rr = block_rows(P);
    double a[4];
    red_init<kOpsInit, 4>(a);
    for (int i = rr.r0 + threadIdx.x; i < rr.r1; i += kBlock) {
        const double fi = f[i];
        a[0] += fi * fi;
        a[1] = fmax(a[1], fi);
        a[2] += isfinite(fi) ? 0.0 : 1.0;
        if (mode == 0) {
            c[i] = c0v;
        } else {
            const double cv = c[i];
            a[3] += isfinite(cv) ? 0.0 : 1.0;
            c[i] = proj0(cv);
        }
    }
    if (grid_reduce<kOpsInit, 4>(a, partials, ticket) && threadIdx.x == 0)
        for (int k = 0; k < 4; k++) S->red[k] = a[k];
}

// Set-up of the inner CG on the face of (c, g + ks):
//   g <- g + ks (gradient at the Cauchy point), free = not (c == 0 and g >= 0),
//   dm = 1/diag on free rows and 0 elsewhere (the mask folded into the
//   Jacobi preconditioner), r = -g on free rows, z = dm r, p0 = p1 = w = 0.
// red: r.z, r.r, #free, nnz of free rows
constexpr uint32_t kOpsSetup = OPS4(OP_SUM, OP_SUM, OP_SUM, OP_SUM);

__global__ __launch_bounds__(kBlock) void k_cg_setup(
    Part P, const int *__restrict__ rp, const double *__restrict__ diag,
    const double *__restrict__ c, double *__restrict__ g, const double *__restrict__ ks,
    uint8_t *__restrict__ mask, double *__restrict__ dm, double *__restrict__ r,
    double *__restrict__ z, double *__restrict__ p0, double *__restrict__ p1,
    double *__restrict__ w, double rtol2, int max_it, double *partials, unsigned *ticket,
    DevScalars *S)
{
    const RowRange rr = block_rows(P);
    double a[4];
    red_init<kOpsSetup, 4>(a);
    for (int i = rr.r0 + threadIdx.x; i < rr.r1; i += kBlock) {
        const double gi = ks ? g[i] + ks[i] : g[i];
        if (ks) g[i] = gi;
        const double cv = c[i];
        const bool fr = !(cv == 0.0 && gi >= 0.0);
        const double dmi = fr ? 1.0 / diag[i] : 0.0;
        const double ri = fr ? -gi : 0.0;
        const double zi = dmi * ri;
        mask[i] = fr ? 1 : 0;
        dm[i] = dmi;
        r[i] = ri;
        z[i] = zi;
        p0[i] = 0.0;
        p1[i] = 0.0;
        w[i] = 0.0;
        a[0] += ri * zi;
        a[1] += ri * ri;
        a[2] += fr ? 1.0 : 0.0;
        a[3] += fr ? (double)(rp[i + 1] - rp[i]) : 0.0;
    }
    if (grid_reduce<kOpsSetup, 4>(a, partials, ticket) && threadIdx.x == 0) {
        S->rz = a[0];
        S->rr = a[1];
        S->rr_stop = rtol2 * a[1];
        S->n_free = a[2];
        S->nnz_free = a[3];
        S->alpha = 0.0;
        S->beta = 0.0;
        S->pq = 0.0;
        S->it = 0;
        S->max_it = max_it;
        S->done = !isfinite(a[0]) ? 4 : ((a[1] == 0.0 || a[2] == 0.0) ? 1 : 0);
        for (int k = 0; k < 4; k++) S->red[k] = a[k];
    }
}

// CG matrix pass with the direction update folded in:
//   p_new = z + beta p_old  (formed for every gathered column, written for own rows)
//   q = K p_new on free rows, alpha = r.z / p_new.q
// Columns outside the free set contribute 0 because z and p_old vanish there.
template <int G>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(Part P, const int *__restrict__ rp,
                                                    const int *__restrict__ ci,
                                                    const double *__restrict__ v,
                                                    const uint8_t *__restrict__ mask,
                                                    const double *__restrict__ z,
                                                    const double *__restrict__ p_old,
                                                    double *__restrict__ p_new,
                                                    double *__restrict__ q, double *partials,
                                                    unsigned *ticket, DevScalars *S)
{
    if (S->done) return;
    constexpr int R = kBlock / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const RowRange rr = block_rows(P);
    const double beta = S->beta;
    auto pv = [&](int j) { return fma(beta, p_old[j], z[j]); };
    double a[1] = {0.0};
    for (int base = rr.r0; base < rr.r1; base += R) {
        const int i = base + grp;
        const bool act = i < rr.r1 && mask[i] != 0;
        const double s = row_dot<G>(rp, ci, v, i, lane, act, pv);
        if (act && lane == 0) {
            const double pi = pv(i);
            p_new[i] = pi;
            q[i] = s;
            a[0] += pi * s;
        }
    }
    if (grid_reduce<OP_SUM, 1>(a, partials, ticket) && threadIdx.x == 0) {
        const double pq = a[0];
        S->pq = pq;
        if (pq > 0.0 && isfinite(pq)) {
            S->alpha = S->rz / pq;
        } else {
            S->alpha = 0.0;
            S->done = isfinite(pq) ? 3 : 4;
        }
    }
}

// CG vector update on free rows: w += alpha p, r -= alpha q, z = dm r;
// beta = r.z(new) / r.z(old); stop when r.r <= rr_stop or at max_it.
constexpr uint32_t kOpsUpd = OPS2(OP_SUM, OP_SUM);

__global__ __launch_bounds__(kBlock) void k_cg_update(Part P, const uint8_t *__restrict__ mask,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q,
                                                      const double *__restrict__ dm,
                                                      double *__restrict__ w, double *__restrict__ r,
                                                      double *__restrict__ z, double *partials,
                                                      unsigned *ticket, DevScalars *S)
{
    if (S->done) return;
    const RowRange rr = block_rows(P);
    const double alpha = S->alpha;
    double a[2] = {0.0, 0.0};
    for (int i = rr.r0 + threadIdx.x; i < rr.r1; i += kBlock) {
        if (!mask[i]) continue;
        const double ri = r[i] - alpha * q[i];
        const double zi = dm[i] * ri;
        w[i] += alpha * p[i];
        r[i] = ri;
        z[i] = zi;
        a[0] += ri * zi;
        a[1] += ri * ri;
    }
    if (grid_reduce<kOpsUpd, 2>(a, partials, ticket) && threadIdx.x == 0) {
        const int it = S->it + 1;
        S->it = it;
        const double rz_old = S->rz;
        S->beta = a[0] / rz_old;
        S->rz = a[0];
        S->rr = a[1];
        if (!isfinite(a[0]) || !isfinite(a[1])) S->done = 4;
        else if (a[1] <= S->rr_stop || it >= S->max_it || !(a[0] > 0.0)) S->done = 1;
    }
}

// Largest step along w before a free variable reaches its bound:
// red: min over w_i < 0 of c_i / (-w_i), g.w, w.w
constexpr uint32_t kOpsBrk = OPS3(OP_MIN, OP_SUM, OP_SUM);

__global__ __launch_bounds__(kBlock) void k_breakpoint(Part P, const double *__restrict__ c,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ g,
                                                       double *partials, unsigned *ticket,
                                                       DevScalars *S)
{
    const RowRange rr = block_rows(P);
    double a[3];
    red_init<kOpsBrk, 3>(a);
    for (int i = rr.r0 + threadIdx.x; i < rr.r1; i += kBlock) {
        const double wi = w[i];
        if (wi < 0.0) a[0] = fmin(a[0], c[i] / (-wi));
        a[1] += g[i] * wi;
        a[2] += wi * wi;
    }
    if (grid_reduce<kOpsBrk, 3>(a, partials, ticket) && threadIdx.x == 0)
        for (int k = 0; k < 3; k++) S->red[k] = a[k];
}

__global__ __launch_bounds__(kBlock) void k_active(Part P, const double *__restrict__ c,
                                                   uint8_t *__restrict__ active)
{
    const RowRange rr = block_rows(P);
    for (int i = rr.r0 + threadIdx.x; i < rr.r1; i += kBlock) active[i] = c[i] == 0.0 ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_vals_mdt_plus_k(int64_t nnz, const double *__restrict__ m,
                                                            double dt, const double *__restrict__ k,
                                                            double *__restrict__ out)
{
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * kBlock)
        out[t] = m[t] / dt + k[t];
}

__global__ __launch_bounds__(kBlock) void k_diag(Part P, const int *__restrict__ rp,
                                                 const int *__restrict__ ci,
                                                 const double *__restrict__ v,
                                                 double *__restrict__ diag)
{
    const RowRange rr = block_rows(P);
    for (int i = rr.r0 + threadIdx.x; i < rr.r1; i += kBlock) {
        double d = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; k++)
            if (ci[k] == i) d = v[k];
        diag[i] = d;
    }
}

// ---------------------------------------------------------------- launchers
#define NN_DISPATCH_G(lanes, KERNEL, grid, ...)                                            \
    switch (lanes) {                                                                       \
    case 4: KERNEL<4><<<grid, kBlock, 0, ctx->stream>>>(__VA_ARGS__); break;               \
    case 8: KERNEL<8><<<grid, kBlock, 0, ctx->stream>>>(__VA_ARGS__); break;               \
    case 16: KERNEL<16><<<grid, kBlock, 0, ctx->stream>>>(__VA_ARGS__); break;             \
    case 32: KERNEL<32><<<grid, kBlock, 0, ctx->stream>>>(__VA_ARGS__); break;             \
    default: KERNEL<64><<<grid, kBlock, 0, ctx->stream>>>(__VA_ARGS__); break;             \
    }

void launch_matvec(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *x, double *y)
{
    if (A->n == 0) return;
    Part P = make_part(A->n);
    NN_DISPATCH_G(A->lanes, k_matvec, P.nb, P, A->rowptr, A->col, vals, x, y);
}

void launch_transient_rhs(nn_ctx *ctx, const nn_matrix *A, const double *c, const double *f,
                          double dt, double *ft)
{
    if (A->n == 0) return;
    Part P = make_part(A->n);
    NN_DISPATCH_G(A->lanes, k_transient_rhs, P.nb, P, A->rowptr, A->col, A->mval, c, f, dt, ft);
}

void launch_init(nn_ctx *ctx, int64_t n, double *c, const double *f, int mode, double c0v)
{
    Part P = make_part(n);
    k_init<<<P.nb, kBlock, 0, ctx->stream>>>(P, c, f, mode, c0v, ctx->partials, ctx->ticket,
                                             ctx->scal);
}

void launch_grad(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *c,
                 const double *f, double *g)
{
    Part P = make_part(A->n);
    NN_DISPATCH_G(A->lanes, k_grad, P.nb, P, A->rowptr, A->col, vals, c, f, g, ctx->partials,
                  ctx->ticket, ctx->scal);
}

void launch_trial(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *c,
                  const double *d, double t, const double *g, const uint8_t *mask, double *ks)
{
    Part P = make_part(A->n);
    NN_DISPATCH_G(A->lanes, k_trial, P.nb, P, A->rowptr, A->col, vals, c, d, t, g, mask, ks,
                  ctx->partials, ctx->ticket, ctx->scal);
}

void launch_apply(nn_ctx *ctx, int64_t n, double *c, const double *d, double t)
{
    Part P = make_part(n);
    k_apply<<<P.nb, kBlock, 0, ctx->stream>>>(P, c, d, t);
}

void launch_cg_setup(nn_ctx *ctx, const nn_matrix *A, const double *diag, const double *c,
                     double *g, const double *ks, double rtol, int max_it)
{
    Part P = make_part(A->n);
    Workspace &W = ctx->ws;
    k_cg_setup<<<P.nb, kBlock, 0, ctx->stream>>>(P, A->rowptr, diag, c, g, ks, W.mask, W.dm, W.r,
                                                 W.z, W.p0, W.p1, W.w, rtol * rtol, max_it,
                                                 ctx->partials, ctx->ticket, ctx->scal);
}

void launch_cg_spmv(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *p_old,
                    double *p_new)
{
    Part P = make_part(A->n);
    Workspace &W = ctx->ws;
    NN_DISPATCH_G(A->lanes, k_cg_spmv, P.nb, P, A->rowptr, A->col, vals, W.mask, W.z, p_old, p_new,
                  W.q, ctx->partials, ctx->ticket, ctx->scal);
}

void launch_cg_update(nn_ctx *ctx, int64_t n, const double *p)
{
    Part P = make_part(n);
    Workspace &W = ctx->ws;
    k_cg_update<<<P.nb, kBlock, 0, ctx->stream>>>(P, W.mask, p, W.q, W.dm, W.w, W.r, W.z,
                                                  ctx->partials, ctx->ticket, ctx->scal);
}

void launch_breakpoint(nn_ctx *ctx, int64_t n, const double *c, const double *w, const double *g)
{
    Part P = make_part(n);
    k_breakpoint<<<P.nb, kBlock, 0, ctx->stream>>>(P, c, w, g, ctx->partials, ctx->ticket,
                                                   ctx->scal);
}

void launch_active(nn_ctx *ctx, int64_t n, const double *c, uint8_t *active)
{
    Part P = make_part(n);
    k_active<<<P.nb, kBlock, 0, ctx->stream>>>(P, c, active);
}

void launch_axpby_vals(nn_ctx *ctx, int64_t nnz, const double *m, double dt, const double *k,
                       double *out)
{
    int64_t nb = (nnz + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    k_vals_mdt_plus_k<<<(int)nb, kBlock, 0, ctx->stream>>>(nnz, m, dt, k, out);
}

void launch_diag(nn_ctx *ctx, const nn_matrix *A, const double *vals, double *diag)
{
    Part P = make_part(A->n);
    k_diag<<<P.nb, kBlock, 0, ctx->stream>>>(P, A->rowptr, A->col, vals, diag);
}

}  // namespace nnqp
