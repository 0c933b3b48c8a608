// Batched solver: many independent non-negative QPs (Sec. 2.1.3, eq.
// non-negative) advanced together by one set of launches.
//
// Every step of the TRON-style outer iteration (the same steps, constants and
// tests as the single-problem solver) is one grid-stride launch over the
// slices of all problems; each problem keeps its own control state (Cauchy
// step, trust radius, CG scalars, stopping test, counters) in per-problem
// device and host arrays, and a problem that has converged drops out of the
// launches.
//
// Layout: the problems keep their own sliced-ELL matrices, reached through
// per-problem pointer tables.  The batch numbers their 64-row slices
// consecutively (a slice never spans two problems) and concatenates the work
// vectors over those slices, so global row s*64 + lane is local row
// (s - first slice of its problem)*64 + lane.  Each reduction leaves one
// partial per slice; a finalize kernel with one block per problem combines the
// slices of its problem in a fixed order.  A member's arithmetic therefore
// depends only on its own data: its result is bitwise the same in any batch
// and for any launch shape the autotuner picks.
//
// The CG iteration (matrix pass, finalize, vector update, finalize) takes all
// its scalars from device memory, so a chunk of iterations is captured once
// per call into a hipGraph and replayed until every member's CG has stopped.
// The autotuner times the batched matrix pass over block sizes and grid sizes
// once per size class and keeps the fastest shape.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "nnqp_internal.hpp"

// 1: CG chunks replayed as a captured graph; 0: launched one by one
#ifndef NNQP_BATCH_GRAPH
#define NNQP_BATCH_GRAPH 1
#endif

namespace nnqp {

namespace {

constexpr int kBNV = 5;          // values per slice partial
constexpr int kFinBlock = 256;   // threads of a finalize block (one block per problem)
constexpr double kMu0 = 0.01;    // sufficient-decrease constant
constexpr double kExtrap = 10.0; // Cauchy extrapolation factor
constexpr double kInterp = 0.1;  // Cauchy interpolation factor
constexpr double kBack = 0.5;    // projected-search backtracking factor
constexpr int kMaxTrials = 60;

// Per-problem state read and written by the batched kernels.
struct BProb {
    double t;          // step of the current trial / apply; 0: not taking part
    double rz;         // r.z of the current CG iteration
    double rr_stop;    // CG stops when r.r <= rr_stop
    double alpha, beta;
    double n_free, nnz_free;
    int it;            // CG iterations done
    int max_it;
    int done;          // CG: 0 running, 1 stopped, 3 breakdown, 4 non-finite
    int ksbuf;         // which K s buffer a Cauchy trial writes
    int active;        // 1 while the problem iterates
    int pad;
};

struct BDev {
    int P, nslices;
    const int *cnt;                 // [2] slices and problems in the current lists
    const int *plist;               // problems taking part in the current step
    const int *slist;               // their slices, problem by problem
    const int *sprob;               // [nslices] problem of each slice
    const int *s0, *nrow;           // per problem: first slice, rows
    const int *const *so;           // per problem sliced-ELL offsets
    const int *const *sc;           // per problem sliced-ELL columns (local)
    const short *const *sd;         // per problem int16 offsets col - row (or null)
    const double *const *v64;       // per problem float64 values
    const float *const *v32;        // per problem float32 values (mixed precision)
    const double *const *diag;      // per problem diagonal
    const int *const *rowptr;       // per problem CSR row pointers
    double *const *c;               // per problem solution vectors (local rows)
    const double *const *f;         // per problem loads of the solve
    const double *const *f0;        // per problem loads (transient step: f of f + M c/dt)
    const double *const *mv;        // per problem capacity values (transient step)
    uint8_t *const *act_out;        // per problem active-set outputs (entries may be null)
    BProb *bp;
    double *part;                   // [nslices][kBNV]
    double *pres;                   // [P][kBNV]
};

__device__ __forceinline__ double bcomb(int op, double a, double b)
{
    return op == OP_SUM ? a + b : (op == OP_MIN ? fmin(a, b) : fmax(a, b));
}

__device__ __forceinline__ double bident(int op)
{
    return op == OP_SUM ? 0.0 : (op == OP_MIN ? INFINITY : -INFINITY);
}

__device__ __forceinline__ double proj0b(double x) { return x > 0.0 ? x : 0.0; }

// Walk the slices of the current list grid-stride, one wavefront per slice.
// For a slice of a problem with take(p): body(p, s, global row, local row, row
// exists, a); every listed slice then stores its wave-combined partials
// (identities when the problem did not take part).
template <int NV, class Take, class Body>
__device__ __forceinline__ void for_bslices(const BDev &B, const int (&ops)[NV], Take take,
                                            Body body)
{
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    const int nlist = B.cnt[0];
    for (int t = blockIdx.x * wpb + wid; t < nlist; t += nw) {
        const int s = B.slist[t];
        double a[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) a[k] = bident(ops[k]);
        const int p = B.sprob[s];
        if (take(p)) {
            const int il = (s - B.s0[p]) * kSlice + lane;
            body(p, s, s * kSlice + lane, il, il < B.nrow[p], a);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
            for (int k = 0; k < NV; k++) a[k] = bcomb(ops[k], a[k], __shfl_xor(a[k], o, 64));
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < NV; k++) B.part[(size_t)s * kBNV + k] = a[k];
    }
}

// Column modes of the batched matrix passes (as in the single-problem
// kernels): int32 columns, or int16 offsets from the row (float32 values,
// when every member has them).  Float64 values load with the non-temporal
// hint, float32 values normally (as in the single-problem kernels).
enum { CM_I32 = 0, CM_D16 = 2 };

__device__ __forceinline__ double bld_val(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float bld_val(const float *p) { return *p; }

// Row sums of slice s of problem p: sum_k val(k) x(col(k)), with the same
// wave-uniform load phases (eight entries each) and column order as the
// single-problem kernels.  Padding and rows past the end hold valid columns.
template <int WMAX, int CM, class VT, class X>
__device__ __forceinline__ double bsell_row(const BDev &B, const VT *__restrict__ sv, int p, int s,
                                            X x)
{
    const int lane = threadIdx.x & 63;
    const int ls = s - B.s0[p];
    const int lrow = ls * kSlice + lane;
    const int *__restrict__ so = B.so[p];
    const int *__restrict__ sc = B.sc[p];
    const short *__restrict__ sd = B.sd[p];
    auto col = [&](int e) {
        if (CM == CM_D16) return lrow + (int)sd[e];
        return sc[e];
    };
    const int off = so[ls];
    const int w = (so[ls + 1] - off) >> 6;
    double acc = 0.0;
    constexpr int H = WMAX < 8 ? WMAX : 8;
#pragma unroll
    for (int h0 = 0; h0 < WMAX; h0 += H) {
        int cc[H];
        VT vv[H];
#pragma unroll
        for (int k = 0; k < H; k++) {
            if (h0 + k < w) {
                cc[k] = col(off + (h0 + k) * kSlice + lane);
                vv[k] = bld_val(sv + off + (h0 + k) * kSlice + lane);
            } else {
                cc[k] = 0;
                vv[k] = VT(0);
            }
        }
#pragma unroll
        for (int k = 0; k < H; k++)
            if (h0 + k < w) acc += (double)vv[k] * x(cc[k]);
    }
    for (int k = WMAX; k < w; k++) {
        const int e = off + k * kSlice + lane;
        acc += (double)bld_val(sv + e) * x(col(e));
    }
    return acc;
}

// ---------------------------------------------------------------- kernels
// c = c0v (mode 0) or P(c) (mode 1); |f|^2, max f, #non-finite f, #non-finite c
__global__ void kb_init(BDev B, int mode, double c0v)
{
    const int ops[4] = {OP_SUM, OP_MAX, OP_SUM, OP_SUM};
    for_bslices<4>(B, ops, [&](int p) { return B.bp[p].active != 0; },
                   [&](int p, int, int, int il, bool row, double (&a)[4]) {
                       if (!row) return;
                       const double fi = B.f[p][il];
                       a[0] += fi * fi;
                       a[1] = fmax(a[1], fi);
                       a[2] += isfinite(fi) ? 0.0 : 1.0;
                       double *c = B.c[p];
                       if (mode == 0) {
                           c[il] = c0v;
                       } else {
                           const double cv = c[il];
                           a[3] += isfinite(cv) ? 0.0 : 1.0;
                           c[il] = proj0b(cv);
                       }
                   });
}

// Right-hand side of a backward-Euler step, ft = f0 + (M c) / dt, written
// into the concatenated vector ft (the solve's loads point into it).
template <int WMAX>
__global__ void kb_transient_rhs(BDev B, double dt, double *__restrict__ ft)
{
    const int ops[1] = {OP_SUM};
    for_bslices<1>(B, ops, [&](int p) { return B.bp[p].active != 0; },
                   [&](int p, int s, int i, int il, bool row, double (&)[1]) {
                       const double *c = B.c[p];
                       const double mc =
                           bsell_row<WMAX, CM_I32>(B, B.mv[p], p, s, [&](int j) { return c[j]; });
                       if (row) ft[i] = B.f0[p][il] + mc / dt;
                   });
}

// g = K c - f; |pg|^2, #non-finite, ||min(c,g)||_inf, min c, #(c == 0)
template <int WMAX>
__global__ void kb_grad(BDev B, double *__restrict__ g)
{
    const int ops[5] = {OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM};
    for_bslices<5>(B, ops, [&](int p) { return B.bp[p].active != 0; },
                   [&](int p, int s, int i, int il, bool row, double (&a)[5]) {
                       const double *c = B.c[p];
                       const double kc =
                           bsell_row<WMAX, CM_I32>(B, B.v64[p], p, s, [&](int j) { return c[j]; });
                       if (!row) return;
                       const double gi = kc - B.f[p][il];
                       const double cv = c[il];
                       g[i] = gi;
                       const double pg = cv > 0.0 ? gi : (gi < 0.0 ? gi : 0.0);
                       a[0] += pg * pg;
                       a[1] += (isfinite(gi) && isfinite(cv)) ? 0.0 : 1.0;
                       a[2] = fmax(a[2], fabs(fmin(cv, gi)));
                       a[3] = fmin(a[3], cv);
                       a[4] += cv == 0.0 ? 1.0 : 0.0;
                   });
}

// Trial of a projected search for the problems with t_p != 0:
// s = P(c + t_p d) - c formed for every gathered column, ks = K s (written to
// buffer ksbuf_p when write_ks); g.s, s.Ks, s.s.  With a mask only free rows
// are formed (d vanishes elsewhere, so s does too).
template <int WMAX, int CM, class VT, class VD>
__global__ void kb_trial(BDev B, const VT *const *vals, const VD *__restrict__ d,
                         const double *__restrict__ g, const uint8_t *__restrict__ mask,
                         double *__restrict__ ks0, double *__restrict__ ks1, int write_ks)
{
    const int ops[3] = {OP_SUM, OP_SUM, OP_SUM};
    for_bslices<3>(B, ops, [&](int p) { return B.bp[p].active != 0 && B.bp[p].t != 0.0; },
                   [&](int p, int s, int i, int il, bool row, double (&a)[3]) {
                       const double t = B.bp[p].t;
                       const double *c = B.c[p];
                       const int r0 = B.s0[p] * kSlice;
                       auto sv = [&](int j) {
                           const double cj = c[j];
                           return proj0b(cj + t * (double)d[r0 + j]) - cj;
                       };
                       const bool live = row && (mask == nullptr || mask[i] != 0);
                       if (__ballot(live) == 0) return;
                       const double ksv = bsell_row<WMAX, CM>(B, vals[p], p, s, sv);
                       if (!live) return;
                       if (write_ks) (B.bp[p].ksbuf ? ks1 : ks0)[i] = ksv;
                       const double si = sv(il);
                       a[0] += g[i] * si;
                       a[1] += si * ksv;
                       a[2] += si * si;
                   });
}

// c = P(c + t_p d) for the problems with t_p != 0
template <class VD>
__global__ void kb_apply(BDev B, const VD *__restrict__ d)
{
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    const int nlist = B.cnt[0];
    for (int k = blockIdx.x * wpb + wid; k < nlist; k += nw) {
        const int s = B.slist[k];
        const int p = B.sprob[s];
        const double t = B.bp[p].t;
        if (!B.bp[p].active || t == 0.0) continue;
        const int il = (s - B.s0[p]) * kSlice + lane;
        if (il >= B.nrow[p]) continue;
        double *c = B.c[p];
        c[il] = proj0b(c[il] + t * (double)d[s * kSlice + lane]);
    }
}

// CG set-up on the face of (c, g + ks_p): g <- g + ks, free = not (c == 0 and
// g >= 0), dm = 1/diag on free rows (0 elsewhere), r = -g on free rows,
// z = dm r, p = q = w = 0.  r.z, r.r, #free, nnz of the free rows.
template <class VV>
__global__ void kb_cg_setup(BDev B, double *__restrict__ g, const double *__restrict__ ks0,
                            const double *__restrict__ ks1, uint8_t *__restrict__ mask,
                            VV *__restrict__ dm, VV *__restrict__ r, VV *__restrict__ z,
                            VV *__restrict__ pv, VV *__restrict__ q, VV *__restrict__ w)
{
    const int ops[4] = {OP_SUM, OP_SUM, OP_SUM, OP_SUM};
    for_bslices<4>(B, ops, [&](int p) { return B.bp[p].active != 0; },
                   [&](int p, int, int i, int il, bool row, double (&a)[4]) {
                       if (!row) {
                           mask[i] = 0;
                           dm[i] = r[i] = z[i] = pv[i] = q[i] = w[i] = VV(0);
                           return;
                       }
                       const double *ks = B.bp[p].ksbuf ? ks1 : ks0;
                       const double gi = g[i] + ks[i];
                       g[i] = gi;
                       const double cv = B.c[p][il];
                       const bool fr = !(cv == 0.0 && gi >= 0.0);
                       const VV dmi = fr ? (VV)(1.0 / B.diag[p][il]) : VV(0);
                       const VV ri = fr ? (VV)(-gi) : VV(0);
                       const VV zi = dmi * ri;
                       mask[i] = fr ? 1 : 0;
                       dm[i] = dmi;
                       r[i] = ri;
                       z[i] = zi;
                       pv[i] = VV(0);
                       q[i] = VV(0);
                       w[i] = VV(0);
                       a[0] += (double)ri * (double)zi;
                       a[1] += (double)ri * (double)ri;
                       a[2] += fr ? 1.0 : 0.0;
                       const int *rp = B.rowptr[p];
                       a[3] += fr ? (double)(rp[il + 1] - rp[il]) : 0.0;
                   });
}

// CG matrix pass for the running problems: p <- z + beta_p p and
// q <- K z + beta_p q on the free rows (one gather of z, as in the
// single-problem pass); p.q.
template <int WMAX, int CM, class VT, class VV>
__global__ void kb_cg_spmv(BDev B, const VT *const *vals, const uint8_t *__restrict__ mask,
                           const VV *__restrict__ z, VV *__restrict__ pv, VV *__restrict__ q)
{
    const int ops[1] = {OP_SUM};
    for_bslices<1>(B, ops, [&](int p) { return B.bp[p].active != 0 && B.bp[p].done == 0; },
                   [&](int p, int s, int i, int, bool row, double (&a)[1]) {
                       const bool live = row && mask[i] != 0;
                       if (__ballot(live) == 0) return;
                       const int r0 = B.s0[p] * kSlice;
                       const double kz = bsell_row<WMAX, CM>(
                           B, vals[p], p, s, [&](int j) { return (double)z[r0 + j]; });
                       if (!live) return;
                       const double beta = B.bp[p].beta;
                       const VV pi = (VV)fma(beta, (double)pv[i], (double)z[i]);
                       const VV qi = (VV)fma(beta, (double)q[i], kz);
                       pv[i] = pi;
                       q[i] = qi;
                       a[0] += (double)pi * (double)qi;
                   });
}

// CG vector update on the free rows of the running problems:
// w += alpha p, r -= alpha q, z = dm r; r.z, r.r
template <class VV>
__global__ void kb_cg_update(BDev B, const uint8_t *__restrict__ mask, const VV *__restrict__ pv,
                             const VV *__restrict__ q, const VV *__restrict__ dm,
                             VV *__restrict__ w, VV *__restrict__ r, VV *__restrict__ z)
{
    const int ops[2] = {OP_SUM, OP_SUM};
    for_bslices<2>(B, ops, [&](int p) { return B.bp[p].active != 0 && B.bp[p].done == 0; },
                   [&](int p, int, int i, int, bool row, double (&a)[2]) {
                       if (!row || !mask[i]) return;
                       const double alpha = B.bp[p].alpha;
                       const VV ri = (VV)((double)r[i] - alpha * (double)q[i]);
                       const VV zi = dm[i] * ri;
                       w[i] = (VV)((double)w[i] + alpha * (double)pv[i]);
                       r[i] = ri;
                       z[i] = zi;
                       a[0] += (double)ri * (double)zi;
                       a[1] += (double)ri * (double)ri;
                   });
}

// Breakpoint of the search along w: min over w < 0 of c/(-w); g.w; w.w
template <class VV>
__global__ void kb_breakpoint(BDev B, const VV *__restrict__ w, const double *__restrict__ g)
{
    const int ops[3] = {OP_MIN, OP_SUM, OP_SUM};
    for_bslices<3>(B, ops, [&](int p) { return B.bp[p].active != 0; },
                   [&](int p, int, int i, int il, bool row, double (&a)[3]) {
                       if (!row) return;
                       const double wi = (double)w[i];
                       if (wi < 0.0) a[0] = fmin(a[0], B.c[p][il] / (-wi));
                       a[1] += g[i] * wi;
                       a[2] += wi * wi;
                   });
}

// active-set outputs: 1 where c == 0
__global__ void kb_active(BDev B)
{
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    for (int s = blockIdx.x * wpb + wid; s < B.nslices; s += nw) {
        const int p = B.sprob[s];
        uint8_t *out = B.act_out[p];
        const int il = (s - B.s0[p]) * kSlice + lane;
        if (out && il < B.nrow[p]) out[il] = B.c[p][il] == 0.0 ? 1 : 0;
    }
}

// Combine the slice partials of listed problem blockIdx.x in a fixed order (thread t
// takes slices t, t + 256, ...; then a wave butterfly; then the four waves in
// order) into pres[p].  MODE adds the CG scalar logic that follows the
// reduction: 1 after the set-up, 2 after the matrix pass, 3 after the update.
// Problems that are inactive (or, for MODE 2 and 3, whose CG has stopped) are
// skipped, so their state is left untouched.
template <int NV, int MODE>
__global__ __launch_bounds__(kFinBlock) void kb_finalize(BDev B, int ops_code, double rtol2)
{
    if ((int)blockIdx.x >= B.cnt[1]) return;
    const int p = B.plist[blockIdx.x];
    BProb &bp = B.bp[p];
    if (!bp.active || (MODE >= 2 && bp.done)) return;
    __shared__ double sh[kFinBlock / 64][NV];
    int ops[NV];
    double a[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) {
        ops[k] = (ops_code >> (2 * k)) & 3;
        a[k] = bident(ops[k]);
    }
    const int s1 = B.s0[p] + (B.nrow[p] + kSlice - 1) / kSlice;
    for (int s = B.s0[p] + threadIdx.x; s < s1; s += kFinBlock)
#pragma unroll
        for (int k = 0; k < NV; k++) a[k] = bcomb(ops[k], a[k], B.part[(size_t)s * kBNV + k]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int k = 0; k < NV; k++) a[k] = bcomb(ops[k], a[k], __shfl_xor(a[k], o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wid][k] = a[k];
    __syncthreads();
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double v = sh[0][k];
        for (int w = 1; w < kFinBlock / 64; w++) v = bcomb(ops[k], v, sh[w][k]);
        a[k] = v;
        B.pres[(size_t)p * kBNV + k] = v;
    }
    if (MODE == 1) {
        // r.z_0, r.r_0, #free, nnz(free); stop before the first iteration
        // when the face is empty or the residual vanishes
        bp.rz = a[0];
        bp.rr_stop = rtol2 * a[1];
        bp.n_free = a[2];
        bp.nnz_free = a[NV > 3 ? 3 : 0];
        bp.beta = 0.0;
        bp.alpha = 0.0;
        bp.it = 0;
        if (!isfinite(a[0]) || !isfinite(a[1])) bp.done = 4;
        else if (a[1] == 0.0 || a[2] == 0.0 || bp.max_it <= 0 || !(a[0] > 0.0)) bp.done = 1;
        else bp.done = 0;
    } else if (MODE == 2) {
        // alpha = r.z / p.q; breakdown on non-positive or non-finite curvature
        const double pq = a[0];
        if (!isfinite(pq)) bp.done = 4;
        else if (!(pq > 0.0)) bp.done = 3;
        else bp.alpha = bp.rz / pq;
    } else if (MODE == 3) {
        // iteration done: beta for the next one, stopping test on r.r
        const double rz = a[0], rr = a[NV > 1 ? 1 : 0];
        bp.it += 1;
        bp.beta = rz / bp.rz;
        bp.rz = rz;
        if (!isfinite(rz) || !isfinite(rr)) bp.done = 4;
        else if (rr <= bp.rr_stop || bp.it >= bp.max_it || !(rz > 0.0)) bp.done = 1;
    }
}

constexpr int opsc(int a, int b = 0, int c = 0, int d = 0, int e = 0)
{
    return a | (b << 2) | (c << 4) | (d << 6) | (e << 8);
}

// ---------------------------------------------------------------- host side
struct Shape {
    int block = 256;   // threads per block
    int per_cu = 8;    // blocks per CU (the grid is capped by the slice count)
};

// size class -> tuned shape (per process; the class is (log2 rows, widest
// slice class, precision))
std::map<std::tuple<int, int, int>, Shape> &shape_cache()
{
    static std::map<std::tuple<int, int, int>, Shape> m;
    return m;
}

int width_class(int wmax) { return wmax <= 8 ? 8 : (wmax <= 16 ? 16 : 32); }

#define NN_BDISPATCH(wmax, KERNEL, grid, block, stream, ...)                                    \
    do {                                                                                        \
        if ((wmax) <= 8) {                                                                      \
            constexpr int WM = 8;                                                               \
            hipLaunchKernelGGL(KERNEL, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);        \
        } else if ((wmax) <= 16) {                                                              \
            constexpr int WM = 16;                                                              \
            hipLaunchKernelGGL(KERNEL, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);        \
        } else {                                                                                \
            constexpr int WM = 32;                                                              \
            hipLaunchKernelGGL(KERNEL, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);        \
        }                                                                                       \
    } while (0)

// Device and pinned host memory of one batched call, released on every exit.
struct Arena {
    std::vector<void *> dev, host;
    bool ok = true;
    template <class T>
    T *d(size_t n)
    {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
            ok = false;
            return nullptr;
        }
        dev.push_back(p);
        return (T *)p;
    }
    template <class T>
    T *h(size_t n)
    {
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(T) * std::max<size_t>(n, 1), hipHostMallocDefault) !=
            hipSuccess) {
            ok = false;
            return nullptr;
        }
        host.push_back(p);
        return (T *)p;
    }
    ~Arena()
    {
        for (void *p : dev) (void)hipFree(p);
        for (void *p : host) (void)hipHostFree(p);
    }
};

// Captured CG chunks, one per launch-size class (the grid of a captured
// launch is fixed; the lists it walks are read from device memory).
struct GraphCache {
    struct G {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::map<int, G> by_class;
    ~GraphCache()
    {
        for (auto &kv : by_class) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        }
    }
};

struct Events {
    std::vector<hipEvent_t> ev;
    ~Events()
    {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    bool create(size_t n, unsigned flags)
    {
        ev.assign(n, nullptr);
        for (hipEvent_t &e : ev)
            if (hipEventCreateWithFlags(&e, flags) != hipSuccess) return false;
        return true;
    }
};

}  // namespace

nn_status solve_batch_impl(nn_ctx *ctx, int P, nn_matrix *const *K, const double *const *f,
                           const nn_opts *o, double *const *c, uint8_t *const *active,
                           nn_stats *stats, double dt)
{
    hipStream_t st = ctx->stream;
    const bool mixed = o->precision == NN_MIXED;
    const bool transient = dt > 0.0;
    std::vector<nn_stats> SP(P);
    for (nn_stats &x : SP) std::memset(&x, 0, sizeof(x));

    // ---- slice numbering
    std::vector<int> s0(P), nrow(P), nsl(P), sprob;
    int wmax = 1;
    int64_t S = 0;
    for (int p = 0; p < P; p++) {
        const int64_t n = K[p]->n;
        nrow[p] = (int)n;
        s0[p] = (int)S;
        nsl[p] = (int)((n + kSlice - 1) / kSlice);
        S += nsl[p];
        if (S * kSlice >= (int64_t)1 << 31)
            return fail(ctx, NN_EINVAL, "batch too large: total rows must stay below 2^31");
        for (int t = 0; t < nsl[p]; t++) sprob.push_back(p);
        if (n > 0) wmax = std::max(wmax, K[p]->wmax);
        if (mixed && n > 0 && !transient && !K[p]->val32) {
            if (hipMalloc(&K[p]->val32, sizeof(float) * std::max<int64_t>(K[p]->nsell, 1)) !=
                hipSuccess)
                return fail(ctx, NN_EOOM, "float32 value allocation");
            launch_to_f32(ctx, K[p]->nsell, K[p]->val, K[p]->val32);
        }
    }
    if (S == 0) {
        if (stats)
            for (int p = 0; p < P; p++) stats[p] = SP[p];
        ctx->err.clear();
        return NN_OK;
    }
    const int64_t R = S * kSlice;
    bool all_d16 = true;
    for (int p = 0; p < P; p++)
        if (K[p]->n > 0 && !K[p]->sl_d16) all_d16 = false;

    // ---- tables, work vectors, lists, pinned state mirrors
    Arena A;
    int *d_sprob = A.d<int>(S), *d_s0 = A.d<int>(P), *d_nrow = A.d<int>(P);
    int *d_list = A.d<int>((size_t)2 + P + S);
    const int **d_so = A.d<const int *>(P), **d_sc = A.d<const int *>(P),
              **d_rp = A.d<const int *>(P);
    const short **d_sd = A.d<const short *>(P);
    const double **d_v64 = A.d<const double *>(P), **d_diag = A.d<const double *>(P),
                 **d_f = A.d<const double *>(P), **d_f0 = A.d<const double *>(P),
                 **d_mv = A.d<const double *>(P);
    const float **d_v32 = A.d<const float *>(P);
    double **d_c = A.d<double *>(P);
    uint8_t **d_act = A.d<uint8_t *>(P);
    BProb *d_bp = A.d<BProb>(P);
    double *d_part = A.d<double>((size_t)S * kBNV), *d_pres = A.d<double>((size_t)P * kBNV);
    double *g = A.d<double>(R), *ks0 = A.d<double>(R), *ks1 = A.d<double>(R);
    double *ft = transient ? A.d<double>(R) : nullptr;
    uint8_t *mask = A.d<uint8_t>(R);
    double *w64 = nullptr, *r64 = nullptr, *z64 = nullptr, *p64 = nullptr, *q64 = nullptr,
           *dm64 = nullptr;
    float *w32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr,
          *dm32 = nullptr;
    if (mixed) {
        w32 = A.d<float>(R), r32 = A.d<float>(R), z32 = A.d<float>(R);
        p32 = A.d<float>(R), q32 = A.d<float>(R), dm32 = A.d<float>(R);
    } else {
        w64 = A.d<double>(R), r64 = A.d<double>(R), z64 = A.d<double>(R);
        p64 = A.d<double>(R), q64 = A.d<double>(R), dm64 = A.d<double>(R);
    }
    BProb *hb = A.h<BProb>(P);
    double *pres = A.h<double>((size_t)P * kBNV);
    const void **tab = (const void **)A.h<void *>((size_t)P * 12);
    // Uploads from pinned memory read their source when they execute, so
    // the host writes each upload into a staging copy that it does not touch
    // again until the copy's event has completed.
    constexpr int kStage = 4;
    BProb *bp_stage[kStage];
    int *lst_stage[kStage];
    for (int k = 0; k < kStage; k++) {
        bp_stage[k] = A.h<BProb>(P);
        lst_stage[k] = A.h<int>((size_t)2 + P + S);
    }
    if (!A.ok) return fail(ctx, NN_EOOM, "batch workspace allocation failed");
    Events ev_bp, ev_lst, ev_t;
    if (!ev_bp.create(kStage, hipEventDisableTiming) || !ev_lst.create(kStage, hipEventDisableTiming) ||
        !ev_t.create(2, hipEventDefault))
        return fail(ctx, NN_EHIP, "event creation");
    hipEvent_t t0 = ev_t.ev[0], t1 = ev_t.ev[1];

    // a transient step solves with the M/dt + K values, loads f + M c/dt
    for (int p = 0; p < P; p++) {
        tab[0 * P + p] = K[p]->sl_off;
        tab[1 * P + p] = K[p]->sl_col;
        tab[2 * P + p] = K[p]->rowptr;
        tab[3 * P + p] = transient ? K[p]->kt : K[p]->val;
        tab[4 * P + p] = transient ? K[p]->kt_diag : K[p]->diag;
        tab[5 * P + p] = transient ? (const void *)(ft + (size_t)s0[p] * kSlice) : f[p];
        tab[6 * P + p] = transient ? K[p]->kt32 : K[p]->val32;
        tab[7 * P + p] = c[p];
        tab[8 * P + p] = active ? active[p] : nullptr;
        tab[9 * P + p] = f[p];
        tab[10 * P + p] = K[p]->mval;
        tab[11 * P + p] = K[p]->sl_d16;
    }
    {
        void *dsts[12] = {d_so, d_sc, d_rp, d_v64, d_diag, d_f, d_v32, d_c, d_act, d_f0, d_mv, d_sd};
        for (int k = 0; k < 12; k++)
            NN_HIP_TRY(ctx, hipMemcpyAsync(dsts[k], tab + (size_t)k * P, sizeof(void *) * P,
                                           hipMemcpyHostToDevice, st));
        NN_HIP_TRY(ctx, hipMemcpyAsync(d_sprob, sprob.data(), sizeof(int) * S,
                                       hipMemcpyHostToDevice, st));
        NN_HIP_TRY(ctx, hipMemcpyAsync(d_s0, s0.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
        NN_HIP_TRY(ctx,
                   hipMemcpyAsync(d_nrow, nrow.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
        // the pageable sources above must stay alive until the copies finish
        NN_HIP_TRY(ctx, hipStreamSynchronize(st));
    }
    BDev B;
    B.P = P;
    B.nslices = (int)S;
    B.cnt = d_list;
    B.plist = d_list + 2;
    B.slist = d_list + 2 + P;
    B.sprob = d_sprob;
    B.s0 = d_s0;
    B.nrow = d_nrow;
    B.so = d_so;
    B.sc = d_sc;
    B.sd = d_sd;
    B.v64 = d_v64;
    B.v32 = d_v32;
    B.diag = d_diag;
    B.rowptr = d_rp;
    B.c = d_c;
    B.f = d_f;
    B.f0 = d_f0;
    B.mv = d_mv;
    B.act_out = d_act;
    B.bp = d_bp;
    B.part = d_part;
    B.pres = d_pres;

    std::memset(hb, 0, sizeof(BProb) * P);
    for (int p = 0; p < P; p++) {
        hb[p].active = nrow[p] > 0 ? 1 : 0;
        hb[p].max_it = o->max_cg;
    }
    int bp_next = 0, lst_next = 0;
    auto push = [&]() {
        const int k = bp_next;
        bp_next = (bp_next + 1) % kStage;
        if (hipEventSynchronize(ev_bp.ev[k]) != hipSuccess) return false;
        std::memcpy(bp_stage[k], hb, sizeof(BProb) * P);
        return hipMemcpyAsync(d_bp, bp_stage[k], sizeof(BProb) * P, hipMemcpyHostToDevice, st) ==
                   hipSuccess &&
               hipEventRecord(ev_bp.ev[k], st) == hipSuccess;
    };
    auto pull_state = [&]() {
        return hipMemcpyAsync(hb, d_bp, sizeof(BProb) * P, hipMemcpyDeviceToHost, st) ==
                   hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    auto pull_res = [&]() {
        return hipMemcpyAsync(pres, d_pres, sizeof(double) * P * kBNV, hipMemcpyDeviceToHost,
                              st) == hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    auto any_active = [&]() {
        for (int p = 0; p < P; p++)
            if (hb[p].active) return true;
        return false;
    };
    // The problems taking part in a step, and their slices, as device lists:
    // rebuilt and uploaded only when the selection changes.
    std::vector<char> sel(P, 0), sel_cur(P, 2);
    int n_sl = 0, n_pr = 0;
    auto select = [&](auto pred) -> bool {
        bool same = true;
        for (int p = 0; p < P; p++) {
            sel[p] = pred(p) ? 1 : 0;
            same = same && sel[p] == sel_cur[p];
        }
        if (same) return true;
        const int k = lst_next;
        lst_next = (lst_next + 1) % kStage;
        if (hipEventSynchronize(ev_lst.ev[k]) != hipSuccess) return false;
        int *h = lst_stage[k];
        int np = 0, ns = 0;
        for (int p = 0; p < P; p++) {
            sel_cur[p] = sel[p];
            if (!sel[p]) continue;
            h[2 + np++] = p;
            for (int t = 0; t < nsl[p]; t++) h[2 + P + ns++] = s0[p] + t;
        }
        h[0] = ns;
        h[1] = np;
        n_sl = ns;
        n_pr = np;
        return hipMemcpyAsync(d_list, h, sizeof(int) * ((size_t)2 + P + ns), hipMemcpyHostToDevice,
                              st) == hipSuccess &&
               hipEventRecord(ev_lst.ev[k], st) == hipSuccess;
    };
    auto is_active = [&](int p) { return hb[p].active != 0; };

    int num_cu = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
            num_cu = prop.multiProcessorCount;
    }
    Shape sh;
    auto grid_for = [&](const Shape &t, int64_t slices) {
        const int64_t blocks = (slices + t.block / 64 - 1) / (t.block / 64);
        return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)num_cu * t.per_cu));
    };

    NN_HIP_TRY(ctx, push() ? hipSuccess : hipErrorUnknown);
    NN_HIP_TRY(ctx, select(is_active) ? hipSuccess : hipErrorUnknown);
    NN_HIP_TRY(ctx, hipEventRecord(t0, st));

    // ---- transient right-hand sides (from c^n, before the start point is set)
    if (transient)
        NN_BDISPATCH(wmax, (kb_transient_rhs<WM>), grid_for(sh, n_sl), sh.block, st, B, dt, ft);
    // ---- start point and load statistics
    hipLaunchKernelGGL(kb_init, dim3(grid_for(sh, n_sl)), dim3(sh.block), 0, st, B,
                       o->c0_mode == 1 ? 1 : 0, o->c0_value);
    hipLaunchKernelGGL((kb_finalize<4, 0>), dim3(std::max(n_pr, 1)), dim3(kFinBlock), 0, st, B,
                       opsc(OP_SUM, OP_MAX, OP_SUM, OP_SUM), 0.0);
    if (!pull_res()) return fail(ctx, NN_EHIP, "batch read-back");
    std::vector<double> normf(P, 0.0), tcau(P, 1.0), delta(P, INFINITY);
    std::vector<int> status(P, NN_EMAXIT), outer(P, 0);
    for (int p = 0; p < P; p++) {
        if (!hb[p].active) {
            status[p] = NN_OK;
            continue;
        }
        const double *r = &pres[(size_t)p * kBNV];
        normf[p] = std::sqrt(r[0]);
        SP[p].norm_f = normf[p];
        SP[p].bytes_moved += 16.0 * nrow[p];
        if (o->delta0 > 0.0) delta[p] = o->delta0;
        if (r[2] != 0.0 || r[3] != 0.0) {
            status[p] = NN_ENONFINITE;
            hb[p].active = 0;
        } else if (!(r[1] > 0.0)) {
            // f <= 0: c = 0 satisfies c >= 0, g = -f >= 0, c.g = 0
            NN_HIP_TRY(ctx, hipMemsetAsync(c[p], 0, sizeof(double) * nrow[p], st));
            status[p] = NN_OK;
            SP[p].n_active = nrow[p];
            hb[p].active = 0;
        }
    }

    // ---- launch shape for this size class
    const auto key = std::make_tuple((int)std::log2((double)R), width_class(wmax), (int)mixed);
    auto &cache = shape_cache();
    if (cache.count(key)) {
        sh = cache[key];
    } else if (any_active()) {
        // time the gradient pass (the batched matrix pass with the most
        // per-row work) for each candidate shape; it writes only g and the
        // slice partials, which the first outer iteration overwrites
        NN_HIP_TRY(ctx, push() ? hipSuccess : hipErrorUnknown);
        NN_HIP_TRY(ctx, select(is_active) ? hipSuccess : hipErrorUnknown);
        float best = INFINITY;
        Shape pick = sh;
        for (int blk : {256, 512, 1024})
            for (int per_cu : {2, 4, 8}) {
                if (blk * per_cu > 4096) continue;
                const Shape cand{blk, per_cu};
                const int gsz = grid_for(cand, n_sl);
                NN_BDISPATCH(wmax, (kb_grad<WM>), gsz, blk, st, B, g);   // warm-up
                NN_HIP_TRY(ctx, hipEventRecord(t0, st));
                for (int rep = 0; rep < 3; rep++)
                    NN_BDISPATCH(wmax, (kb_grad<WM>), gsz, blk, st, B, g);
                NN_HIP_TRY(ctx, hipEventRecord(t1, st));
                NN_HIP_TRY(ctx, hipEventSynchronize(t1));
                float ms = 0.f;
                NN_HIP_TRY(ctx, hipEventElapsedTime(&ms, t0, t1));
                if (ms < best) {
                    best = ms;
                    pick = cand;
                }
            }
        sh = pick;
        cache[key] = sh;
        if (o->verbose)
            std::fprintf(stderr,
                         "nnqp batch shape: %lld rows, slice width %d -> %d threads, %d blocks/CU\n",
                         (long long)R, wmax, sh.block, sh.per_cu);
        NN_HIP_TRY(ctx, hipEventRecord(t0, st));   // the call's clock restarts after tuning
    }
    const int blk = sh.block;
    auto grid = [&]() { return grid_for(sh, n_sl); };
    auto fgrid = [&]() { return std::max(n_pr, 1); };

    // ---- launch helpers (each on the current lists)
    const double *gptr = g;
    auto trial = [&](bool along_w, const uint8_t *m, int write_ks) {
        const int gr = grid();
        if (mixed && all_d16) {
            if (along_w)
                NN_BDISPATCH(wmax, (kb_trial<WM, CM_D16, float, float>), gr, blk, st, B, d_v32,
                             (const float *)w32, gptr, m, ks0, ks1, write_ks);
            else
                NN_BDISPATCH(wmax, (kb_trial<WM, CM_D16, float, double>), gr, blk, st, B, d_v32,
                             gptr, gptr, m, ks0, ks1, write_ks);
        } else if (mixed) {
            if (along_w)
                NN_BDISPATCH(wmax, (kb_trial<WM, CM_I32, float, float>), gr, blk, st, B, d_v32,
                             (const float *)w32, gptr, m, ks0, ks1, write_ks);
            else
                NN_BDISPATCH(wmax, (kb_trial<WM, CM_I32, float, double>), gr, blk, st, B, d_v32,
                             gptr, gptr, m, ks0, ks1, write_ks);
        } else {
            NN_BDISPATCH(wmax, (kb_trial<WM, CM_I32, double, double>), gr, blk, st, B, d_v64,
                         along_w ? (const double *)w64 : gptr, gptr, m, ks0, ks1, write_ks);
        }
        hipLaunchKernelGGL((kb_finalize<3, 0>), dim3(fgrid()), dim3(kFinBlock), 0, st, B,
                           opsc(OP_SUM, OP_SUM, OP_SUM), 0.0);
    };
    auto apply = [&](bool along_w) {
        if (mixed && along_w)
            hipLaunchKernelGGL((kb_apply<float>), dim3(grid()), dim3(blk), 0, st, B,
                               (const float *)w32);
        else
            hipLaunchKernelGGL((kb_apply<double>), dim3(grid()), dim3(blk), 0, st, B,
                               along_w ? (const double *)w64 : gptr);
    };
    // one CG iteration on stream s with launch grids gr (slices) and fg
    // (problems), optionally bracketed by timing events
    auto cg_iter = [&](hipStream_t s, int gr, int fg, hipEvent_t *ev) {
        if (ev) (void)hipEventRecord(ev[0], s);
        if (mixed && all_d16)
            NN_BDISPATCH(wmax, (kb_cg_spmv<WM, CM_D16, float, float>), gr, blk, s, B, d_v32, mask,
                         z32, p32, q32);
        else if (mixed)
            NN_BDISPATCH(wmax, (kb_cg_spmv<WM, CM_I32, float, float>), gr, blk, s, B, d_v32, mask,
                         z32, p32, q32);
        else
            NN_BDISPATCH(wmax, (kb_cg_spmv<WM, CM_I32, double, double>), gr, blk, s, B, d_v64, mask,
                         z64, p64, q64);
        if (ev) (void)hipEventRecord(ev[1], s);
        hipLaunchKernelGGL((kb_finalize<1, 2>), dim3(fg), dim3(kFinBlock), 0, s, B, opsc(OP_SUM),
                           0.0);
        if (ev) (void)hipEventRecord(ev[2], s);
        if (mixed)
            hipLaunchKernelGGL((kb_cg_update<float>), dim3(gr), dim3(blk), 0, s, B, mask, p32, q32,
                               dm32, w32, r32, z32);
        else
            hipLaunchKernelGGL((kb_cg_update<double>), dim3(gr), dim3(blk), 0, s, B, mask, p64,
                               q64, dm64, w64, r64, z64);
        if (ev) (void)hipEventRecord(ev[3], s);
        hipLaunchKernelGGL((kb_finalize<2, 3>), dim3(fg), dim3(kFinBlock), 0, s, B,
                           opsc(OP_SUM, OP_SUM), 0.0);
    };

    // ---- CG chunks.  Without profiling a chunk is captured into a graph on
    // the context's private capture stream (the caller's stream may be the
    // legacy default stream, which cannot be captured) and replayed on the
    // caller's stream; one graph per size class of the running list (the
    // grid is fixed at capture, the lists are read from device memory).
    // With profiling on, or if capture fails, the launches are enqueued one
    // by one, bracketed by events when profiling.
    const int chunk = o->cg_chunk > 0 ? o->cg_chunk : 16;
    GraphCache graphs;
    bool use_graph = NNQP_BATCH_GRAPH && !ctx->prof;
    if (use_graph && !ctx->cap_stream &&
        hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        ctx->cap_stream = nullptr;
        use_graph = false;
    }
    auto graph_for = [&](int slices) -> hipGraphExec_t {
        int cls = 0;
        while ((1 << cls) < slices) cls++;
        auto it = graphs.by_class.find(cls);
        if (it != graphs.by_class.end()) return it->second.exec;
        const int gr = grid_for(sh, (int64_t)1 << cls);
        const int fg = std::min(P, 1 << cls);   // a listed problem owns at least one slice
        if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        for (int k = 0; k < chunk; k++) cg_iter(ctx->cap_stream, gr, fg, nullptr);
        hipGraph_t gph = nullptr;
        const bool ended = hipStreamEndCapture(ctx->cap_stream, &gph) == hipSuccess && gph;
        (void)hipGetLastError();
        if (!ended) {
            if (gph) (void)hipGraphDestroy(gph);
            return nullptr;
        }
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0) != hipSuccess || !ex) {
            (void)hipGraphDestroy(gph);
            (void)hipGetLastError();
            return nullptr;
        }
        graphs.by_class[cls] = GraphCache::G{gph, ex};
        return ex;
    };
    Events ev_cg;
    if (ctx->prof && !ev_cg.create((size_t)4 * chunk, hipEventDefault))
        return fail(ctx, NN_EHIP, "event creation");
    hipEvent_t *chunk_ev = ctx->prof ? ev_cg.ev.data() : nullptr;

    const double vb = mixed ? 4.0 : 8.0;   // bytes per CG vector entry and per value
    const double ib = (mixed && all_d16) ? 2.0 : 4.0;   // bytes per column index
    std::vector<int> it_before(P);
    std::vector<double> b_spmv(chunk), b_upd(chunk);
    nn_status err = NN_OK;
#define NN_BFAIL(msg)                  \
    {                                  \
        err = fail(ctx, NN_EHIP, msg); \
        break;                         \
    }

    enum { C_FIRST, C_EXT, C_INT, C_DONE };
    std::vector<int> cst(P), cur(P), nstep(P), sst(P);
    std::vector<double> t(P), gs(P), sks(P), ss(P), bmin(P), wn(P), ts(P);
    auto ok_dec = [&](int p, double a, double b, double s2) {
        return a < 0.0 && a + 0.5 * b <= kMu0 * a && std::sqrt(s2) <= delta[p];
    };
    auto stepping = [&](int p) { return hb[p].active != 0 && hb[p].t != 0.0; };
    for (int it_outer = 0; any_active(); it_outer++) {
        // ---- 1. gradient, convergence test per problem
        for (int p = 0; p < P; p++) hb[p].t = 0.0;
        if (!push() || !select(is_active)) NN_BFAIL("batch state upload");
        prof_begin(ctx, KC_GRAD, -1.0);
        NN_BDISPATCH(wmax, (kb_grad<WM>), grid(), blk, st, B, g);
        prof_end(ctx);
        hipLaunchKernelGGL((kb_finalize<5, 0>), dim3(fgrid()), dim3(kFinBlock), 0, st, B,
                           opsc(OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM), 0.0);
        if (!pull_res()) NN_BFAIL("batch read-back");
        for (int p = 0; p < P; p++) {
            if (!hb[p].active) continue;
            const double *r = &pres[(size_t)p * kBNV];
            const double n = nrow[p], nz = (double)K[p]->nnz;
            SP[p].spmvs++;
            SP[p].bytes_moved += 4.0 * (n + 1) + 12.0 * nz + 32.0 * n;
            if (r[1] != 0.0) {
                status[p] = NN_ENONFINITE;
                hb[p].active = 0;
                continue;
            }
            SP[p].kkt_rel = std::sqrt(r[0]) / normf[p];
            SP[p].kkt_nat_inf = r[2];
            SP[p].min_c = r[3];
            SP[p].n_active = (int32_t)r[4];
            SP[p].outer_its = outer[p];
            if (mixed) SP[p].refinements = outer[p] + 1;
            if (SP[p].kkt_rel <= o->tol) {
                status[p] = NN_OK;
                hb[p].active = 0;
            } else if (outer[p] >= o->max_outer) {
                status[p] = NN_EMAXIT;
                hb[p].active = 0;
            }
        }
        if (!any_active()) break;

        // ---- 2. Cauchy points: per-problem projected searches along -g
        // (start from the previous step, extrapolate x10 while the decrease
        // test holds, else interpolate x0.1 until it holds)
        for (int p = 0; p < P; p++) {
            cst[p] = hb[p].active ? C_FIRST : C_DONE;
            cur[p] = 0;
            nstep[p] = 0;
            t[p] = tcau[p];
        }
        for (;;) {
            bool any = false;
            for (int p = 0; p < P; p++) {
                hb[p].t = 0.0;
                if (!hb[p].active || cst[p] == C_DONE) continue;
                any = true;
                hb[p].t = -(cst[p] == C_EXT ? t[p] * kExtrap : t[p]);
                hb[p].ksbuf = cst[p] == C_EXT ? (cur[p] ^ 1) : cur[p];
            }
            if (!any) break;
            if (!push() || !select(stepping)) NN_BFAIL("batch state upload");
            prof_begin(ctx, KC_TRIAL, -1.0);
            trial(false, nullptr, 1);
            prof_end(ctx);
            if (!pull_res()) NN_BFAIL("batch read-back");
            for (int p = 0; p < P; p++) {
                if (!hb[p].active || cst[p] == C_DONE) continue;
                const double *r = &pres[(size_t)p * kBNV];
                const double n = nrow[p], nz = (double)K[p]->nnz;
                SP[p].spmvs++;
                SP[p].cauchy_trials++;
                SP[p].bytes_moved += 4.0 * (n + 1) + (ib + vb) * nz + 32.0 * n;
                const bool ok = ok_dec(p, r[0], r[1], r[2]);
                if (cst[p] == C_FIRST) {
                    if (ok) {
                        gs[p] = r[0], sks[p] = r[1], ss[p] = r[2];
                        cst[p] = C_EXT;
                    } else {
                        cst[p] = C_INT;
                        t[p] *= kInterp;
                    }
                } else if (cst[p] == C_EXT) {
                    if (!ok) {
                        cst[p] = C_DONE;
                    } else {
                        const bool same = r[0] == gs[p] && r[1] == sks[p];
                        t[p] *= kExtrap;
                        cur[p] ^= 1;
                        gs[p] = r[0], sks[p] = r[1], ss[p] = r[2];
                        // stop when every moving variable has reached its bound
                        if (same || ++nstep[p] >= 20) cst[p] = C_DONE;
                    }
                } else {
                    gs[p] = r[0], sks[p] = r[1], ss[p] = r[2];
                    if (ok) {
                        cst[p] = C_DONE;
                    } else if (++nstep[p] >= kMaxTrials || !(r[0] < 0.0)) {
                        // no decrease along -g at this precision: stationary up to rounding
                        status[p] = NN_EMAXIT;
                        hb[p].active = 0;
                        cst[p] = C_DONE;
                    } else {
                        t[p] *= kInterp;
                    }
                }
            }
        }
        if (err != NN_OK) break;
        if (!any_active()) break;
        for (int p = 0; p < P; p++) {
            hb[p].t = 0.0;
            if (!hb[p].active) continue;
            tcau[p] = t[p];
            hb[p].t = -t[p];
            hb[p].ksbuf = cur[p];
            SP[p].bytes_moved += 24.0 * nrow[p];
        }
        if (!push() || !select(is_active)) NN_BFAIL("batch state upload");
        apply(false);

        // ---- 3. Jacobi-PCG on every free face together
        if (mixed)
            hipLaunchKernelGGL((kb_cg_setup<float>), dim3(grid()), dim3(blk), 0, st, B, g, ks0,
                               ks1, mask, dm32, r32, z32, p32, q32, w32);
        else
            hipLaunchKernelGGL((kb_cg_setup<double>), dim3(grid()), dim3(blk), 0, st, B, g, ks0,
                               ks1, mask, dm64, r64, z64, p64, q64, w64);
        hipLaunchKernelGGL((kb_finalize<4, 1>), dim3(fgrid()), dim3(kFinBlock), 0, st, B,
                           opsc(OP_SUM, OP_SUM, OP_SUM, OP_SUM), o->inner_rtol * o->inner_rtol);
        if (!pull_state()) NN_BFAIL("batch read-back");
        for (int p = 0; p < P; p++) {
            it_before[p] = 0;
            if (hb[p].active) SP[p].bytes_moved += 88.0 * nrow[p];
        }
        auto running = [&](int p) { return hb[p].active != 0 && hb[p].done == 0; };
        for (int guard = 0; guard <= o->max_cg / chunk + 1; guard++) {
            if (!select(running)) NN_BFAIL("batch list upload");
            if (n_pr == 0) break;
            hipGraphExec_t ex = use_graph ? graph_for(n_sl) : nullptr;
            if (ex) {
                if (hipGraphLaunch(ex, st) != hipSuccess) NN_BFAIL("graph launch");
            } else {
                for (int k = 0; k < chunk; k++)
                    cg_iter(st, grid(), fgrid(), chunk_ev ? chunk_ev + (size_t)4 * k : nullptr);
            }
            if (!pull_state()) NN_BFAIL("batch read-back");
            // launch k of the chunk did work for the problems that ran more
            // than k iterations in it; byte model as in the single-problem
            // solver (mask, free-row values and indices, gathered and
            // streamed vectors)
            std::fill(b_spmv.begin(), b_spmv.end(), 0.0);
            std::fill(b_upd.begin(), b_upd.end(), 0.0);
            int ran_max = 0;
            for (int p = 0; p < P; p++) {
                if (!hb[p].active) continue;
                const int ran = hb[p].it - it_before[p];
                if (ran <= 0) continue;
                const double n = nrow[p], nf = hb[p].n_free, nzf = hb[p].nnz_free;
                const double bs = n + 4.0 * nf + (ib + vb) * nzf + 5.0 * vb * nf;
                const double bu = n + 8.0 * vb * nf;
                for (int k = 0; k < ran && k < chunk; k++) {
                    b_spmv[k] += bs;
                    b_upd[k] += bu;
                }
                SP[p].bytes_moved += ran * (bs + bu);
                ran_max = std::max(ran_max, ran);
                it_before[p] = hb[p].it;
            }
            if (chunk_ev) {
                for (int k = 0; k < ran_max && k < chunk; k++) {
                    float m1 = 0.f, m2 = 0.f;
                    if (hipEventElapsedTime(&m1, chunk_ev[4 * k], chunk_ev[4 * k + 1]) ==
                            hipSuccess &&
                        hipEventElapsedTime(&m2, chunk_ev[4 * k + 2], chunk_ev[4 * k + 3]) ==
                            hipSuccess) {
                        if ((ctx->prof_mask >> KC_CG_SPMV) & 1) prof_add(ctx, KC_CG_SPMV, m1, b_spmv[k]);
                        if ((ctx->prof_mask >> KC_CG_UPDATE) & 1) prof_add(ctx, KC_CG_UPDATE, m2, b_upd[k]);
                    }
                }
            }
        }
        if (err != NN_OK) break;
        for (int p = 0; p < P; p++) {
            if (!hb[p].active) continue;
            SP[p].cg_its += hb[p].it;
            SP[p].spmvs += hb[p].it;
            if (hb[p].done == 4) {
                status[p] = NN_ENONFINITE;
                hb[p].active = 0;
            } else if (hb[p].done == 3) {
                status[p] = NN_ENOTSPD;
                hb[p].active = 0;
            } else if (hb[p].done == 0) {
                status[p] = NN_EMAXIT;   // CG still running after the launch guard
                hb[p].active = 0;
            }
        }
        if (!any_active()) break;

        // ---- 4. projected searches along w (no matrix pass when no free
        // variable reaches its bound before the step)
        for (int p = 0; p < P; p++) hb[p].t = 0.0;
        if (!push() || !select(is_active)) NN_BFAIL("batch state upload");
        if (mixed)
            hipLaunchKernelGGL((kb_breakpoint<float>), dim3(grid()), dim3(blk), 0, st, B, w32, gptr);
        else
            hipLaunchKernelGGL((kb_breakpoint<double>), dim3(grid()), dim3(blk), 0, st, B, w64,
                               gptr);
        hipLaunchKernelGGL((kb_finalize<3, 0>), dim3(fgrid()), dim3(kFinBlock), 0, st, B,
                           opsc(OP_MIN, OP_SUM, OP_SUM), 0.0);
        if (!pull_res()) NN_BFAIL("batch read-back");
        for (int p = 0; p < P; p++) {
            sst[p] = 0;   // 0 no step, 1 searching, 2 step chosen
            if (!hb[p].active) continue;
            SP[p].bytes_moved += 24.0 * nrow[p];
            const double *r = &pres[(size_t)p * kBNV];
            bmin[p] = r[0];
            wn[p] = std::sqrt(r[2]);
            if (hb[p].it > 0 && r[1] < 0.0 && wn[p] > 0.0) {
                ts[p] = std::min(1.0, delta[p] / wn[p]);
                sst[p] = bmin[p] >= ts[p] ? 2 : 1;
                nstep[p] = 0;
            }
        }
        for (;;) {
            bool any = false;
            for (int p = 0; p < P; p++) {
                hb[p].t = 0.0;
                if (hb[p].active && sst[p] == 1) {
                    hb[p].t = ts[p];
                    any = true;
                }
            }
            if (!any) break;
            if (!push() || !select(stepping)) NN_BFAIL("batch state upload");
            prof_begin(ctx, KC_TRIAL, -1.0);
            trial(true, mask, 0);
            prof_end(ctx);
            if (!pull_res()) NN_BFAIL("batch read-back");
            for (int p = 0; p < P; p++) {
                if (!hb[p].active || sst[p] != 1) continue;
                const double *r = &pres[(size_t)p * kBNV];
                const double n = nrow[p], nz = (double)K[p]->nnz;
                SP[p].spmvs++;
                SP[p].search_trials++;
                SP[p].bytes_moved += 4.0 * (n + 1) + (ib + vb) * nz + 32.0 * n;
                if (r[0] < 0.0 && r[0] + 0.5 * r[1] <= kMu0 * r[0]) {
                    sst[p] = 2;
                } else {
                    ts[p] *= kBack;
                    if (ts[p] <= bmin[p]) {
                        ts[p] = bmin[p];   // no bound is crossed: decrease is guaranteed
                        sst[p] = 2;
                    } else if (++nstep[p] >= kMaxTrials) {
                        sst[p] = 2;
                    }
                }
            }
        }
        if (err != NN_OK) break;
        for (int p = 0; p < P; p++) {
            hb[p].t = 0.0;
            if (!hb[p].active) continue;
            double step = std::sqrt(ss[p]);
            if (sst[p] == 2 && ts[p] > 0.0) {
                hb[p].t = ts[p];
                step += ts[p] * wn[p];
                SP[p].bytes_moved += 24.0 * nrow[p];
            }
            // ---- 5. radius update (exact model: ratio one)
            if (std::isfinite(delta[p]) && step >= 0.99 * delta[p]) delta[p] *= 4.0;
            outer[p]++;
        }
        if (!push() || !select(stepping)) NN_BFAIL("batch state upload");
        if (n_pr > 0) apply(true);
        if (o->verbose) {
            int na = 0;
            for (int p = 0; p < P; p++) na += hb[p].active ? 1 : 0;
            std::fprintf(stderr,
                         "nnqp batch outer %3d: %d of %d problems iterating; member 0: kkt %.3e "
                         "free %.0f cauchy t %.3g cg %d breakpoint %.3g step %.3g\n",
                         it_outer, na, P, SP[0].kkt_rel, hb[0].n_free, tcau[0], hb[0].it, bmin[0],
                         sst[0] == 2 ? ts[0] : 0.0);
        }
    }
#undef NN_BFAIL
    // ---- outputs
    if (active) {
        const int64_t blocks = std::min<int64_t>((S + 3) / 4, (int64_t)num_cu * 8);
        hipLaunchKernelGGL(kb_active, dim3((int)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, B);
    }
    (void)hipEventRecord(t1, st);
    const hipError_t e = hipEventSynchronize(t1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    prof_collect(ctx);
    if (err != NN_OK) return err;
    if (e != hipSuccess) return fail(ctx, NN_EHIP, hipGetErrorString(e));
    int first_bad = -1;
    for (int p = 0; p < P; p++) {
        SP[p].seconds = ms * 1e-3;   // the whole batched call
        SP[p].status = status[p];
        if (status[p] != NN_OK && first_bad < 0) first_bad = p;
    }
    if (stats)
        for (int p = 0; p < P; p++) stats[p] = SP[p];
    if (first_bad >= 0) {
        char msg[160];
        std::snprintf(msg, sizeof(msg),
                      "batch member %d (the first affected) ended with status %d; every member's "
                      "status is in its stats",
                      first_bad, status[first_bad]);
        return fail(ctx, (nn_status)status[first_bad], msg);
    }
    ctx->err.clear();
    return NN_OK;
}

}  // namespace nnqp
