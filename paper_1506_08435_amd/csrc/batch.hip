// Batched solver: many independent non-negative QPs (Sec. 2.1.3, eq.
// non-negative) advanced together.
//
// Each member runs the single-problem method (the same steps, constants and
// tests: gradient and KKT test, Cauchy search, Jacobi-PCG on the free face,
// projected search, trust-region update), but the members do not move in
// lockstep: every member carries its own phase in a device-resident state
// machine, and one global step advances every member by one step of its own
// phase.  A global step is four launches over all members:
//
//   row pass     per slice, by the member's phase: gradient g = K c - f,
//                Cauchy trial along -g, CG matrix pass, or projected-search
//                trial along the CG step (one sliced-ELL pass each);
//   transition   one block per member: combine its slice partials, take the
//                decision the host takes in the single-problem solver
//                (convergence, trial accepted, CG step length) and choose
//                the member's vector operation;
//   vector pass  per slice, by that operation: Cauchy step with CG set-up,
//                CG vector update, breakpoint search, or step along w;
//   transition   combine the vector-pass partials (CG scalars, breakpoint),
//                choose the member's next phase.
//
// A member that needs many iterations therefore does not hold the others
// back: while it is in a long CG, the others run their own Cauchy searches,
// gradients and CGs in the same launches.  The host only replays chunks of
// global steps (captured once per size class as hipGraphs) and, between
// chunks, drops finished members from the device lists the launches walk.
//
// Layout: the members keep their own sliced-ELL matrices, reached through
// per-member pointer tables.  The batch numbers their 64-row slices
// consecutively (a slice never spans two members) and concatenates the work
// vectors over those slices, so global row s*64 + lane is local row
// (s - first slice of its member)*64 + lane.  Every reduction leaves one
// partial per slice, and a member's partials are combined by its own block
// in a fixed order: a member's arithmetic depends only on its own data, so
// its result is bitwise the same in any batch and for any launch shape.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "nnqp_internal.hpp"

// 1: chunks of global steps replayed as captured graphs; 0: launched one by one
#ifndef NNQP_BATCH_GRAPH
#define NNQP_BATCH_GRAPH 1
#endif

namespace nnqp {

namespace {

constexpr int kBNV = 5;          // values per slice partial
constexpr int kFinBlock = 256;   // threads of a transition block (one block per member)
constexpr double kMu0 = 0.01;    // sufficient-decrease constant
constexpr double kExtrap = 10.0; // Cauchy extrapolation factor
constexpr double kInterp = 0.1;  // Cauchy interpolation factor
constexpr double kBack = 0.5;    // projected-search backtracking factor
constexpr int kMaxTrials = 60;

// member phases: what the next row pass does for the member
enum : int {
    PH_DONE = 0,    // finished (status set)
    PH_GRAD = 1,    // gradient and convergence test
    PH_CAUCHY = 2,  // Cauchy search trial along -g
    PH_CG = 3,      // CG iteration
    PH_BREAK = 4,   // breakpoint of the step along w (vector pass only)
    PH_SEARCH = 5,  // projected-search trial along w
    PH_APPLYW = 6   // take the step along w (vector pass only)
};
// vector-pass operations chosen by the first transition
enum : int { VO_NONE = 0, VO_SETUP = 1, VO_UPDATE = 2, VO_BREAK = 3, VO_APPLYW = 4 };
// Cauchy search sub-states
enum : int { CS_FIRST = 0, CS_EXT = 1, CS_INT = 2 };

// Per-member state, in device memory (mirrored on the host between chunks).
struct BState {
    // control
    int phase, vop, status, outer;
    int cst, cur, ksbuf, ntrial;     // Cauchy sub-state, accepted K s buffer, trial buffer, trials
    int it, cgdone, nsearch, max_outer;
    int max_cg, pad0;
    double t, tcau, ttrial;          // accepted Cauchy step, its start value, signed trial step
    double gs, sks, ss;              // accepted Cauchy trial: g.s, s.Ks, s.s
    double delta, normf, tol, rtol2;
    double rz, rr_stop, alpha, beta, n_free, nnz_free;   // CG
    double bmin, wn, ts, stepn;      // projected search along w, step length of the iteration
    double n, nnz, ib, vb;           // rows, nonzeros, index and value bytes (byte model)
    // report
    double kkt_rel, kkt_nat, min_c, bytes;
    int n_active, cg_its, spmvs, cauchy_trials, search_trials, refinements, mixed, pad1;
};

// One entry of the current slice list with everything a pass needs before
// the member's phase: slice, member, first entry, and width << 7 | rows of the
// slice that exist.  Rebuilt on the device whenever the list changes, so a
// wavefront fetches its next slice with one load and no dependent lookups.
struct SRec {
    int s, p, off, wv;
};

struct BDev {
    int P, nslices;
    const int *cnt;                 // [2] slices and members in the current lists
    const int *plist;               // members taking part in the current launches
    const int *slist;               // their slices, member by member
    SRec *srec;                     // [cnt[0]] records of slist
    const int *sprob;               // [nslices] member of each slice
    const int *s0, *nrow;           // per member: first slice, rows
    const int *const *so;           // per member sliced-ELL offsets
    const int *const *sc;           // per member sliced-ELL columns (local)
    const short *const *sd;         // per member int16 offsets col - row (or null)
    const double *const *v64;       // per member float64 values
    const float *const *v32;        // per member float32 values (mixed precision)
    const double *const *diag;      // per member diagonal
    const int *const *rowptr;       // per member CSR row pointers
    double *const *c;               // per member solution vectors (local rows)
    const double *const *f;         // per member loads of the solve
    const double *const *f0;        // per member loads (transient step: f of f + M c/dt)
    const double *const *mv;        // per member capacity values (transient step)
    uint8_t *const *act_out;        // per member active-set outputs (entries may be null)
    BState *st;
    double *part;                   // [nslices][kBNV]
    double *pres;                   // [P][kBNV] (start-up reductions)
    // the batch as one block-diagonal sliced-ELL matrix and concatenated
    // vectors (global rows s*64 + lane), copied in at the start of a call
    const int *gso;                 // [nslices+1] first entry of each slice
    const int *gcol;                // global column of each entry
    const short *gd16;              // col - row (int16), or null
    const double *gv64;             // float64 values of the solve
    const float *gv32;              // float32 values (mixed precision), or null
    double *cg, *fg;                // solution and load
    const double *dg;               // diagonal of the solve's matrix (1 on rows past the end)
    const int *rlen;                // entries of each row (0 past the end)
    double lo, hi;                  // bounds lo <= c <= hi of every member
};

// Work vectors of the batched solve, concatenated over the slices.
template <class VV>
struct BVec {
    double *g, *ks0, *ks1;
    uint8_t *mask;
    VV *w, *r, *z, *p, *q, *dm;
};

__device__ __forceinline__ double bcomb(int op, double a, double b)
{
    return op == OP_SUM ? a + b : (op == OP_MIN ? fmin(a, b) : fmax(a, b));
}

__device__ __forceinline__ double bident(int op)
{
    return op == OP_SUM ? 0.0 : (op == OP_MIN ? INFINITY : -INFINITY);
}

// projection on [lo, hi]; NaN maps to lo (+0.0 for lo = 0)
__device__ __forceinline__ double projb(const BDev &B, double x)
{
    const double y = x > B.lo ? x : B.lo;
    return y < B.hi ? y : B.hi;
}

// Walk the slices of the current list grid-stride, one wavefront per slice.
// For a slice of a member with take(p): body(p, s, global row, local row, row
// exists, a); every listed slice then stores its wave-combined partials
// (identities when the member did not take part).
template <int NV, class Take, class Body>
__device__ __forceinline__ void for_bslices(const BDev &B, const int (&ops)[NV], Take take,
                                            Body body)
{
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
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
enum { CM_I32 = 0, CM_D16 = 2, CM_Q4 = 3, CM_P2 = 4 };

// Position of entry k of lane l in a slice of width w of the quad layout
// (CM_Q4), relative to the slice's first entry: entries 4j .. 4j+3 of a row
// side by side at 256 j + 4 l, two left over as a pair at 256 (w / 4) + 2 l,
// an odd last one in its column-major place 64 k + l.  A row of seven
// entries (2D P1) then takes three value loads and three offset loads
// instead of seven of each.
__host__ __device__ __forceinline__ int quad_pos(int k, int l, int w)
{
    const int nq = w >> 2, np = (w - 4 * nq) >> 1;
    if (k < 4 * nq) return 256 * (k >> 2) + 4 * l + (k & 3);
    if (k < 4 * nq + 2 * np) return 256 * nq + 2 * l + (k - 4 * nq);
    return 64 * k + l;
}

// The same for the paired layout (CM_P2): entries 2j, 2j+1 of a row side by
// side at 128 j + 2 l, an odd last one in its column-major place.
__host__ __device__ __forceinline__ int pair_pos(int k, int l, int w)
{
    const int np = w >> 1;
    if (k < 2 * np) return 128 * (k >> 1) + 2 * l + (k & 1);
    return 64 * k + l;
}

// Four (quad) or two (pair) consecutive values of the quad layout, with the
// same load hint as bld_val.
__device__ __forceinline__ void bld_quad(const double *p, double (&v)[4])
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
    const d2 b = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p + 2));
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}
__device__ __forceinline__ void bld_quad(const float *p, float (&v)[4])
{
    const float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
}
__device__ __forceinline__ void bld_pair(const double *p, double &a, double &b)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void bld_pair(const float *p, float &a, float &b)
{
    const float2 v = *reinterpret_cast<const float2 *>(p);
    a = v.x;
    b = v.y;
}

__device__ __forceinline__ double bld_val(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float bld_val(const float *p) { return *p; }

// Row sums of slice s of member p: sum_k val(k) x(col(k)), with the same
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

#ifndef NNQP_BATCH_FLAT8
#define NNQP_BATCH_FLAT8 1   // slices of width <= 8: every load of the row issued before any use
#endif

// The row sum of gsell_row_at for slices of width w <= 8 (2D P1 rows),
// written so that no load waits for another: every matrix load of the row is
// issued under wave-uniform guards that only move raw bits (no column is
// decoded inside a guard, which would make the compiler wait for that load
// there), then every gather is issued, then the products are added in entry
// order.  A slot past the row's entries keeps offset 0 (column i, a valid
// row) or column i, and value 0, and its product is not added (a select, so
// a non-finite x_i cannot leak in): the sum is bitwise the one of the
// guarded walk, entry by entry with fused multiply-adds.  On the 512-member
// batch the row pass went from 95 to 73 us (float64) and from 76 to 55 us
// (mixed): the guarded walk waited for every pair's offsets and for every
// gather in turn.
template <int CM, class VT, class X>
__device__ __forceinline__ double gsell_row8(const BDev &B, const VT *__restrict__ sv, int i,
                                             int off, int w, X x)
{
    const int lane = threadIdx.x & 63;
    const short *__restrict__ gd = B.gd16;
    double acc = 0.0;
    if constexpr (CM == CM_Q4) {
        // quads 0 and 1 (entries 0-7), the pair left over (two entries
        // after the quads), the odd last entry: the entry order
        const int nq = w >> 2, rem = w & 3;
        VT q[2][4];
        int2 dq[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            if (k < nq) {
                const int e = off + k * 4 * kSlice + 4 * lane;
                bld_quad(sv + e, q[k]);
                dq[k] = *reinterpret_cast<const int2 *>(gd + e);
            } else {
#pragma unroll
                for (int t = 0; t < 4; t++) q[k][t] = VT(0);
                dq[k] = make_int2(0, 0);
            }
        }
        VT pa = VT(0), pb = VT(0), so = VT(0);
        int dp = 0, dso = 0;
        if (rem >= 2) {
            const int e = off + nq * 4 * kSlice + 2 * lane;
            bld_pair(sv + e, pa, pb);
            dp = *reinterpret_cast<const int *>(gd + e);
        }
        if (rem & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            so = bld_val(sv + e);
            dso = gd[e];
        }
        double xv[11];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            xv[4 * k] = x(i + (int)(short)(dq[k].x & 0xffff));
            xv[4 * k + 1] = x(i + (dq[k].x >> 16));
            xv[4 * k + 2] = x(i + (int)(short)(dq[k].y & 0xffff));
            xv[4 * k + 3] = x(i + (dq[k].y >> 16));
        }
        xv[8] = x(i + (int)(short)(dp & 0xffff));
        xv[9] = x(i + (dp >> 16));
        xv[10] = x(i + dso);
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const double y = __builtin_fma((double)q[k][t], xv[4 * k + t], acc);
                acc = k < nq ? y : acc;
            }
        const double y8 = __builtin_fma((double)pa, xv[8], acc);
        acc = rem >= 2 ? y8 : acc;
        const double y9 = __builtin_fma((double)pb, xv[9], acc);
        acc = rem >= 2 ? y9 : acc;
        const double y10 = __builtin_fma((double)so, xv[10], acc);
        acc = (rem & 1) ? y10 : acc;
        return acc;
    } else if constexpr (CM == CM_P2) {
        // pairs 0-3 (entries 0-7), the odd last entry
        const int np = w >> 1;
        VT v[4][2];
        int d[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (k < np) {
                const int e = off + k * 2 * kSlice + 2 * lane;
                bld_pair(sv + e, v[k][0], v[k][1]);
                d[k] = *reinterpret_cast<const int *>(gd + e);
            } else {
                v[k][0] = v[k][1] = VT(0);
                d[k] = 0;
            }
        }
        VT so = VT(0);
        int dso = 0;
        if (w & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            so = bld_val(sv + e);
            dso = gd[e];
        }
        double xv[9];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            xv[2 * k] = x(i + (int)(short)(d[k] & 0xffff));
            xv[2 * k + 1] = x(i + (d[k] >> 16));
        }
        xv[8] = x(i + dso);
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int t = 0; t < 2; t++) {
                const double y = __builtin_fma((double)v[k][t], xv[2 * k + t], acc);
                acc = k < np ? y : acc;
            }
        const double y8 = __builtin_fma((double)so, xv[8], acc);
        acc = (w & 1) ? y8 : acc;
        return acc;
    } else {
        // column-major entries 0-7 (int32 global columns or int16 offsets)
        const int *__restrict__ gc = B.gcol;
        VT v[8];
        int cc[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (k < w) {
                const int e = off + k * kSlice + lane;
                v[k] = bld_val(sv + e);
                cc[k] = CM == CM_D16 ? (int)gd[e] : gc[e];
            } else {
                v[k] = VT(0);
                cc[k] = CM == CM_D16 ? 0 : i;
            }
        }
        double xv[8];
#pragma unroll
        for (int k = 0; k < 8; k++) xv[k] = x(CM == CM_D16 ? i + cc[k] : cc[k]);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const double y = __builtin_fma((double)v[k], xv[k], acc);
            acc = k < w ? y : acc;
        }
        return acc;
    }
}

// Row sums over the concatenated matrix for global row i = s*64 + lane of a
// slice whose first entry (off) and width (w) are known; global columns
// (int16 offsets from the row in CM_D16 mode).
template <int WMAX, int CM, class VT, class X>
__device__ __forceinline__ double gsell_row_at(const BDev &B, const VT *__restrict__ sv, int i,
                                               int off, int w, X x)
{
    if constexpr (WMAX == 8 && NNQP_BATCH_FLAT8) return gsell_row8<CM>(B, sv, i, off, w, x);
    const int lane = threadIdx.x & 63;
    const int *__restrict__ gc = B.gcol;
    const short *__restrict__ gd = B.gd16;
    auto col = [&](int e) {
        if (CM == CM_D16 || CM == CM_Q4 || CM == CM_P2) return i + (int)gd[e];
        return gc[e];
    };
    double acc = 0.0;
    if constexpr (CM == CM_P2) {
        // pairs in entry order, then the odd entry: the column-major sum order
        const int np = w >> 1;
        constexpr int HP = (WMAX < 8 ? WMAX : 8) / 2;   // pairs per load phase
#pragma unroll
        for (int h0 = 0; h0 < WMAX / 2; h0 += HP) {
            int cc[2 * HP];
            VT vv[2 * HP];
#pragma unroll
            for (int k = 0; k < HP; k++) {
                if (h0 + k < np) {
                    const int e = off + (h0 + k) * 2 * kSlice + 2 * lane;
                    bld_pair(sv + e, vv[2 * k], vv[2 * k + 1]);
                    const int d2 = *reinterpret_cast<const int *>(gd + e);
                    cc[2 * k] = i + (int)(short)(d2 & 0xffff);
                    cc[2 * k + 1] = i + (d2 >> 16);
                } else {
                    cc[2 * k] = cc[2 * k + 1] = 0;
                    vv[2 * k] = vv[2 * k + 1] = VT(0);
                }
            }
#pragma unroll
            for (int k = 0; k < 2 * HP; k++)
                if (h0 + k / 2 < np) acc += (double)vv[k] * x(cc[k]);
        }
        for (int k = WMAX / 2; k < np; k++) {   // slices wider than the unrolled part
            const int e = off + k * 2 * kSlice + 2 * lane;
            acc += (double)bld_val(sv + e) * x(col(e));
            acc += (double)bld_val(sv + e + 1) * x(col(e + 1));
        }
        if (w & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            acc += (double)bld_val(sv + e) * x(col(e));
        }
        return acc;
    }
    if constexpr (CM == CM_Q4) {
        // quads in entry order, then the left-over pair, then the odd entry:
        // the same sum order as the column-major walk
        const int nq = w >> 2, rem = w & 3;
        constexpr int HQ = (WMAX < 8 ? WMAX : 8) / 4;   // quads per load phase
#pragma unroll
        for (int h0 = 0; h0 < WMAX / 4; h0 += HQ) {
            int cc[4 * HQ];
            VT vv[4 * HQ];
#pragma unroll
            for (int k = 0; k < HQ; k++) {
                if (h0 + k < nq) {
                    const int e = off + (h0 + k) * 4 * kSlice + 4 * lane;
                    VT q[4];
                    bld_quad(sv + e, q);
                    const int2 d = *reinterpret_cast<const int2 *>(gd + e);
                    cc[4 * k] = i + (int)(short)(d.x & 0xffff);
                    cc[4 * k + 1] = i + (d.x >> 16);
                    cc[4 * k + 2] = i + (int)(short)(d.y & 0xffff);
                    cc[4 * k + 3] = i + (d.y >> 16);
#pragma unroll
                    for (int t = 0; t < 4; t++) vv[4 * k + t] = q[t];
                } else {
#pragma unroll
                    for (int t = 0; t < 4; t++) {
                        cc[4 * k + t] = 0;
                        vv[4 * k + t] = VT(0);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 4 * HQ; k++)
                if (h0 + k / 4 < nq) acc += (double)vv[k] * x(cc[k]);
        }
        for (int k = WMAX / 4; k < nq; k++) {   // slices wider than the unrolled part
            const int e = off + k * 4 * kSlice + 4 * lane;
#pragma unroll
            for (int t = 0; t < 4; t++) acc += (double)bld_val(sv + e + t) * x(col(e + t));
        }
        if (rem >= 2) {
            const int e = off + nq * 4 * kSlice + 2 * lane;
            VT a, b;
            bld_pair(sv + e, a, b);
            const int d2 = *reinterpret_cast<const int *>(gd + e);
            acc += (double)a * x(i + (int)(short)(d2 & 0xffff));
            acc += (double)b * x(i + (d2 >> 16));
        }
        if (rem & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            acc += (double)bld_val(sv + e) * x(col(e));
        }
        return acc;
    }
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

// The same for slice s, reading its first entry and width.
template <int WMAX, int CM, class VT, class X>
__device__ __forceinline__ double gsell_row(const BDev &B, const VT *__restrict__ sv, int s, int i,
                                            X x)
{
    const int off = B.gso[s];
    return gsell_row_at<WMAX, CM>(B, sv, i, off, (B.gso[s + 1] - off) >> 6, x);
}

__device__ __forceinline__ bool running(const BDev &B, int p) { return B.st[p].phase != PH_DONE; }

// Records of the current slice list (see SRec), one thread per entry.
__global__ void kb_recs(BDev B)
{
    const int nlist = B.cnt[0];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nlist; t += gridDim.x * blockDim.x) {
        const int s = B.slist[t];
        const int p = B.sprob[s];
        const int off = B.gso[s];
        const int w = (B.gso[s + 1] - off) >> 6;
        const int left = B.nrow[p] - (s - B.s0[p]) * kSlice;
        const int nv = left < 0 ? 0 : (left > kSlice ? kSlice : left);
        B.srec[t] = SRec{s, p, off, (w << 7) | nv};
    }
}

// Copy the members into the concatenated layout (every slice of the batch):
// c, f, diagonal and row lengths into the global vectors; slice offsets
// (ebase[p] + the member's own offset), global columns, int16 offsets and
// values into the global matrix arrays, in the quad layout when int16
// offsets are made (every member has them), else column-major.  Rows past a member's end get c = 0,
// f = 0, diagonal 1, length 0; their entries keep their valid columns.
__global__ void kb_gather(BDev B, const int64_t *__restrict__ ebase, int *__restrict__ gso,
                          int *__restrict__ gcol, short *__restrict__ gd16,
                          double *__restrict__ gv64, float *__restrict__ gv32,
                          double *__restrict__ dg, int *__restrict__ rlen, int copy_f, int layout)
{
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    for (int s = blockIdx.x * wpb + wid; s < B.nslices; s += nw) {
        const int p = B.sprob[s];
        const int ls = s - B.s0[p];
        const int il = ls * kSlice + lane, i = s * kSlice + lane;
        const int r0 = B.s0[p] * kSlice;
        const bool row = il < B.nrow[p];
        B.cg[i] = row ? B.c[p][il] : 0.0;
        if (copy_f) B.fg[i] = row ? B.f[p][il] : 0.0;
        dg[i] = row ? B.diag[p][il] : 1.0;
        rlen[i] = row ? B.rowptr[p][il + 1] - B.rowptr[p][il] : 0;
        const int *so = B.so[p];
        const int src = so[ls], w = (so[ls + 1] - src) >> 6;
        const int dst = (int)(ebase[p] + src);
        if (lane == 0) gso[s] = dst;
        const int *sc = B.sc[p];
        const short *sd = B.sd[p];
        const double *v64 = B.v64[p];
        const float *v32 = B.v32[p];
        for (int k = 0; k < w; k++) {
            const int es = src + k * kSlice + lane;
            const int ed = dst + (layout == CM_Q4   ? quad_pos(k, lane, w)
                                  : layout == CM_P2 ? pair_pos(k, lane, w)
                                                    : k * kSlice + lane);
            gcol[ed] = sc[es] + r0;
            if (gd16) gd16[ed] = sd[es];
            gv64[ed] = v64[es];
            if (gv32) gv32[ed] = v32[es];
        }
    }
}

// Copy the solution back to the members' vectors, and the active sets.
__global__ void kb_scatter(BDev B)
{
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    for (int s = blockIdx.x * wpb + wid; s < B.nslices; s += nw) {
        const int p = B.sprob[s];
        const int il = (s - B.s0[p]) * kSlice + lane;
        if (il >= B.nrow[p]) continue;
        const double cv = B.cg[s * kSlice + lane];
        B.c[p][il] = cv;
        uint8_t *out = B.act_out[p];
        if (out) out[il] = cv == B.lo ? 1 : (cv == B.hi ? 2 : 0);
    }
}

// ---------------------------------------------------------------- start-up kernels
// c = c0v (mode 0) or P(c) (mode 1); |f|^2, max f, #non-finite f, #non-finite c
__global__ void kb_init(BDev B, int mode, double c0v)
{
    const int ops[4] = {OP_SUM, OP_MAX, OP_SUM, OP_SUM};
    for_bslices<4>(B, ops, [&](int p) { return running(B, p); },
                   [&](int, int, int i, int, bool row, double (&a)[4]) {
                       if (!row) return;
                       const double fi = B.fg[i];
                       a[0] += fi * fi;
                       a[1] = fmax(a[1], fi);
                       a[2] += isfinite(fi) ? 0.0 : 1.0;
                       double *c = B.cg;
                       if (mode == 0) {
                           c[i] = c0v;
                       } else {
                           const double cv = c[i];
                           a[3] += isfinite(cv) ? 0.0 : 1.0;
                           c[i] = projb(B, cv);
                       }
                   });
}

// Right-hand side of a backward-Euler step, ft = f0 + (M c) / dt, written
// into the concatenated vector ft (the solve's loads point into it).
template <int WMAX>
__global__ void kb_transient_rhs(BDev B, double dt, double *__restrict__ ft)
{
    const int ops[1] = {OP_SUM};
    for_bslices<1>(B, ops, [&](int p) { return running(B, p); },
                   [&](int p, int s, int i, int il, bool row, double (&)[1]) {
                       const double *c = B.c[p];
                       const double mc =
                           bsell_row<WMAX, CM_I32>(B, B.mv[p], p, s, [&](int j) { return c[j]; });
                       if (row) ft[i] = B.f0[p][il] + mc / dt;
                       else ft[i] = 0.0;
                   });
}

// g = K c - f over the listed slices (the launch-shape tuner times this pass)
template <int WMAX, int CM>
__global__ void kb_grad(BDev B, double *__restrict__ g)
{
    const int ops[1] = {OP_SUM};
    for_bslices<1>(B, ops, [&](int p) { return running(B, p); },
                   [&](int, int s, int i, int, bool row, double (&a)[1]) {
                       const double *c = B.cg;
                       const double kc =
                           gsell_row<WMAX, CM>(B, B.gv64, s, i, [&](int j) { return c[j]; });
                       if (!row) return;
                       g[i] = kc - B.fg[i];
                       a[0] += g[i];
                   });
}

// Combine NV slice partials of member p in a fixed order (thread t takes
// slices t, t + 256, ...; then a wave butterfly; then the four waves in
// order).  Every thread of the block calls it; thread 0 gets true and the
// result, the others false.
template <int NV>
__device__ __forceinline__ bool member_reduce(const BDev &B, int p, const int (&ops)[NV],
                                              double (&a)[NV])
{
    __shared__ double sh[kFinBlock / 64][kBNV];
#pragma unroll
    for (int k = 0; k < NV; k++) a[k] = bident(ops[k]);
    const int s1 = B.s0[p] + (B.nrow[p] + kSlice - 1) / kSlice;
    for (int s = B.s0[p] + threadIdx.x; s < s1; s += kFinBlock)
#pragma unroll
        for (int k = 0; k < NV; k++) a[k] = bcomb(ops[k], a[k], B.part[(size_t)s * kBNV + k]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int k = 0; k < NV; k++) a[k] = bcomb(ops[k], a[k], __shfl_xor(a[k], o, 64));
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wid][k] = a[k];
    __syncthreads();
    if (threadIdx.x != 0) return false;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double v = sh[0][k];
        for (int w = 1; w < kFinBlock / 64; w++) v = bcomb(ops[k], v, sh[w][k]);
        a[k] = v;
    }
    return true;
}

// start-up reduction: |f|^2, max f, #non-finite f, #non-finite c into pres
__global__ __launch_bounds__(kFinBlock) void kb_reduce_init(BDev B)
{
    if ((int)blockIdx.x >= B.cnt[1]) return;
    const int p = B.plist[blockIdx.x];
    const int ops[4] = {OP_SUM, OP_MAX, OP_SUM, OP_SUM};
    double a[4];
    if (!member_reduce<4>(B, p, ops, a)) return;
    for (int k = 0; k < 4; k++) B.pres[(size_t)p * kBNV + k] = a[k];
}

// ---------------------------------------------------------------- global step
// Row pass: per listed slice, the matrix pass of the member's phase.
// (Compiled for eight waves per SIMD, i.e. at most 64 VGPRs, the 512-member
// batch's pass took 81 instead of 74 us in float64 and 70 instead of 55 us in
// mixed precision: the compiler then waits for loads earlier.)
//   GRAD    g = K c - f (float64 values); |pg|^2, #non-finite, ||min(c,g)||_inf,
//           min c, #(c == 0)
//   CAUCHY  s = P(c + ttrial g) - c gathered, ks = K s into buffer ksbuf;
//           g.s, s.Ks, s.s
//   CG      p <- z + beta p, q <- K z + beta q on the free rows; p.q
//   SEARCH  s = P(c + ts w) - c on the free rows, K s; g.s, s.Ks, s.s
template <int WMAX, int CM, class VT, class VV>
__global__ void kb_rows(BDev B, const VT *__restrict__ gvals, BVec<VV> V)
{
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    const int nlist = B.cnt[0];
    const double *__restrict__ c = B.cg;
    int k = blockIdx.x * wpb + wid;
    // Software pipeline over the wavefront's slices: the record of the slice
    // after next, and the phase, CG state and free-row mask of the next one,
    // are fetched while this slice works, so a slice starts with its matrix
    // loads.  (No pass of this kernel writes them.)
    SRec r1 = k < nlist ? B.srec[k] : SRec{0, 0, 0, 0};
    SRec r2 = k + nw < nlist ? B.srec[k + nw] : SRec{0, 0, 0, 0};
    int ph1 = k < nlist ? B.st[r1.p].phase : PH_DONE;
    int cd1 = k < nlist ? B.st[r1.p].cgdone : 1;
    uint8_t m1 = k < nlist ? V.mask[r1.s * kSlice + lane] : 0;
    for (; k < nlist; k += nw) {
        const SRec R = r1;
        const int ph = ph1;
        const int cgdone = cd1;
        const bool free_row = m1 != 0;
        if (k + nw < nlist) {
            r1 = r2;
            ph1 = B.st[r1.p].phase;
            cd1 = B.st[r1.p].cgdone;
            m1 = V.mask[r1.s * kSlice + lane];
            if (k + 2 * nw < nlist) r2 = B.srec[k + 2 * nw];
        }
        const int s = R.s;
        const int p = R.p;
        const int off = R.off, wsl = R.wv >> 7;   // first entry and width of the slice
        const BState &S = B.st[p];
        const int i = s * kSlice + lane;
        const bool row = lane < (R.wv & 127);
        double a[kBNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (ph == PH_GRAD) {
            a[2] = -INFINITY;
            a[3] = INFINITY;
            const double kc = gsell_row_at<WMAX, CM>(B, B.gv64, i, off, wsl, [&](int j) { return c[j]; });
            if (row) {
                const double gi = kc - B.fg[i];
                const double cv = c[i];
                V.g[i] = gi;
                const double pg = cv > B.lo ? (cv < B.hi ? gi : fmax(gi, 0.0)) : fmin(gi, 0.0);
                a[0] = pg * pg;
                a[1] = (isfinite(gi) && isfinite(cv)) ? 0.0 : 1.0;
                a[2] = fabs(fmax(cv - B.hi, fmin(gi, cv - B.lo)));
                a[3] = cv;
                a[4] = (cv == B.lo || cv == B.hi) ? 1.0 : 0.0;
            }
        } else if (ph == PH_CAUCHY) {
            const double t = S.ttrial;
            const double *__restrict__ g = V.g;
            auto sv = [&](int j) {
                const double cj = c[j];
                return projb(B, cj + t * g[j]) - cj;
            };
            const double ksv = gsell_row_at<WMAX, CM>(B, gvals, i, off, wsl, sv);
            if (row) {
                (S.ksbuf ? V.ks1 : V.ks0)[i] = ksv;
                const double si = sv(i);
                a[0] = g[i] * si;
                a[1] = si * ksv;
                a[2] = si * si;
            }
        } else if (ph == PH_CG) {
            const bool live = cgdone == 0 && row && free_row;
            if (__ballot(live) != 0) {
                const VV *__restrict__ z = V.z;
                // float64 vectors: the own-row values load before the gathers
                // (2 % faster on the 512-member batch; 5 % slower with
                // float32 vectors, which load them after)
                VV pold = VV(0), qold = VV(0), zi = VV(0);
                if constexpr (sizeof(VV) == 8) {
                    if (live) {
                        pold = V.p[i];
                        qold = V.q[i];
                        zi = z[i];
                    }
                }
                const double kz =
                    gsell_row_at<WMAX, CM>(B, gvals, i, off, wsl, [&](int j) { return (double)z[j]; });
                if (live) {
                    if constexpr (sizeof(VV) != 8) {
                        pold = V.p[i];
                        qold = V.q[i];
                        zi = z[i];
                    }
                    const double beta = S.beta;
                    const VV pi = (VV)fma(beta, (double)pold, (double)zi);
                    const VV qi = (VV)fma(beta, (double)qold, kz);
                    V.p[i] = pi;
                    V.q[i] = qi;
                    a[0] = (double)pi * (double)qi;
                }
            }
        } else if (ph == PH_SEARCH) {
            const bool live = row && free_row;
            if (__ballot(live) != 0) {
                const double t = S.ts;
                const VV *__restrict__ w = V.w;
                auto sv = [&](int j) {
                    const double cj = c[j];
                    return projb(B, cj + t * (double)w[j]) - cj;
                };
                const double ksv = gsell_row_at<WMAX, CM>(B, gvals, i, off, wsl, sv);
                if (live) {
                    const double si = sv(i);
                    a[0] = V.g[i] * si;
                    a[1] = si * ksv;
                    a[2] = si * si;
                }
            }
        } else {
            continue;   // no row work: the transition does not read these partials
        }
        // wave combination (the phase is uniform in the wave): only the
        // values the phase reports
        const int nv = ph == PH_GRAD ? 5 : (ph == PH_CG ? 1 : 3);
        if (nv == 1) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) a[0] += __shfl_xor(a[0], o, 64);
        } else if (nv == 3) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
                for (int v = 0; v < 3; v++) a[v] += __shfl_xor(a[v], o, 64);
        } else {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                a[0] += __shfl_xor(a[0], o, 64);
                a[1] += __shfl_xor(a[1], o, 64);
                a[2] = fmax(a[2], __shfl_xor(a[2], o, 64));
                a[3] = fmin(a[3], __shfl_xor(a[3], o, 64));
                a[4] += __shfl_xor(a[4], o, 64);
            }
        }
        if (lane == 0)
            for (int v = 0; v < nv; v++) B.part[(size_t)s * kBNV + v] = a[v];
    }
}

__device__ __forceinline__ void radius_update(BState &S)
{
    if (isfinite(S.delta) && S.stepn >= 0.99 * S.delta) S.delta *= 4.0;
}

// First transition: combine the row-pass partials of the member and decide.
__global__ __launch_bounds__(kFinBlock) void kb_step1(BDev B)
{
    if ((int)blockIdx.x >= B.cnt[1]) return;
    const int p = B.plist[blockIdx.x];
    BState &S = B.st[p];
    const int ph = S.phase;
    double a[kBNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (ph == PH_GRAD) {
        const int ops[5] = {OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM};
        if (!member_reduce<5>(B, p, ops, a)) return;
    } else if (ph == PH_CAUCHY || ph == PH_SEARCH) {
        const int ops[3] = {OP_SUM, OP_SUM, OP_SUM};
        double b[3];
        if (!member_reduce<3>(B, p, ops, b)) return;
        a[0] = b[0], a[1] = b[1], a[2] = b[2];
    } else if (ph == PH_CG) {
        const int ops[1] = {OP_SUM};
        double b[1];
        if (!member_reduce<1>(B, p, ops, b)) return;
        a[0] = b[0];
    } else if (threadIdx.x != 0) {
        return;
    }
    const double n = S.n, nnz = S.nnz;
    const double trial_bytes = 4.0 * (n + 1) + (S.ib + S.vb) * nnz + 32.0 * n;
    S.vop = VO_NONE;
    if (ph == PH_GRAD) {
        // gradient, KKT report, convergence test
        S.spmvs++;
        S.bytes += 4.0 * (n + 1) + (S.ib + 8.0) * nnz + 32.0 * n;
        if (a[1] != 0.0) {
            S.status = NN_ENONFINITE;
            S.phase = PH_DONE;
            return;
        }
        S.kkt_rel = sqrt(a[0]) / S.normf;
        S.kkt_nat = a[2];
        S.min_c = a[3];
        S.n_active = (int)a[4];
        if (S.mixed) S.refinements = S.outer + 1;
        if (S.kkt_rel <= S.tol) {
            S.status = NN_OK;
            S.phase = PH_DONE;
        } else if (S.outer >= S.max_outer) {
            S.status = NN_EMAXIT;
            S.phase = PH_DONE;
        } else {
            // Cauchy search from the previous step length
            S.cst = CS_FIRST;
            S.t = S.tcau;
            S.cur = 0;
            S.ntrial = 0;
            S.ttrial = -S.t;
            S.ksbuf = 0;
            S.phase = PH_CAUCHY;
        }
    } else if (ph == PH_CAUCHY) {
        S.spmvs++;
        S.cauchy_trials++;
        S.bytes += trial_bytes;
        const bool ok = a[0] < 0.0 && a[0] + 0.5 * a[1] <= kMu0 * a[0] && sqrt(a[2]) <= S.delta;
        bool accept = false;
        if (S.cst == CS_FIRST) {
            if (ok) {
                S.gs = a[0], S.sks = a[1], S.ss = a[2];
                S.cst = CS_EXT;
            } else {
                S.cst = CS_INT;
                S.t *= kInterp;
            }
        } else if (S.cst == CS_EXT) {
            if (!ok) {
                accept = true;
            } else {
                const bool same = a[0] == S.gs && a[1] == S.sks;
                S.t *= kExtrap;
                S.cur ^= 1;
                S.gs = a[0], S.sks = a[1], S.ss = a[2];
                // stop when every moving variable has reached its bound
                if (same || ++S.ntrial >= 20) accept = true;
            }
        } else {
            S.gs = a[0], S.sks = a[1], S.ss = a[2];
            if (ok) {
                accept = true;
            } else if (++S.ntrial >= kMaxTrials || !(a[0] < 0.0)) {
                // no decrease along -g at this precision: stationary up to rounding
                S.status = NN_EMAXIT;
                S.phase = PH_DONE;
                return;
            } else {
                S.t *= kInterp;
            }
        }
        if (accept) {
            S.tcau = S.t;
            S.stepn = sqrt(S.ss);
            S.vop = VO_SETUP;   // Cauchy step and CG set-up in the vector pass
            S.phase = PH_CG;
        } else if (S.cst == CS_EXT) {
            S.ttrial = -S.t * kExtrap;
            S.ksbuf = S.cur ^ 1;
        } else {
            S.ttrial = -S.t;
            S.ksbuf = S.cur;
        }
    } else if (ph == PH_CG) {
        // alpha = r.z / p.q; breakdown on non-positive or non-finite curvature
        const double pq = a[0];
        if (S.cgdone != 0) {
            S.phase = PH_BREAK;
        } else if (!isfinite(pq)) {
            S.status = NN_ENONFINITE;
            S.phase = PH_DONE;
        } else if (!(pq > 0.0)) {
            S.status = NN_ENOTSPD;
            S.phase = PH_DONE;
        } else {
            S.alpha = S.rz / pq;
            S.vop = VO_UPDATE;
        }
    } else if (ph == PH_SEARCH) {
        S.spmvs++;
        S.search_trials++;
        S.bytes += trial_bytes;
        bool accept = false;
        if (a[0] < 0.0 && a[0] + 0.5 * a[1] <= kMu0 * a[0]) {
            accept = true;
        } else {
            S.ts *= kBack;
            if (S.ts <= S.bmin) {
                S.ts = S.bmin;   // no bound is crossed: decrease is guaranteed
                accept = true;
            } else if (++S.nsearch >= kMaxTrials) {
                accept = true;
            }
        }
        if (accept) {
            S.vop = VO_APPLYW;
            S.phase = PH_APPLYW;
        }
    } else if (ph == PH_BREAK) {
        S.vop = VO_BREAK;
    } else if (ph == PH_APPLYW) {
        S.vop = VO_APPLYW;
    }
}

// Vector pass: per listed slice, the operation the first transition chose.
//   SETUP   c = P(c - t g), g += K s (accepted Cauchy trial); free = not
//           (c == 0 and g >= 0); dm = 1/diag, r = -g on free rows; z = dm r;
//           p = q = w = 0; r.z, r.r, #free, nnz of the free rows
//   UPDATE  w += alpha p, r -= alpha q, z = dm r on free rows; r.z, r.r
//   BREAK   min over w < 0 of c/(-w), g.w, w.w
//   APPLYW  c = P(c + ts w)
template <class VV>
__global__ void kb_vec(BDev B, BVec<VV> V)
{
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int nw = gridDim.x * wpb;
    const int nlist = B.cnt[0];
    int k = blockIdx.x * wpb + wid;
    // the same pipeline over the slice records as the row pass; the mask of
    // the next slice is read ahead too (only a set-up writes a mask, and only
    // its own slice's, which it does not read)
    SRec r1 = k < nlist ? B.srec[k] : SRec{0, 0, 0, 0};
    SRec r2 = k + nw < nlist ? B.srec[k + nw] : SRec{0, 0, 0, 0};
    int op1 = k < nlist ? B.st[r1.p].vop : VO_NONE;
    uint8_t m1 = k < nlist ? V.mask[r1.s * kSlice + lane] : 0;
    for (; k < nlist; k += nw) {
        const SRec R = r1;
        const int vop = op1;
        const bool free_row = m1 != 0;
        if (k + nw < nlist) {
            r1 = r2;
            op1 = B.st[r1.p].vop;
            m1 = V.mask[r1.s * kSlice + lane];
            if (k + 2 * nw < nlist) r2 = B.srec[k + 2 * nw];
        }
        if (vop == VO_NONE) continue;
        const int s = R.s;
        const BState &S = B.st[R.p];
        const int i = s * kSlice + lane;
        const bool row = lane < (R.wv & 127);
        double *__restrict__ c = B.cg;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        if (vop == VO_SETUP) {
            if (!row) {
                V.mask[i] = 0;
                V.dm[i] = V.r[i] = V.z[i] = V.p[i] = V.q[i] = V.w[i] = VV(0);
            } else {
                const double gi0 = V.g[i];
                const double cv = projb(B, c[i] - S.t * gi0);
                const double gi = gi0 + (S.cur ? V.ks1 : V.ks0)[i];
                c[i] = cv;
                V.g[i] = gi;
                const bool fr = !((cv == B.lo && gi >= 0.0) || (cv == B.hi && gi <= 0.0));
                const VV dmi = fr ? (VV)(1.0 / B.dg[i]) : VV(0);
                const VV ri = fr ? (VV)(-gi) : VV(0);
                const VV zi = dmi * ri;
                V.mask[i] = fr ? 1 : 0;
                V.dm[i] = dmi;
                V.r[i] = ri;
                V.z[i] = zi;
                V.p[i] = VV(0);
                V.q[i] = VV(0);
                V.w[i] = VV(0);
                a[0] = (double)ri * (double)zi;
                a[1] = (double)ri * (double)ri;
                a[2] = fr ? 1.0 : 0.0;
                a[3] = fr ? (double)B.rlen[i] : 0.0;
            }
        } else if (vop == VO_UPDATE) {
            if (row && free_row) {
                const double alpha = S.alpha;
                const VV ri = (VV)((double)V.r[i] - alpha * (double)V.q[i]);
                const VV zi = V.dm[i] * ri;
                V.w[i] = (VV)((double)V.w[i] + alpha * (double)V.p[i]);
                V.r[i] = ri;
                V.z[i] = zi;
                a[0] = (double)ri * (double)zi;
                a[1] = (double)ri * (double)ri;
            }
        } else if (vop == VO_BREAK) {
            a[0] = INFINITY;
            if (row) {
                const double wi = (double)V.w[i];
                if (wi < 0.0) a[0] = (c[i] - B.lo) / (-wi);
                else if (wi > 0.0) a[0] = (B.hi - c[i]) / wi;
                a[1] = V.g[i] * wi;
                a[2] = wi * wi;
            }
        } else {   // VO_APPLYW
            if (row) c[i] = projb(B, c[i] + S.ts * (double)V.w[i]);
            continue;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const double other = __shfl_xor(a[v], o, 64);
                a[v] = (vop == VO_BREAK && v == 0) ? fmin(a[v], other) : a[v] + other;
            }
        }
        if (lane == 0)
#pragma unroll
            for (int v = 0; v < 4; v++) B.part[(size_t)s * kBNV + v] = a[v];
    }
}

// Second transition: combine the vector-pass partials and choose the phase
// of the member's next global step.
__global__ __launch_bounds__(kFinBlock) void kb_step2(BDev B)
{
    if ((int)blockIdx.x >= B.cnt[1]) return;
    const int p = B.plist[blockIdx.x];
    BState &S = B.st[p];
    const int vop = S.vop;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (vop == VO_SETUP) {
        const int ops[4] = {OP_SUM, OP_SUM, OP_SUM, OP_SUM};
        if (!member_reduce<4>(B, p, ops, a)) return;
    } else if (vop == VO_UPDATE) {
        const int ops[2] = {OP_SUM, OP_SUM};
        double b[2];
        if (!member_reduce<2>(B, p, ops, b)) return;
        a[0] = b[0], a[1] = b[1];
    } else if (vop == VO_BREAK) {
        const int ops[3] = {OP_MIN, OP_SUM, OP_SUM};
        double b[3];
        if (!member_reduce<3>(B, p, ops, b)) return;
        a[0] = b[0], a[1] = b[1], a[2] = b[2];
    } else if (threadIdx.x != 0) {
        return;
    }
    const double n = S.n;
    if (vop == VO_SETUP) {
        // CG start on the free face: stop before the first iteration when the
        // face is empty or the residual vanishes
        S.bytes += 24.0 * n + 88.0 * n;
        S.rz = a[0];
        S.rr_stop = S.rtol2 * a[1];
        S.n_free = a[2];
        S.nnz_free = a[3];
        S.beta = 0.0;
        S.alpha = 0.0;
        S.it = 0;
        if (!isfinite(a[0]) || !isfinite(a[1])) {
            S.status = NN_ENONFINITE;
            S.phase = PH_DONE;
        } else if (a[1] == 0.0 || a[2] == 0.0 || S.max_cg <= 0 || !(a[0] > 0.0)) {
            S.cgdone = 1;
            S.phase = PH_BREAK;
        } else {
            S.cgdone = 0;
            S.phase = PH_CG;
        }
    } else if (vop == VO_UPDATE) {
        // iteration done: beta for the next one, stopping test on r.r
        const double rz = a[0], rr = a[1];
        const double nf = S.n_free, nzf = S.nnz_free;
        S.bytes += n + 4.0 * nf + (S.ib + S.vb) * nzf + 5.0 * S.vb * nf + n + 8.0 * S.vb * nf;
        S.it += 1;
        S.cg_its++;
        S.spmvs++;
        S.beta = rz / S.rz;
        S.rz = rz;
        if (!isfinite(rz) || !isfinite(rr)) {
            S.status = NN_ENONFINITE;
            S.phase = PH_DONE;
        } else if (rr <= S.rr_stop || S.it >= S.max_cg || !(rz > 0.0)) {
            S.cgdone = 1;
            S.phase = PH_BREAK;
        }
    } else if (vop == VO_BREAK) {
        S.bytes += 24.0 * n;
        S.bmin = a[0];
        S.wn = sqrt(a[2]);
        if (S.it > 0 && a[1] < 0.0 && S.wn > 0.0) {
            S.ts = fmin(1.0, S.delta / S.wn);
            S.nsearch = 0;
            S.phase = S.bmin >= S.ts ? PH_APPLYW : PH_SEARCH;
        } else {
            // no step along w: radius update on the Cauchy step, next iteration
            radius_update(S);
            S.outer++;
            S.phase = PH_GRAD;
        }
    } else if (vop == VO_APPLYW) {
        S.bytes += 24.0 * n;
        S.stepn += S.ts * S.wn;
        radius_update(S);
        S.outer++;
        S.phase = PH_GRAD;
    }
    S.vop = VO_NONE;
}

// ---------------------------------------------------------------- host side
struct Shape {
    int block = 256;   // threads per block
    int per_cu = 8;    // blocks per CU (the grid is capped by the slice count)
};

// size class -> tuned shape (per process; the class is (log2 rows, widest
// slice class, precision)).  Contexts on different threads share it, so every
// access holds shape_mutex(); the launch shape changes no arithmetic.
std::map<std::tuple<int, int, int>, Shape> &shape_cache()
{
    static std::map<std::tuple<int, int, int>, Shape> m;
    return m;
}

std::mutex &shape_mutex()
{
    static std::mutex mu;
    return mu;
}

int width_class(int wmax) { return wmax <= 8 ? 8 : (wmax <= 16 ? 16 : 32); }

// The same with the kernel's own begin and end recorded into e0, e1 when
// they are not null (hipExtLaunchKernelGGL).
#ifndef NNQP_BATCH_PAIRS
#define NNQP_BATCH_PAIRS 1   // float64 batches read the concatenated matrix in pairs
#endif

#define NN_BLAUNCH_EV(KERNEL, grid, block, stream, e0, e1, ...)                                 \
    do {                                                                                        \
        if (e0)                                                                                 \
            hipExtLaunchKernelGGL(KERNEL, dim3(grid), dim3(block), 0, stream, e0, e1, 0,         \
                                  __VA_ARGS__);                                                 \
        else                                                                                    \
            hipLaunchKernelGGL(KERNEL, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);        \
    } while (0)
#define NN_BDISPATCH_EV(wmax, KERNEL, grid, block, stream, e0, e1, ...)                         \
    do {                                                                                        \
        if ((wmax) <= 8) {                                                                      \
            constexpr int WM = 8;                                                               \
            NN_BLAUNCH_EV(KERNEL, grid, block, stream, e0, e1, __VA_ARGS__);                    \
        } else if ((wmax) <= 16) {                                                              \
            constexpr int WM = 16;                                                              \
            NN_BLAUNCH_EV(KERNEL, grid, block, stream, e0, e1, __VA_ARGS__);                    \
        } else {                                                                                \
            constexpr int WM = 32;                                                              \
            NN_BLAUNCH_EV(KERNEL, grid, block, stream, e0, e1, __VA_ARGS__);                    \
        }                                                                                       \
    } while (0)

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
    const DevAlloc &al;   // the context's device memory hooks
    std::vector<void *> dev, host;
    bool ok = true;
    explicit Arena(const DevAlloc &a) : al(a) {}
    template <class T>
    T *d(size_t n)
    {
        void *p = nullptr;
        if (dev_malloc(al, &p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
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
        for (void *p : dev) dev_free(al, p);
        for (void *p : host) (void)hipHostFree(p);
    }
};

// Captured chunks of global steps, one per launch-size class (the grid of a
// captured launch is fixed; the lists it walks are read from device memory).
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

// Algorithmic bytes of the row pass of one member in its current state (the
// same byte model as the member's own transitions).
double row_bytes(const BState &S)
{
    const double n = S.n, nnz = S.nnz;
    switch (S.phase) {
    case PH_GRAD:
        return 4.0 * (n + 1) + (S.ib + 8.0) * nnz + 32.0 * n;
    case PH_CAUCHY:
    case PH_SEARCH:
        return 4.0 * (n + 1) + (S.ib + S.vb) * nnz + 32.0 * n;
    case PH_CG:
        return S.cgdone ? 0.0
                        : n + 4.0 * S.n_free + (S.ib + S.vb) * S.nnz_free + 5.0 * S.vb * S.n_free;
    default:
        return 0.0;
    }
}

// The same under the paper's CSR model (4-byte column indices; the CG
// matrix pass as a masked SpMV plus a separate direction update).
double row_bytes_csr(const BState &S)
{
    const double n = S.n, nnz = S.nnz;
    switch (S.phase) {
    case PH_GRAD:
        return 4.0 * (n + 1) + 12.0 * nnz + 32.0 * n;
    case PH_CAUCHY:
    case PH_SEARCH:
        return 4.0 * (n + 1) + (4.0 + S.vb) * nnz + 32.0 * n;
    case PH_CG:
        return S.cgdone ? 0.0
                        : (4.0 + S.vb) * S.nnz_free + (4.0 + 6.0 * S.vb) * S.n_free;
    default:
        return 0.0;
    }
}

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
            if (dev_malloc(K[p]->al, &K[p]->val32, sizeof(float) * std::max<int64_t>(K[p]->nsell, 1)) !=
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
    const double vb = mixed ? 4.0 : 8.0;                // bytes per CG vector entry and per value
    // Mixed precision reads the concatenated matrix in the quad layout (int16
    // offsets, four float32 values per load): on the 512-member batch the row
    // pass takes 67 instead of 107 us.  Float64 reads it in pairs (int16
    // offset pairs, one 16-byte load per value pair): 95-97 instead of
    // 90-106 us (its quad layout was no faster, column-major int16 offsets
    // slower).
    const bool quad = mixed && all_d16;
    const bool pair = !mixed && all_d16 && NNQP_BATCH_PAIRS;
    const int layout = quad ? CM_Q4 : (pair ? CM_P2 : CM_I32);
    const double ib = quad || pair ? 2.0 : 4.0;   // bytes per column index

    // ---- tables, work vectors, lists, pinned state mirrors
    Arena A(ctx->al);
    int *d_sprob = A.d<int>(S), *d_s0 = A.d<int>(P), *d_nrow = A.d<int>(P);
    int *d_list = A.d<int>((size_t)2 + P + S);
    SRec *d_srec = A.d<SRec>(S);
    const int **d_so = A.d<const int *>(P), **d_sc = A.d<const int *>(P),
              **d_rp = A.d<const int *>(P);
    const short **d_sd = A.d<const short *>(P);
    const double **d_v64 = A.d<const double *>(P), **d_diag = A.d<const double *>(P),
                 **d_f = A.d<const double *>(P), **d_f0 = A.d<const double *>(P),
                 **d_mv = A.d<const double *>(P);
    const float **d_v32 = A.d<const float *>(P);
    double **d_c = A.d<double *>(P);
    uint8_t **d_act = A.d<uint8_t *>(P);
    BState *d_st = A.d<BState>(P);
    double *d_part = A.d<double>((size_t)S * kBNV), *d_pres = A.d<double>((size_t)P * kBNV);
    double *g = A.d<double>(R), *ks0 = A.d<double>(R), *ks1 = A.d<double>(R);
    uint8_t *mask = A.d<uint8_t>(R);
    // concatenated layout: vectors and the block-diagonal matrix
    std::vector<int64_t> ebase(P);
    int64_t E = 0;
    for (int p = 0; p < P; p++) {
        ebase[p] = E;
        E += K[p]->n > 0 ? K[p]->nsell : 0;
    }
    if (E >= (int64_t)1 << 31) return fail(ctx, NN_EINVAL, "batch too large: sliced-ELL entries must stay below 2^31");
    double *cg = A.d<double>(R), *fg = A.d<double>(R), *dg = A.d<double>(R);
    int *rlen = A.d<int>(R);
    double *ft = fg;   // a transient step's loads f + M c/dt are formed in place
    int *gso = A.d<int>(S + 1), *gcol = A.d<int>(E);
    int64_t *d_ebase = A.d<int64_t>(P);
    double *gv64 = A.d<double>(E);
    float *gv32 = mixed ? A.d<float>(E) : nullptr;
    short *gd16 = quad || pair ? A.d<short>(E) : nullptr;
    BVec<double> V64{g, ks0, ks1, mask, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    BVec<float> V32{g, ks0, ks1, mask, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (mixed) {
        V32.w = A.d<float>(R), V32.r = A.d<float>(R), V32.z = A.d<float>(R);
        V32.p = A.d<float>(R), V32.q = A.d<float>(R), V32.dm = A.d<float>(R);
    } else {
        V64.w = A.d<double>(R), V64.r = A.d<double>(R), V64.z = A.d<double>(R);
        V64.p = A.d<double>(R), V64.q = A.d<double>(R), V64.dm = A.d<double>(R);
    }
    BState *hs = A.h<BState>(P);
    double *pres = A.h<double>((size_t)P * kBNV);
    const void **tab = (const void **)A.h<void *>((size_t)P * 12);
    // Uploads from pinned memory read their source when they execute, so
    // the host writes each upload into a staging copy that it does not touch
    // again until the copy's event has completed.
    constexpr int kStage = 4;
    BState *st_stage[kStage];
    int *lst_stage[kStage];
    for (int k = 0; k < kStage; k++) {
        st_stage[k] = A.h<BState>(P);
        lst_stage[k] = A.h<int>((size_t)2 + P + S);
    }
    if (!A.ok) return fail(ctx, NN_EOOM, "batch workspace allocation failed");
    Events ev_st, ev_lst, ev_t;
    if (!ev_st.create(kStage, hipEventDisableTiming) ||
        !ev_lst.create(kStage, hipEventDisableTiming) || !ev_t.create(2, hipEventDefault))
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
        NN_HIP_TRY(ctx, hipMemcpyAsync(d_ebase, ebase.data(), sizeof(int64_t) * P,
                                       hipMemcpyHostToDevice, st));
        const int e_total = (int)E;
        NN_HIP_TRY(ctx, hipMemcpyAsync(gso + S, &e_total, sizeof(int), hipMemcpyHostToDevice, st));
        // the pageable sources above must stay alive until the copies finish
        NN_HIP_TRY(ctx, hipStreamSynchronize(st));
    }
    BDev B;
    B.P = P;
    B.nslices = (int)S;
    B.cnt = d_list;
    B.plist = d_list + 2;
    B.slist = d_list + 2 + P;
    B.srec = d_srec;
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
    B.st = d_st;
    B.part = d_part;
    B.pres = d_pres;
    B.gso = gso;
    B.gcol = gcol;
    B.gd16 = gd16;
    B.gv64 = gv64;
    B.gv32 = gv32;
    B.cg = cg;
    B.fg = fg;
    B.dg = dg;
    B.rlen = rlen;
    B.lo = o->lower;
    B.hi = o->upper;

    // ---- member states
    std::memset(hs, 0, sizeof(BState) * P);
    for (int p = 0; p < P; p++) {
        BState &M = hs[p];
        M.phase = nrow[p] > 0 ? PH_GRAD : PH_DONE;
        M.status = NN_OK;
        M.max_outer = o->max_outer;
        M.max_cg = o->max_cg;
        M.tcau = 1.0;
        M.delta = o->delta0 > 0.0 ? o->delta0 : INFINITY;
        M.tol = o->tol;
        M.rtol2 = o->inner_rtol * o->inner_rtol;
        M.n = (double)nrow[p];
        M.nnz = (double)K[p]->nnz;
        M.ib = ib;
        M.vb = vb;
        M.mixed = mixed ? 1 : 0;
    }
    int st_next = 0, lst_next = 0;
    auto push = [&]() {
        const int k = st_next;
        st_next = (st_next + 1) % kStage;
        if (hipEventSynchronize(ev_st.ev[k]) != hipSuccess) return false;
        std::memcpy(st_stage[k], hs, sizeof(BState) * P);
        return hipMemcpyAsync(d_st, st_stage[k], sizeof(BState) * P, hipMemcpyHostToDevice, st) ==
                   hipSuccess &&
               hipEventRecord(ev_st.ev[k], st) == hipSuccess;
    };
    auto pull = [&]() {
        return hipMemcpyAsync(hs, d_st, sizeof(BState) * P, hipMemcpyDeviceToHost, st) ==
                   hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    // The members still running, and their slices, as device lists: rebuilt
    // and uploaded only when the set changes.
    std::vector<char> sel(P, 0), sel_cur(P, 2);
    int n_sl = 0, n_pr = 0;
    // The slice records read the concatenated layout's slice offsets (gso),
    // which kb_gather writes: they are built once it has run, and again
    // whenever the list changes after that.
    bool layout_ready = false;
    auto build_recs = [&]() -> bool {
        hipLaunchKernelGGL(kb_recs, dim3((unsigned)std::max(1, (n_sl + 255) / 256)), dim3(256), 0, st,
                           B);
        return hipGetLastError() == hipSuccess;
    };
    auto select = [&]() -> bool {
        bool same = true;
        for (int p = 0; p < P; p++) {
            sel[p] = hs[p].phase != PH_DONE ? 1 : 0;
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
        if (hipMemcpyAsync(d_list, h, sizeof(int) * ((size_t)2 + P + ns), hipMemcpyHostToDevice,
                           st) != hipSuccess ||
            hipEventRecord(ev_lst.ev[k], st) != hipSuccess)
            return false;
        return !layout_ready || build_recs();
    };

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
    NN_HIP_TRY(ctx, select() ? hipSuccess : hipErrorUnknown);
    NN_HIP_TRY(ctx, hipEventRecord(t0, st));

    // ---- transient right-hand sides (from c^n, before the start point is set)
    if (transient)
        NN_BDISPATCH(wmax, (kb_transient_rhs<WM>), grid_for(sh, n_sl), sh.block, st, B, dt, ft);
    // ---- the members into the concatenated layout
    {
        const int64_t blocks = std::min<int64_t>((S + 3) / 4, (int64_t)num_cu * 8);
        hipLaunchKernelGGL(kb_gather, dim3((int)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, B,
                           (const int64_t *)d_ebase, gso, gcol, gd16, gv64, gv32, dg, rlen,
                           transient ? 0 : 1, layout);
        layout_ready = true;
        NN_HIP_TRY(ctx, build_recs() ? hipSuccess : hipErrorUnknown);
    }
    // ---- start point and load statistics
    hipLaunchKernelGGL(kb_init, dim3(grid_for(sh, n_sl)), dim3(sh.block), 0, st, B,
                       o->c0_mode == 1 ? 1 : 0, std::min(std::max(o->c0_value, o->lower), o->upper));
    hipLaunchKernelGGL(kb_reduce_init, dim3(std::max(n_pr, 1)), dim3(kFinBlock), 0, st, B);
    NN_HIP_TRY(ctx, hipMemcpyAsync(pres, d_pres, sizeof(double) * P * kBNV, hipMemcpyDeviceToHost,
                                   st));
    NN_HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int p = 0; p < P; p++) {
        BState &M = hs[p];
        if (M.phase == PH_DONE) continue;
        const double *r = &pres[(size_t)p * kBNV];
        M.normf = std::sqrt(r[0]);
        M.bytes += 16.0 * nrow[p];
        if (r[2] != 0.0 || r[3] != 0.0) {
            M.status = NN_ENONFINITE;
            M.phase = PH_DONE;
        } else if (o->lower == 0.0 && !(r[1] > 0.0)) {
            // f <= 0 with lower bound 0: c = 0 satisfies c >= 0, g = -f >= 0, c.g = 0
            NN_HIP_TRY(ctx, hipMemsetAsync(cg + (size_t)s0[p] * kSlice, 0,
                                           sizeof(double) * nrow[p], st));
            M.n_active = nrow[p];
            M.phase = PH_DONE;
        }
    }
    NN_HIP_TRY(ctx, push() ? hipSuccess : hipErrorUnknown);
    NN_HIP_TRY(ctx, select() ? hipSuccess : hipErrorUnknown);

    // ---- launch shape for this size class
    const auto key = std::make_tuple((int)std::log2((double)R), width_class(wmax), (int)mixed);
    auto &cache = shape_cache();
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(shape_mutex());
        auto it = cache.find(key);
        if (it != cache.end()) {
            sh = it->second;
            cached = true;
        }
    }
    if (!cached && n_pr > 0) {
        // time the gradient pass over all running members for each candidate
        // shape; it writes only g and the slice partials, which the first
        // global step overwrites
        float best = INFINITY;
        Shape pick = sh;
        for (int blk : {256, 512, 1024})
            for (int per_cu : {2, 4, 8}) {
                if (blk * per_cu > 4096) continue;
                const Shape cand{blk, per_cu};
                const int gsz = grid_for(cand, n_sl);
                if (quad) NN_BDISPATCH(wmax, (kb_grad<WM, CM_Q4>), gsz, blk, st, B, g);   // warm-up
                else if (pair) NN_BDISPATCH(wmax, (kb_grad<WM, CM_P2>), gsz, blk, st, B, g);
                else NN_BDISPATCH(wmax, (kb_grad<WM, CM_I32>), gsz, blk, st, B, g);
                NN_HIP_TRY(ctx, hipEventRecord(t0, st));
                for (int rep = 0; rep < 3; rep++)
                    if (quad) NN_BDISPATCH(wmax, (kb_grad<WM, CM_Q4>), gsz, blk, st, B, g);
                    else if (pair) NN_BDISPATCH(wmax, (kb_grad<WM, CM_P2>), gsz, blk, st, B, g);
                    else NN_BDISPATCH(wmax, (kb_grad<WM, CM_I32>), gsz, blk, st, B, g);
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
        {
            std::lock_guard<std::mutex> lk(shape_mutex());
            cache[key] = sh;
        }
        if (o->verbose)
            std::fprintf(stderr,
                         "nnqp batch shape: %lld rows, slice width %d -> %d threads, %d blocks/CU\n",
                         (long long)R, wmax, sh.block, sh.per_cu);
        NN_HIP_TRY(ctx, hipEventRecord(t0, st));   // the call's clock restarts after tuning
    }
    const int blk = sh.block;

    // ---- one global step on stream s with grids gr (slices) and fg (members),
    // the row and vector passes optionally bracketed by timing events
    // (with events, the row and vector passes record their own begin and
    // end into ev[0..1] and ev[2..3])
    auto step = [&](hipStream_t s, int gr, int fg, hipEvent_t *ev) {
        hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
        if (quad)
            NN_BDISPATCH_EV(wmax, (kb_rows<WM, CM_Q4, float, float>), gr, blk, s, e0, e1, B,
                            (const float *)gv32, V32);
        else if (mixed)
            NN_BDISPATCH_EV(wmax, (kb_rows<WM, CM_I32, float, float>), gr, blk, s, e0, e1, B,
                            (const float *)gv32, V32);
        else if (pair)
            NN_BDISPATCH_EV(wmax, (kb_rows<WM, CM_P2, double, double>), gr, blk, s, e0, e1, B,
                            (const double *)gv64, V64);
        else
            NN_BDISPATCH_EV(wmax, (kb_rows<WM, CM_I32, double, double>), gr, blk, s, e0, e1, B,
                            (const double *)gv64, V64);
        hipLaunchKernelGGL(kb_step1, dim3(fg), dim3(kFinBlock), 0, s, B);
        if (ev && mixed)
            hipExtLaunchKernelGGL((kb_vec<float>), dim3(gr), dim3(blk), 0, s, ev[2], ev[3], 0, B, V32);
        else if (ev)
            hipExtLaunchKernelGGL((kb_vec<double>), dim3(gr), dim3(blk), 0, s, ev[2], ev[3], 0, B, V64);
        else if (mixed)
            hipLaunchKernelGGL((kb_vec<float>), dim3(gr), dim3(blk), 0, s, B, V32);
        else
            hipLaunchKernelGGL((kb_vec<double>), dim3(gr), dim3(blk), 0, s, B, V64);
        hipLaunchKernelGGL(kb_step2, dim3(fg), dim3(kFinBlock), 0, s, B);
    };

    // ---- chunks of global steps.  Without profiling a chunk is captured
    // into a graph on the context's private capture stream (the caller's
    // stream may be the legacy default stream, which cannot be captured) and
    // replayed on the caller's stream, one graph per size class of the
    // running list.  With profiling on, or if capture fails, steps are
    // launched one by one (with profiling, one step per chunk, each pass
    // bracketed by events).
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
        const int fg = std::min(P, 1 << cls);   // a listed member owns at least one slice
        if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        for (int k = 0; k < chunk; k++) step(ctx->cap_stream, gr, fg, nullptr);
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
    Events ev_step;
    if (ctx->prof && !ev_step.create(4, hipEventDefault))
        return fail(ctx, NN_EHIP, "event creation");

    // Every member's step count is bounded by its caps (outer iterations,
    // trials per search, CG iterations); the guard only stops a runaway loop.
    const int64_t max_steps =
        (int64_t)(o->max_outer + 1) * (4 + 2 * kMaxTrials + 21 + o->max_cg) + 16;
    nn_status err = NN_OK;
    int64_t steps = 0;
    while (steps < max_steps) {
        if (!select()) {
            err = fail(ctx, NN_EHIP, "batch list upload");
            break;
        }
        if (n_pr == 0) break;
        const int gr = grid_for(sh, n_sl);
        if (ctx->prof) {
            // one step; algorithmic bytes of the row pass from the states
            double brow = 0.0, brow_csr = 0.0;
            for (int p = 0; p < P; p++)
                if (hs[p].phase != PH_DONE) {
                    brow += row_bytes(hs[p]);
                    brow_csr += row_bytes_csr(hs[p]);
                }
            step(st, gr, std::max(n_pr, 1), ev_step.ev.data());
            steps++;
            if (!pull()) {
                err = fail(ctx, NN_EHIP, "batch read-back");
                break;
            }
            float m1 = 0.f, m2 = 0.f;
            if (brow > 0.0 && ((ctx->prof_mask >> KC_CG_SPMV) & 1) &&
                hipEventElapsedTime(&m1, ev_step.ev[0], ev_step.ev[1]) == hipSuccess)
                prof_add(ctx, KC_CG_SPMV, m1, brow, brow_csr);
            if (((ctx->prof_mask >> KC_CG_UPDATE) & 1) &&
                hipEventElapsedTime(&m2, ev_step.ev[2], ev_step.ev[3]) == hipSuccess)
                prof_add(ctx, KC_CG_UPDATE, m2, 0.0);
            (void)hipGetLastError();
            continue;
        }
        hipGraphExec_t ex = use_graph ? graph_for(n_sl) : nullptr;
        if (ex) {
            if (hipGraphLaunch(ex, st) != hipSuccess) {
                err = fail(ctx, NN_EHIP, "graph launch");
                break;
            }
        } else {
            for (int k = 0; k < chunk; k++) step(st, gr, std::max(n_pr, 1), nullptr);
        }
        steps += chunk;
        if (!pull()) {
            err = fail(ctx, NN_EHIP, "batch read-back");
            break;
        }
        if (o->verbose) {
            int nr = 0, ncg = 0;
            for (int p = 0; p < P; p++) {
                nr += hs[p].phase != PH_DONE ? 1 : 0;
                ncg += hs[p].phase == PH_CG ? 1 : 0;
            }
            std::fprintf(stderr,
                         "nnqp batch step %lld: %d of %d members running (%d in CG); member 0: "
                         "outer %d kkt %.3e\n",
                         (long long)steps, nr, P, ncg, hs[0].outer, hs[0].kkt_rel);
        }
    }
    if (err == NN_OK && steps >= max_steps) {
        for (int p = 0; p < P; p++)
            if (hs[p].phase != PH_DONE) {
                hs[p].status = NN_EMAXIT;
                hs[p].phase = PH_DONE;
            }
    }
    // ---- outputs: the solutions back into the members' vectors, active sets
    {
        const int64_t blocks = std::min<int64_t>((S + 3) / 4, (int64_t)num_cu * 8);
        hipLaunchKernelGGL(kb_scatter, dim3((int)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, B);
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
        const BState &M = hs[p];
        nn_stats &Q = SP[p];
        Q.kkt_rel = M.kkt_rel;
        Q.kkt_nat_inf = M.kkt_nat;
        Q.min_c = M.min_c;
        Q.norm_f = M.normf;
        Q.outer_its = M.outer;
        Q.cg_its = M.cg_its;
        Q.spmvs = M.spmvs;
        Q.n_active = M.n_active;
        Q.cauchy_trials = M.cauchy_trials;
        Q.search_trials = M.search_trials;
        Q.refinements = M.refinements;
        Q.status = M.status;
        Q.bytes_moved = M.bytes;
        Q.seconds = ms * 1e-3;   // the whole batched call
        if (M.status != NN_OK && first_bad < 0) first_bad = p;
    }
    if (stats)
        for (int p = 0; p < P; p++) stats[p] = SP[p];
    if (first_bad >= 0) {
        char msg[160];
        std::snprintf(msg, sizeof(msg),
                      "batch member %d (the first affected) ended with status %d; every member's "
                      "status is in its stats",
                      first_bad, hs[first_bad].status);
        return fail(ctx, (nn_status)hs[first_bad].status, msg);
    }
    ctx->err.clear();
    return NN_OK;
}

}  // namespace nnqp
