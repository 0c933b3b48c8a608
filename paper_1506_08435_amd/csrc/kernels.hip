// Row-parallel kernels of the non-negative QP solver for gfx950.
//
// Every kernel here is bound by HBM bandwidth (sparse matrix-vector products
// at ~0.14 flop/byte and vector streams), so the design goal is bytes and
// latency, not flops:
//  - K is held in sliced-ELL form (64-row slices, one lane per row, entries
//    column-major within a slice): a wavefront's index/value loads are single
//    contiguous segments, each lane issues all of its row's loads before the
//    first gather, and the row sum is a plain sequential chain (no cross-lane
//    shuffles, fixed order);
//  - vector updates and dot products are fused into the passes that already
//    touch the same rows;
//  - reductions leave one partial per block and are never combined with
//    atomics or fences: the host combines what it reads, and the CG scalars
//    are combined by every block of the next kernel in the same fixed order,
//    so results are bitwise reproducible and no cross-XCD synchronisation is
//    needed inside a kernel.
#include <cmath>

#include "nnqp_internal.hpp"
#include "rows.hpp"

namespace nnqp {

Part make_part(int64_t n, int max_blocks)
{
    Part p;
    p.n = (int)n;
    p.nslices = (int)((n + kSlice - 1) / kSlice);
    int64_t nb = (p.nslices + kWaves - 1) / kWaves;
    if (nb < 1) nb = 1;
    if (nb > max_blocks) nb = max_blocks;
    p.nb = (int)nb;
    return p;
}

// ---------------------------------------------------------------- kernels
template <int WMAX, class Cols>
__global__ __launch_bounds__(kBlock) void k_matvec(Part P, const int *__restrict__ so, Cols sc,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ x, double *__restrict__ y)
{
    sell_rows<WMAX>(P, so, sc, v, AllRows(), NoPre(), [&](int j) { return x[j]; },
                    [&](int i, double s, int) { y[i] = s; });
}

// ft = f + (M c) / dt
template <int WMAX, class Cols>
__global__ __launch_bounds__(kBlock) void k_transient_rhs(Part P, const int *__restrict__ so, Cols sc,
                                                          const double *__restrict__ m,
                                                          const double *__restrict__ c,
                                                          const double *__restrict__ f, double dt,
                                                          double *__restrict__ ft)
{
    sell_rows<WMAX>(P, so, sc, m, AllRows(), [&](int i) { return f[i]; },
                    [&](int j) { return c[j]; },
                    [&](int i, double s, double fi) { ft[i] = fi + s / dt; });
}

// g = K c - f with the projected-gradient report:
// |pg|^2, #non-finite, ||c - P(c - g)||_inf, min c, #(c at a bound)
// pg_i = g_i strictly inside [lo, hi], min(g_i, 0) at lo, max(g_i, 0) at hi;
// the natural residual c - P(c - g) = max(c - hi, min(g, c - lo)) (min(c, g)
// for [0, inf)).
constexpr uint32_t kOpsGrad = OPS5(OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM);

template <int WMAX, class Cols>
__global__ __launch_bounds__(kBlock) void k_grad(Part P, const int *__restrict__ so, Cols sc,
                                                 const double *__restrict__ v,
                                                 const double *__restrict__ c,
                                                 const double *__restrict__ f,
                                                 double *__restrict__ g, double *partials, Box B)
{
    double a[5];
    red_init<kOpsGrad, 5>(a);
    sell_rows<WMAX>(P, so, sc, v, AllRows(), [&](int i) { return Two{c[i], f[i]}; },
                    [&](int j) { return c[j]; }, [&](int i, double s, Two cf) {
        const double gi = s - cf.b;
        const double cv = cf.a;
        g[i] = gi;
        const double pg = cv > B.lo ? (cv < B.hi ? gi : fmax(gi, 0.0)) : fmin(gi, 0.0);
        a[0] += pg * pg;
        a[1] += (isfinite(gi) && isfinite(cv)) ? 0.0 : 1.0;
        a[2] = fmax(a[2], fabs(fmax(cv - B.hi, fmin(gi, cv - B.lo))));
        a[3] = fmin(a[3], cv);
        a[4] += (cv == B.lo || cv == B.hi) ? 1.0 : 0.0;
    });
    block_partial<kOpsGrad, 5>(a, slot_ptr(partials, SLOT_HOST));
}

// Residual report of an unconstrained solve: r = K c - f (not stored);
// |r|^2, #non-finite, max c, min c, #(c < 0)
constexpr uint32_t kOpsResid = OPS5(OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM);

template <int WMAX, class Cols>
__global__ __launch_bounds__(kBlock) void k_resid(Part P, const int *__restrict__ so, Cols sc,
                                                  const double *__restrict__ v,
                                                  const double *__restrict__ c,
                                                  const double *__restrict__ f, double *partials)
{
    double a[5];
    red_init<kOpsResid, 5>(a);
    sell_rows<WMAX>(P, so, sc, v, AllRows(), [&](int i) { return Two{c[i], f[i]}; },
                    [&](int j) { return c[j]; }, [&](int, double s, Two cf) {
                        const double ri = s - cf.b;
                        a[0] += ri * ri;
                        a[1] += (isfinite(ri) && isfinite(cf.a)) ? 0.0 : 1.0;
                        a[2] = fmax(a[2], cf.a);
                        a[3] = fmin(a[3], cf.a);
                        a[4] += cf.a < 0.0 ? 1.0 : 0.0;
                    });
    block_partial<kOpsResid, 5>(a, slot_ptr(partials, SLOT_HOST));
}

// c += w (no projection: the unconstrained solve)
template <class VV>
__global__ __launch_bounds__(kBlock) void k_add(Part P, double *__restrict__ c,
                                                const VV *__restrict__ w)
{
    for_rows(P, [&](int i, bool act) {
        if (act) c[i] += (double)w[i];
    });
}

// Trial point of a projected search: s = P(c + t d) - c, formed for every
// gathered column; ks = K s; report g.s, s.Ks, s.s.  Rows with mask == 0 are
// skipped when a mask is given (there d = 0, so s = 0 and they add nothing).
constexpr uint32_t kOpsTrial = OPS3(OP_SUM, OP_SUM, OP_SUM);

template <int WMAX, class VT, class VD, class Cols>
__global__ __launch_bounds__(kBlock) void k_trial(Part P, const int *__restrict__ so, Cols sc,
                                                  const VT *__restrict__ v,
                                                  const double *__restrict__ c,
                                                  const VD *__restrict__ d, double t,
                                                  const double *__restrict__ g,
                                                  const uint8_t *__restrict__ mask,
                                                  double *__restrict__ ks, double *partials, Box B)
{
    auto sv = [&](int j) {
        const double cj = c[j];
        return proj_box(cj + t * (double)d[j], B) - cj;
    };
    double a[3];
    red_init<kOpsTrial, 3>(a);
    sell_rows<WMAX>(P, so, sc, v, [&](int i) { return mask == nullptr || mask[i] != 0; },
                    [&](int i) { return Two{sv(i), g[i]}; }, sv, [&](int i, double s, Two sg) {
                        if (ks) ks[i] = s;
                        const double si = sg.a;
                        a[0] += sg.b * si;
                        a[1] += si * s;
                        a[2] += si * si;
                    });
    block_partial<kOpsTrial, 3>(a, slot_ptr(partials, SLOT_HOST));
}

// Cauchy ladder: the projected steepest-descent trial s_k = P(c - t_k g) - c
// for kLadder step lengths in one matrix pass (the entries are read once and
// each gathered column yields all kLadder trial values); ks_k = K s_k; per k
// the sums g.s_k, s_k.Ks_k, s_k.s_k as values 3k, 3k+1, 3k+2 of a
// 3 kLadder-value partial starting at SLOT_U0 (it may span SLOT_U1).
struct Ladder {
    double t[kLadder];
    double *ks[kLadder];
};

#ifndef NNQP_LADDER_PHASE
#define NNQP_LADDER_PHASE 4   // entries per load phase of the Cauchy ladder pass
#endif

template <int WMAX, class VT, class Cols>
__global__ __launch_bounds__(kBlock) void k_ladder(Part P, const int *__restrict__ so, Cols sc,
                                                   const VT *__restrict__ v,
                                                   const double *__restrict__ c,
                                                   const double *__restrict__ g, Ladder L, Box B,
                                                   double *partials)
{
    double a[3 * kLadder];
#pragma unroll
    for (int k = 0; k < 3 * kLadder; k++) a[k] = 0.0;
    auto trials = [&](int j, double (&out)[kLadder]) {
        const double cj = c[j], gj = g[j];
#pragma unroll
        for (int k = 0; k < kLadder; k++) out[k] = proj_box(cj - L.t[k] * gj, B) - cj;
    };
    auto pre = [&](int i) { return Two{c[i], g[i]}; };
    auto epi = [&](int i, double (&kv)[kLadder], Two cg) {
        double si[kLadder];
        trials(i, si);
#pragma unroll
        for (int k = 0; k < kLadder; k++) {
            L.ks[k][i] = kv[k];
            a[3 * k] += cg.b * si[k];
            a[3 * k + 1] += si[k] * kv[k];
            a[3 * k + 2] += si[k] * si[k];
        }
    };
    // the nine running sums stay in registers for the whole pass, so the
    // entries load NNQP_LADDER_PHASE at a time
    sell_rows_n<WMAX, kLadder, VT, Cols, decltype(pre), decltype(trials), decltype(epi),
                NNQP_LADDER_PHASE>(P, so, sc, v, pre, trials, epi);
    block_partial<0u, 3 * kLadder>(a, slot_ptr(partials, SLOT_U0));
}

// c = P(c + t d)
template <class VD>
__global__ __launch_bounds__(kBlock) void k_apply(Part P, double *__restrict__ c,
                                                  const VD *__restrict__ d, double t, Box B)
{
    for_rows(P, [&](int i, bool act) {
        if (act) c[i] = proj_box(c[i] + t * (double)d[i], B);
    });
}

// c = c0v (mode 0) or c = P(c) (mode 1); report |f|^2, max f, #non-finite f,
// #non-finite c (before projection)
constexpr uint32_t kOpsInit = OPS4(OP_SUM, OP_MAX, OP_SUM, OP_SUM);

__global__ __launch_bounds__(kBlock) void k_init(Part P, double *__restrict__ c,
                                                 const double *__restrict__ f, int mode, double c0v,
                                                 double *partials, Box B)
{
    double a[4];
    red_init<kOpsInit, 4>(a);
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        const double fi = f[i];
        a[0] += fi * fi;
        a[1] = fmax(a[1], fi);
        a[2] += isfinite(fi) ? 0.0 : 1.0;
        if (mode == 0) {
            c[i] = c0v;
        } else {
            const double cv = c[i];
            a[3] += isfinite(cv) ? 0.0 : 1.0;
            c[i] = proj_box(cv, B);
        }
    });
    block_partial<kOpsInit, 4>(a, slot_ptr(partials, SLOT_HOST));
}

// Set-up of the inner CG on the face of (c, g + ks):
//   g <- g + ks (gradient at the Cauchy point), free = not (c == 0 and g >= 0),
//   dm = 1/diag on free rows and 0 elsewhere (the mask folded into the
//   Jacobi preconditioner), r = -g on free rows, z = dm r, p = q = w = 0.
// Partials (SLOT_U0): r.z, r.r, #free, nnz of free rows.
constexpr uint32_t kOpsU = OPS4(OP_SUM, OP_SUM, OP_SUM, OP_SUM);

template <class VV>
__global__ __launch_bounds__(kBlock) void k_cg_setup(
    Part P, const int *__restrict__ rp, const double *__restrict__ diag,
    const double *__restrict__ c, double *__restrict__ g, const double *__restrict__ ks,
    uint8_t *__restrict__ mask, VV *__restrict__ dm, VV *__restrict__ r, VV *__restrict__ z,
    VV *__restrict__ p, VV *__restrict__ q, VV *__restrict__ w, double *partials, DevScalars *S,
    Box B, int face, VV *__restrict__ cres, VV *__restrict__ cdz0, VV *__restrict__ cdz1,
    double inv_theta)
{
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        const double gi = ks ? g[i] + ks[i] : g[i];
        if (ks) g[i] = gi;
        const double cv = c[i];
        const bool fr = face == FACE_ALL ? true
                      : face == FACE_INTERIOR ? (cv != B.lo && cv != B.hi)
                      : !((cv == B.lo && gi >= 0.0) || (cv == B.hi && gi <= 0.0));
        const VV dmi = fr ? (VV)(1.0 / diag[i]) : VV(0);
        const VV ri = fr ? (VV)(-gi) : VV(0);
        // Jacobi z = dm r, or the first Chebyshev term dm r / theta
        const VV zi = cres ? (VV)((double)dmi * (double)ri * inv_theta) : dmi * ri;
        mask[i] = fr ? 1 : 0;
        dm[i] = dmi;
        r[i] = ri;
        z[i] = zi;
        p[i] = VV(0);
        q[i] = VV(0);
        w[i] = VV(0);
        if (cres) {
            cres[i] = ri;
            cdz0[i] = zi;
            cdz1[i] = VV(0);
        }
        a[0] += (double)ri * (double)zi;
        a[1] += (double)ri * (double)ri;
        a[2] += fr ? 1.0 : 0.0;
        a[3] += fr ? (double)(rp[i + 1] - rp[i]) : 0.0;
    });
    block_partial<kOpsU, 4>(a, slot_ptr(partials, SLOT_U0));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S->done = 0;
        S->it = 0;
        S->ww[0] = 0.0;   // w = 0
        S->tr_hit = 0;
    }
}

// CG iteration j, matrix pass.
// Prologue (identical in every block): r.z_j and r.r_j from the partials the
// previous kernel left in slot U[j%2]; stop if r.r_j <= rtol^2 r.r_0, at the
// iteration cap, or when the previous update stopped on the trust-region
// boundary; beta_j = r.z_j / r.z_{j-1} (0 for j = 0).
// Body: the direction update p <- z + beta p and its product q = K p are
// formed together, using K p = K z + beta (K p_old): only z is gathered, and
// p, q are updated in place on the free rows; partials of p.q into SLOT_Q
// (with TR, also p.p and w.p, which the update needs for |w + alpha p|).
// Columns outside the free set contribute 0 because z vanishes there.
template <int WMAX, class VT, class VV, class Cols, bool TR>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(Part P, const int *__restrict__ so, Cols sc,
                                                    const VT *__restrict__ v,
                                                    const uint8_t *__restrict__ mask,
                                                    const VV *__restrict__ z,
                                                    VV *__restrict__ p, VV *__restrict__ q,
                                                    const VV *__restrict__ w,
                                                    double *partials, DevScalars *S, int j,
                                                    int max_it, double rtol2)
{
    if (S->done) return;
    double u[4];
    combine_partials<kOpsU, 4>(slot_ptr(partials, (j & 1) ? SLOT_U1 : SLOT_U0), P.nb, u);
    const double rz = u[0], rr2 = u[1];
    const double rr_stop = j == 0 ? rtol2 * rr2 : S->rr_stop;
    int done = 0;
    if (TR && j > 0 && S->tr_hit) done = 2;
    else if (!isfinite(rz) || !isfinite(rr2)) done = 4;
    else if ((j == 0 && (rr2 == 0.0 || u[2] == 0.0)) || (j > 0 && rr2 <= rr_stop) ||
             j >= max_it || !(rz > 0.0))
        done = 1;
    const double beta = j == 0 ? 0.0 : rz / S->rzh[(j - 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (j == 0) {
            S->rr_stop = rr_stop;
            S->n_free = u[2];
            S->nnz_free = u[3];
        }
        S->rzh[j & 1] = rz;
        if (done) {
            S->done = done;
            S->it = j;
        }
    }
    if (done) return;
    constexpr int NQ = TR ? 3 : 1;
    double a[NQ];
#pragma unroll
    for (int k = 0; k < NQ; k++) a[k] = 0.0;
    sell_rows<WMAX>(P, so, sc, v, [&](int i) { return mask[i] != 0; },
                    [&](int i) { return Three{(double)p[i], (double)q[i], (double)z[i]}; },
                    [&](int jj) { return (double)z[jj]; }, [&](int i, double kz, Three pqz) {
                        const VV pi = (VV)fma(beta, pqz.a, pqz.c);
                        const VV qi = (VV)fma(beta, pqz.b, kz);
                        p[i] = pi;
                        q[i] = qi;
                        a[0] += (double)pi * (double)qi;
                        if constexpr (TR) {
                            a[1] += (double)pi * (double)pi;
                            a[2] += (double)w[i] * (double)pi;
                        }
                    });
    block_partial<0u, NQ>(a, slot_ptr(partials, SLOT_Q));
}

// CG iteration j, vector update on free rows.
// Prologue: p.q_j from SLOT_Q, alpha_j = r.z_j / p.q_j (r.z_j stored by the
// matrix pass).  Body: w += alpha p, r -= alpha q, z = dm r; partials of
// r.z_{j+1}, r.r_{j+1} into slot U[(j+1)%2].  With the Chebyshev
// preconditioner (cres set) z starts as dm r / theta, the Chebyshev residual
// and first increment are set, and the last Chebyshev pass replaces r.z.
// With a finite trust region (TR, radius^2 delta2) the step alpha that
// would take |w + alpha p| past the radius is cut to the tau >= 0 with
// |w + tau p| = radius (Steihaug's truncated CG, as TRON's inner solve),
// using |w|^2 kept on the device by the recurrence
// |w + t p|^2 = |w|^2 + 2 t w.p + t^2 p.p; the next matrix pass then ends
// the CG (done = 2).
template <class VV, bool TR>
__global__ __launch_bounds__(kBlock) void k_cg_update(Part P, const uint8_t *__restrict__ mask,
                                                      const VV *__restrict__ p,
                                                      const VV *__restrict__ q,
                                                      const VV *__restrict__ dm,
                                                      VV *__restrict__ w, VV *__restrict__ r,
                                                      VV *__restrict__ z, double *partials,
                                                      DevScalars *S, int j, VV *__restrict__ cres,
                                                      VV *__restrict__ cdz0, double inv_theta,
                                                      double delta2)
{
    if (S->done) return;
    constexpr int NQ = TR ? 3 : 1;
    double pqa[NQ];
    combine_partials<0u, NQ>(slot_ptr(partials, SLOT_Q), P.nb, pqa);
    const double pq = pqa[0];
    if (!(pq > 0.0 && isfinite(pq))) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S->done = isfinite(pq) ? 3 : 4;
            S->it = j;
        }
        return;
    }
    double alpha = S->rzh[j & 1] / pq;
    if constexpr (TR) {
        const double pp = pqa[1], wp = pqa[2], ww = S->ww[j & 1];
        double wn = ww + alpha * (2.0 * wp + alpha * pp);
        int hit = 0;
        if (wn >= delta2) {
            // positive root of pp t^2 + 2 wp t + (ww - delta2) = 0 (ww <= delta2),
            // in the form without cancellation for either sign of wp
            const double room = fmax(delta2 - ww, 0.0);
            const double disc = sqrt(wp * wp + pp * room);
            alpha = wp >= 0.0 ? room / (wp + disc) : (disc - wp) / pp;
            wn = delta2;
            hit = 1;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S->ww[(j + 1) & 1] = wn;
            S->tr_hit = hit;
        }
    }
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for_rows(P, [&](int i, bool act) {
        if (!act || !mask[i]) return;
        const VV ri = (VV)((double)r[i] - alpha * (double)q[i]);
        const VV zi = cres ? (VV)((double)dm[i] * (double)ri * inv_theta) : dm[i] * ri;
        w[i] = (VV)((double)w[i] + alpha * (double)p[i]);
        r[i] = ri;
        z[i] = zi;
        if (cres) {
            cres[i] = ri;
            cdz0[i] = zi;
        }
        a[0] += (double)ri * (double)zi;
        a[1] += (double)ri * (double)ri;
    });
    block_partial<kOpsU, 4>(a, slot_ptr(partials, ((j + 1) & 1) ? SLOT_U1 : SLOT_U0));
    if (blockIdx.x == 0 && threadIdx.x == 0) S->it = j + 1;
}

// One step of the Chebyshev iteration for A_FF z = r from z = 0 with the
// Jacobi splitting (the polynomial preconditioner of the inner CG), on the
// free rows: res -= A dzp (dzp gathered; zero off the face), dzn = ca dzp +
// cb dm res, z += dzn.  The last step leaves r.z in value 0 of `slot` (the
// slot whose r.r the update or set-up kernel wrote).
template <int WMAX, class VT, class VV, class Cols>
__global__ __launch_bounds__(kBlock) void k_cheb(Part P, const int *__restrict__ so, Cols sc,
                                                 const VT *__restrict__ v,
                                                 const uint8_t *__restrict__ mask,
                                                 const VV *__restrict__ dm,
                                                 const VV *__restrict__ r, VV *__restrict__ res,
                                                 const VV *__restrict__ dzp, VV *__restrict__ dzn,
                                                 VV *__restrict__ z, double ca, double cb,
                                                 int last, int slot, double *partials,
                                                 DevScalars *S)
{
    if (S->done) return;
    double a[1] = {0.0};
    sell_rows<WMAX>(P, so, sc, v, [&](int i) { return mask[i] != 0; },
                    [&](int i) { return Three{(double)res[i], (double)dzp[i], (double)z[i]}; },
                    [&](int jj) { return (double)dzp[jj]; }, [&](int i, double kd, Three x) {
                        const double rn = x.a - kd;
                        const double dn = ca * x.b + cb * (double)dm[i] * rn;
                        const VV zn = (VV)(x.c + dn);
                        res[i] = (VV)rn;
                        dzn[i] = (VV)dn;
                        z[i] = zn;
                        a[0] += (double)r[i] * (double)zn;
                    });
    if (last) block_partial<OP_SUM, 1>(a, slot_ptr(partials, slot));
}

// Gershgorin bound of the spectrum of D^-1 A: max over rows of sum_j |a_ij| / a_ii
// (an upper bound for every principal submatrix too).
__global__ __launch_bounds__(kBlock) void k_gersh(Part P, const int *__restrict__ so,
                                                  const double *__restrict__ v,
                                                  const double *__restrict__ diag, double *partials)
{
    double a[1] = {0.0};
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        const int s = i / kSlice, lane = i % kSlice;
        const int off = so[s], w = (so[s + 1] - off) / kSlice;
        double sum = 0.0;
        for (int k = 0; k < w; k++) sum += fabs(v[off + k * kSlice + lane]);
        a[0] = fmax(a[0], sum / diag[i]);
    });
    block_partial<OP_MAX, 1>(a, slot_ptr(partials, SLOT_HOST));
}

// Largest step along w before a free variable reaches a bound:
// min over w_i < 0 of (c_i - lo) / (-w_i) and over w_i > 0 of (hi - c_i) / w_i
// (+inf for hi = +inf), g.w, w.w
constexpr uint32_t kOpsBrk = OPS3(OP_MIN, OP_SUM, OP_SUM);

template <class VV>
__global__ __launch_bounds__(kBlock) void k_breakpoint(Part P, const double *__restrict__ c,
                                                       const VV *__restrict__ w,
                                                       const double *__restrict__ g,
                                                       double *partials, Box B)
{
    double a[3];
    red_init<kOpsBrk, 3>(a);
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        const double wi = (double)w[i];
        if (wi < 0.0) a[0] = fmin(a[0], (c[i] - B.lo) / (-wi));
        else if (wi > 0.0) a[0] = fmin(a[0], (B.hi - c[i]) / wi);
        a[1] += g[i] * wi;
        a[2] += wi * wi;
    });
    block_partial<kOpsBrk, 3>(a, slot_ptr(partials, SLOT_HOST));
}

__global__ __launch_bounds__(kBlock) void k_active(Part P, const double *__restrict__ c,
                                                   uint8_t *__restrict__ active, Box B)
{
    for_rows(P, [&](int i, bool act) {
        if (act) active[i] = c[i] == B.lo ? 1 : (c[i] == B.hi ? 2 : 0);
    });
}

__global__ __launch_bounds__(kBlock) void k_vals_mdt_plus_k(int64_t nnz, const double *__restrict__ m,
                                                            double dt, const double *__restrict__ k,
                                                            double *__restrict__ out)
{
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * kBlock)
        out[t] = m[t] / dt + k[t];
}

// Paired copy of a sliced-ELL array (the layout of nn_matrix::d16p): within
// slice s of width w, entry k of lane l moves from off + 64 k + l to
// off + 128 (k / 2) + 2 l + k % 2 for k < 2 (w / 2); an odd last column stays.
template <class T>
__global__ __launch_bounds__(kBlock) void k_pair(Part P, const int *__restrict__ so,
                                                 const T *__restrict__ src, T *__restrict__ dst)
{
    const int lane = threadIdx.x & 63, wid = wave_id();
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += P.nb * kWaves) {
        const int off = so[s], w = (so[s + 1] - off) / kSlice, wp = 2 * (w / 2);
        for (int k = 0; k < w; k++) {
            const int from = off + k * kSlice + lane;
            const int to = k < wp ? off + (k / 2) * 2 * kSlice + 2 * lane + (k & 1) : from;
            dst[to] = src[from];
        }
    }
}

// Quad copy of a sliced-ELL array (the layout of nn_matrix::d16q): within
// slice s of width w, entry k of lane l moves to off + 256 (k / 4) + 4 l + k % 4
// for k < 4 (w / 4); the next two, if there are two left, to
// off + 256 (w / 4) + 2 l + (k - 4 (w / 4)); an odd last one stays.
template <class T>
__global__ __launch_bounds__(kBlock) void k_quad(Part P, const int *__restrict__ so,
                                                 const T *__restrict__ src, T *__restrict__ dst)
{
    const int lane = threadIdx.x & 63, wid = wave_id();
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += P.nb * kWaves) {
        const int off = so[s], w = (so[s + 1] - off) / kSlice;
        const int nq = w / 4, np = (w - 4 * nq) / 2;
        for (int k = 0; k < w; k++) {
            const int from = off + k * kSlice + lane;
            int to = from;
            if (k < 4 * nq) to = off + (k / 4) * 4 * kSlice + 4 * lane + (k & 3);
            else if (k < 4 * nq + 2 * np) to = off + nq * 4 * kSlice + 2 * lane + (k - 4 * nq);
            dst[to] = src[from];
        }
    }
}

// float32 copy of a value array (round to nearest)
__global__ __launch_bounds__(kBlock) void k_to_f32(int64_t m, const double *__restrict__ a,
                                                   float *__restrict__ b)
{
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * kBlock)
        b[t] = (float)a[t];
}

// diag[i] = entry of row i in column i (sliced-ELL)
__global__ __launch_bounds__(kBlock) void k_diag(Part P, const int *__restrict__ so,
                                                 const int *__restrict__ sc,
                                                 const double *__restrict__ v,
                                                 double *__restrict__ diag)
{
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        const int s = i / kSlice, lane = i % kSlice;
        const int off = so[s], w = (so[s + 1] - off) / kSlice;
        double d = 0.0;
        bool found = false;
        for (int k = 0; k < w; k++) {
            const int e = off + k * kSlice + lane;
            if (!found && sc[e] == i) {   // the real entry precedes any padding
                d = v[e];
                found = true;
            }
        }
        diag[i] = d;
    });
}

// CSR (rowptr-ordered values) -> sliced-ELL: entry k of row i goes to
// so[i/64] + k*64 + i%64; padding entries get column i and value 0.
__global__ __launch_bounds__(kBlock) void k_csr_to_sell(Part P, const int *__restrict__ rp,
                                                        const int *__restrict__ ci,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ mval,
                                                        const int *__restrict__ so,
                                                        int *__restrict__ sc, double *__restrict__ sv,
                                                        double *__restrict__ smv)
{
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        const int s = i / kSlice, lane = i % kSlice;
        const int off = so[s], w = (so[s + 1] - off) / kSlice;
        const int k0 = rp[i], len = rp[i + 1] - rp[i];
        for (int k = 0; k < w; k++) {
            const int e = off + k * kSlice + lane;
            const bool real = k < len;
            sc[e] = real ? ci[k0 + k] : i;
            sv[e] = real ? val[k0 + k] : 0.0;
            if (smv) smv[e] = real ? mval[k0 + k] : 0.0;
        }
    });
}

// The rows of the last slice past n keep their padding: fill them so every
// entry of the sliced-ELL arrays is defined (column 0, value 0).
__global__ __launch_bounds__(kBlock) void k_sell_tail(int n, int nslices, const int *__restrict__ so,
                                                      int *__restrict__ sc, double *__restrict__ sv,
                                                      double *__restrict__ smv)
{
    const int s = nslices - 1;
    if (s < 0) return;
    const int off = so[s], w = (so[s + 1] - off) / kSlice;
    for (int t = threadIdx.x; t < w * kSlice; t += kBlock) {
        const int lane = t % kSlice;
        if (s * kSlice + lane < n) continue;
        sc[off + t] = 0;
        sv[off + t] = 0.0;
        if (smv) smv[off + t] = 0.0;
    }
}

// int16 offsets col - row of the sliced-ELL entries and the largest |col - row|
// over real rows (one partial per block, SLOT_HOST).  Lanes past the last row
// get offsets that point at the last row, so every decoded column is valid.
__global__ __launch_bounds__(kBlock) void k_sell_d16(Part P, const int *__restrict__ so,
                                                     const int *__restrict__ sc,
                                                     short *__restrict__ sd, double *partials)
{
    double a[1];
    red_init<OP_MAX, 1>(a);
    for_rows(P, [&](int i, bool act) {
        const int s = i / kSlice, lane = i % kSlice;
        const int off = so[s], w = (so[s + 1] - off) / kSlice;
        for (int k = 0; k < w; k++) {
            const int e = off + k * kSlice + lane;
            const int d = act ? sc[e] - i : (P.n - 1) - i;
            if (act) a[0] = fmax(a[0], (double)abs(d));
            sd[e] = (short)max(-32768, min(32767, d));
        }
    });
    block_partial<OP_MAX, 1>(a, slot_ptr(partials, SLOT_HOST));
}

// ---------------------------------------------------------------- launchers
// (NN_DISPATCH_W, in rows.hpp, instantiates a kernel for the matrix's slice
// width class.)

void launch_matvec(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *x, double *y)
{
    if (A->n == 0) return;
    Part P = make_part(A->n);
    NN_DISPATCH_W(A->wmax, (k_matvec<WM, ColsI32>), P.nb, P, A->sl_off, ColsI32{A->sl_col}, vals, x, y);
}

void launch_transient_rhs(nn_ctx *ctx, const nn_matrix *A, const double *c, const double *f,
                          double dt, double *ft)
{
    if (A->n == 0) return;
    Part P = make_part(A->n);
    NN_DISPATCH_W(A->wmax, (k_transient_rhs<WM, ColsI32>), P.nb, P, A->sl_off, ColsI32{A->sl_col}, A->mval,
                  c, f, dt, ft);
}

void launch_init(nn_ctx *ctx, int64_t n, double *c, const double *f, int mode, double c0v, Box B)
{
    Part P = make_part(n);
    k_init<<<P.nb, kBlock, 0, ctx->stream>>>(P, c, f, mode, c0v, ctx->partials, B);
}

void launch_grad(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *vals_p,
                 const double *c, const double *f, double *g, Box B)
{
    Part P = make_part(A->n);
    if (vals_p && A->d16p)
        NN_DISPATCH_W(A->wmax, (k_grad<WM, ColsD16P>), P.nb, P, A->sl_off, ColsD16P{A->d16p}, vals_p,
                      c, f, g, ctx->partials, B);
    else
        NN_DISPATCH_W(A->wmax, (k_grad<WM, ColsI32>), P.nb, P, A->sl_off, ColsI32{A->sl_col}, vals,
                      c, f, g, ctx->partials, B);
}

void launch_trial(nn_ctx *ctx, const nn_matrix *A, const Vals &V, const double *c, Dir d,
                  double t, const double *g, const uint8_t *mask, double *ks, Box B)
{
    Part P = make_part(A->n);
    if (V.v32q && A->d16q) {
        const ColsD16Q cols{A->d16q};
        if (d.f32)
            NN_DISPATCH_W(A->wmax, (k_trial<WM, float, float, ColsD16Q>), P.nb, P, A->sl_off, cols,
                          V.v32q, c, d.f32, t, g, mask, ks, ctx->partials, B);
        else
            NN_DISPATCH_W(A->wmax, (k_trial<WM, float, double, ColsD16Q>), P.nb, P, A->sl_off, cols,
                          V.v32q, c, d.f64, t, g, mask, ks, ctx->partials, B);
    } else if (V.v32 && A->sl_d16) {
        const ColsD16 cols{A->sl_d16};
        if (d.f32)
            NN_DISPATCH_W(A->wmax, (k_trial<WM, float, float, ColsD16>), P.nb, P, A->sl_off, cols,
                          V.v32, c, d.f32, t, g, mask, ks, ctx->partials, B);
        else
            NN_DISPATCH_W(A->wmax, (k_trial<WM, float, double, ColsD16>), P.nb, P, A->sl_off, cols,
                          V.v32, c, d.f64, t, g, mask, ks, ctx->partials, B);
    } else if (V.v32) {
        const ColsI32 cols{A->sl_col};
        if (d.f32)
            NN_DISPATCH_W(A->wmax, (k_trial<WM, float, float, ColsI32>), P.nb, P, A->sl_off, cols,
                          V.v32, c, d.f32, t, g, mask, ks, ctx->partials, B);
        else
            NN_DISPATCH_W(A->wmax, (k_trial<WM, float, double, ColsI32>), P.nb, P, A->sl_off, cols,
                          V.v32, c, d.f64, t, g, mask, ks, ctx->partials, B);
    } else if (V.v64p && A->d16p) {
        const ColsD16P cols{A->d16p};
        if (d.f32)
            NN_DISPATCH_W(A->wmax, (k_trial<WM, double, float, ColsD16P>), P.nb, P, A->sl_off, cols,
                          V.v64p, c, d.f32, t, g, mask, ks, ctx->partials, B);
        else
            NN_DISPATCH_W(A->wmax, (k_trial<WM, double, double, ColsD16P>), P.nb, P, A->sl_off, cols,
                          V.v64p, c, d.f64, t, g, mask, ks, ctx->partials, B);
    } else {
        const ColsI32 cols{A->sl_col};
        if (d.f32)
            NN_DISPATCH_W(A->wmax, (k_trial<WM, double, float, ColsI32>), P.nb, P, A->sl_off, cols,
                          V.v64, c, d.f32, t, g, mask, ks, ctx->partials, B);
        else
            NN_DISPATCH_W(A->wmax, (k_trial<WM, double, double, ColsI32>), P.nb, P, A->sl_off, cols,
                          V.v64, c, d.f64, t, g, mask, ks, ctx->partials, B);
    }
}

void launch_ladder(nn_ctx *ctx, const nn_matrix *A, const Vals &V, const double *c,
                   const double *g, const double *t, double *const *ks, Box B)
{
    // 3 kLadder accumulators per lane: one 1024-thread block per CU
    Part P = make_part(A->n, kLadderBlocks);
    Ladder L;
    for (int k = 0; k < kLadder; k++) {
        L.t[k] = t[k];
        L.ks[k] = ks[k];
    }
    if (V.v32q && A->d16q)
        NN_DISPATCH_W(A->wmax, (k_ladder<WM, float, ColsD16Q>), P.nb, P, A->sl_off,
                      ColsD16Q{A->d16q}, V.v32q, c, g, L, B, ctx->partials);
    else if (V.v32 && A->sl_d16)
        NN_DISPATCH_W(A->wmax, (k_ladder<WM, float, ColsD16>), P.nb, P, A->sl_off,
                      ColsD16{A->sl_d16}, V.v32, c, g, L, B, ctx->partials);
    else if (V.v32)
        NN_DISPATCH_W(A->wmax, (k_ladder<WM, float, ColsI32>), P.nb, P, A->sl_off,
                      ColsI32{A->sl_col}, V.v32, c, g, L, B, ctx->partials);
    else if (V.v64p && A->d16p)
        NN_DISPATCH_W(A->wmax, (k_ladder<WM, double, ColsD16P>), P.nb, P, A->sl_off,
                      ColsD16P{A->d16p}, V.v64p, c, g, L, B, ctx->partials);
    else
        NN_DISPATCH_W(A->wmax, (k_ladder<WM, double, ColsI32>), P.nb, P, A->sl_off,
                      ColsI32{A->sl_col}, V.v64, c, g, L, B, ctx->partials);
}

void launch_apply(nn_ctx *ctx, int64_t n, double *c, Dir d, double t, Box B)
{
    Part P = make_part(n);
    if (d.f32) k_apply<float><<<P.nb, kBlock, 0, ctx->stream>>>(P, c, d.f32, t, B);
    else k_apply<double><<<P.nb, kBlock, 0, ctx->stream>>>(P, c, d.f64, t, B);
}

void launch_resid(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *c,
                  const double *f)
{
    Part P = make_part(A->n);
    NN_DISPATCH_W(A->wmax, (k_resid<WM, ColsI32>), P.nb, P, A->sl_off, ColsI32{A->sl_col}, vals, c,
                  f, ctx->partials);
}

void launch_add(nn_ctx *ctx, int64_t n, double *c, const double *w)
{
    Part P = make_part(n);
    k_add<double><<<P.nb, kBlock, 0, ctx->stream>>>(P, c, w);
}

void launch_cg_setup(nn_ctx *ctx, const nn_matrix *A, const double *diag, const double *c,
                     double *g, const double *ks, bool f32, Box B, int face,
                     const Cheb *ch)
{
    Part P = make_part(A->n);
    Workspace &W = ctx->ws;
    const double it = ch ? 1.0 / ch->theta : 0.0;
    if (f32)
        k_cg_setup<float><<<P.nb, kBlock, 0, ctx->stream>>>(
            P, A->rowptr, diag, c, g, ks, W.mask, W.dm32, W.r32, W.z32, W.p32, W.q32, W.w32,
            ctx->partials, ctx->scal, B, face, ch ? W.cres32 : nullptr,
            ch ? W.cdz32[0] : nullptr, ch ? W.cdz32[1] : nullptr, it);
    else
        k_cg_setup<double><<<P.nb, kBlock, 0, ctx->stream>>>(
            P, A->rowptr, diag, c, g, ks, W.mask, W.dm, W.r, W.z, W.p0, W.q, W.w, ctx->partials,
            ctx->scal, B, face, ch ? W.cres : nullptr, ch ? W.cdz[0] : nullptr,
            ch ? W.cdz[1] : nullptr, it);
}

void launch_cheb(nn_ctx *ctx, const nn_matrix *A, const Vals &V, const Cheb &ch, int step,
                 int slot)
{
    Part P = make_part(A->n);
    Workspace &W = ctx->ws;
    const double ca = ch.ca[step], cb = ch.cb[step];
    const int last = step == ch.degree - 1 ? 1 : 0;
    const int ip = (step - 1) & 1, in = step & 1;
    if (V.v32 && A->sl_d16) {
        NN_DISPATCH_W(A->wmax, (k_cheb<WM, float, float, ColsD16>), P.nb, P, A->sl_off,
                      ColsD16{A->sl_d16}, V.v32, W.mask, W.dm32, W.r32, W.cres32, W.cdz32[ip],
                      W.cdz32[in], W.z32, ca, cb, last, slot, ctx->partials, ctx->scal);
    } else if (V.v32) {
        NN_DISPATCH_W(A->wmax, (k_cheb<WM, float, float, ColsI32>), P.nb, P, A->sl_off,
                      ColsI32{A->sl_col}, V.v32, W.mask, W.dm32, W.r32, W.cres32, W.cdz32[ip],
                      W.cdz32[in], W.z32, ca, cb, last, slot, ctx->partials, ctx->scal);
    } else {
        NN_DISPATCH_W(A->wmax, (k_cheb<WM, double, double, ColsI32>), P.nb, P, A->sl_off,
                      ColsI32{A->sl_col}, V.v64, W.mask, W.dm, W.r, W.cres, W.cdz[ip], W.cdz[in],
                      W.z, ca, cb, last, slot, ctx->partials, ctx->scal);
    }
}

void launch_gersh(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *diag)
{
    Part P = make_part(A->n);
    k_gersh<<<P.nb, kBlock, 0, ctx->stream>>>(P, A->sl_off, vals, diag, ctx->partials);
}

template <bool TR>
static void cg_spmv_tr(nn_ctx *ctx, const nn_matrix *A, const Vals &V, int j, int max_it,
                       double rtol)
{
    Part P = make_part(A->n);
    Workspace &W = ctx->ws;
    if (V.v32q && A->d16q) {
        NN_DISPATCH_W(A->wmax, (k_cg_spmv<WM, float, float, ColsD16Q, TR>), P.nb, P, A->sl_off,
                      ColsD16Q{A->d16q}, V.v32q, W.mask, W.z32, W.p32, W.q32, W.w32,
                      ctx->partials, ctx->scal, j, max_it, rtol * rtol);
    } else if (V.v32 && A->sl_d16) {
        NN_DISPATCH_W(A->wmax, (k_cg_spmv<WM, float, float, ColsD16, TR>), P.nb, P, A->sl_off,
                      ColsD16{A->sl_d16}, V.v32, W.mask, W.z32, W.p32, W.q32, W.w32,
                      ctx->partials, ctx->scal, j, max_it, rtol * rtol);
    } else if (V.v32) {
        NN_DISPATCH_W(A->wmax, (k_cg_spmv<WM, float, float, ColsI32, TR>), P.nb, P, A->sl_off,
                      ColsI32{A->sl_col}, V.v32, W.mask, W.z32, W.p32, W.q32, W.w32,
                      ctx->partials, ctx->scal, j, max_it, rtol * rtol);
    } else if (V.v64p && A->d16p) {
        NN_DISPATCH_W(A->wmax, (k_cg_spmv<WM, double, double, ColsD16P, TR>), P.nb, P, A->sl_off,
                      ColsD16P{A->d16p}, V.v64p, W.mask, W.z, W.p0, W.q, W.w, ctx->partials,
                      ctx->scal, j, max_it, rtol * rtol);
    } else {
        NN_DISPATCH_W(A->wmax, (k_cg_spmv<WM, double, double, ColsI32, TR>), P.nb, P, A->sl_off,
                      ColsI32{A->sl_col}, V.v64, W.mask, W.z, W.p0, W.q, W.w, ctx->partials,
                      ctx->scal, j, max_it, rtol * rtol);
    }
}

void launch_cg_spmv(nn_ctx *ctx, const nn_matrix *A, const Vals &V, int j, int max_it, double rtol,
                    bool tr)
{
    if (tr) cg_spmv_tr<true>(ctx, A, V, j, max_it, rtol);
    else cg_spmv_tr<false>(ctx, A, V, j, max_it, rtol);
}

template <bool TR>
static void cg_update_tr(nn_ctx *ctx, int64_t n, int j, bool f32, const Cheb *ch, double delta2)
{
    Part P = make_part(n);
    Workspace &W = ctx->ws;
    const double it = ch ? 1.0 / ch->theta : 0.0;
    if (f32)
        k_cg_update<float, TR><<<P.nb, kBlock, 0, ctx->stream>>>(
            P, W.mask, W.p32, W.q32, W.dm32, W.w32, W.r32, W.z32, ctx->partials, ctx->scal, j,
            ch ? W.cres32 : nullptr, ch ? W.cdz32[0] : nullptr, it, delta2);
    else
        k_cg_update<double, TR><<<P.nb, kBlock, 0, ctx->stream>>>(
            P, W.mask, W.p0, W.q, W.dm, W.w, W.r, W.z, ctx->partials, ctx->scal, j,
            ch ? W.cres : nullptr, ch ? W.cdz[0] : nullptr, it, delta2);
}

void launch_cg_update(nn_ctx *ctx, int64_t n, int j, bool f32, const Cheb *ch, double delta2)
{
    if (std::isfinite(delta2)) cg_update_tr<true>(ctx, n, j, f32, ch, delta2);
    else cg_update_tr<false>(ctx, n, j, f32, ch, delta2);
}

void launch_breakpoint(nn_ctx *ctx, int64_t n, const double *c, Dir w, const double *g, Box B)
{
    Part P = make_part(n);
    if (w.f32)
        k_breakpoint<float><<<P.nb, kBlock, 0, ctx->stream>>>(P, c, w.f32, g, ctx->partials, B);
    else
        k_breakpoint<double><<<P.nb, kBlock, 0, ctx->stream>>>(P, c, w.f64, g, ctx->partials, B);
}

void launch_quad_f32(nn_ctx *ctx, const nn_matrix *A, const float *src, float *dst)
{
    Part P = make_part(A->n);
    k_quad<float><<<P.nb, kBlock, 0, ctx->stream>>>(P, A->sl_off, src, dst);
}

void launch_quad_d16(nn_ctx *ctx, const nn_matrix *A, const short *src, short *dst)
{
    Part P = make_part(A->n);
    k_quad<short><<<P.nb, kBlock, 0, ctx->stream>>>(P, A->sl_off, src, dst);
}

void launch_pair_f64(nn_ctx *ctx, const nn_matrix *A, const double *src, double *dst)
{
    Part P = make_part(A->n);
    k_pair<double><<<P.nb, kBlock, 0, ctx->stream>>>(P, A->sl_off, src, dst);
}

void launch_pair_d16(nn_ctx *ctx, const nn_matrix *A, const short *src, short *dst)
{
    Part P = make_part(A->n);
    k_pair<short><<<P.nb, kBlock, 0, ctx->stream>>>(P, A->sl_off, src, dst);
}

void launch_to_f32(nn_ctx *ctx, int64_t m, const double *a, float *b)
{
    int64_t nb = (m + kBlock - 1) / kBlock;
    if (nb > 2048) nb = 2048;
    if (nb < 1) nb = 1;
    k_to_f32<<<(int)nb, kBlock, 0, ctx->stream>>>(m, a, b);
}

void launch_active(nn_ctx *ctx, int64_t n, const double *c, uint8_t *active, Box B)
{
    Part P = make_part(n);
    k_active<<<P.nb, kBlock, 0, ctx->stream>>>(P, c, active, B);
}

void launch_axpby_vals(nn_ctx *ctx, int64_t nnz, const double *m, double dt, const double *k,
                       double *out)
{
    int64_t nb = (nnz + kBlock - 1) / kBlock;
    if (nb > 2048) nb = 2048;
    if (nb < 1) nb = 1;
    k_vals_mdt_plus_k<<<(int)nb, kBlock, 0, ctx->stream>>>(nnz, m, dt, k, out);
}

void launch_sell_d16(nn_ctx *ctx, const nn_matrix *A, short *sd)
{
    Part P = make_part(A->n);
    k_sell_d16<<<P.nb, kBlock, 0, ctx->stream>>>(P, A->sl_off, A->sl_col, sd, ctx->partials);
}

void launch_diag(nn_ctx *ctx, const nn_matrix *A, const double *vals, double *diag)
{
    Part P = make_part(A->n);
    k_diag<<<P.nb, kBlock, 0, ctx->stream>>>(P, A->sl_off, A->sl_col, vals, diag);
}

void launch_csr_to_sell(nn_ctx *ctx, nn_matrix *A, const double *csr_val, const double *csr_mval)
{
    Part P = make_part(A->n);
    k_csr_to_sell<<<P.nb, kBlock, 0, ctx->stream>>>(P, A->rowptr, A->col, csr_val, csr_mval,
                                                    A->sl_off, A->sl_col, A->val, A->mval);
    k_sell_tail<<<1, kBlock, 0, ctx->stream>>>((int)A->n, P.nslices, A->sl_off, A->sl_col, A->val,
                                               A->mval);
}

}  // namespace nnqp
