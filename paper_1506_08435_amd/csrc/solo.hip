// One-workgroup TRON solve for small problems.
//
// A solve of a few thousand rows is bound by launches and host round trips,
// not by bytes: each CG iteration of the multi-block path is two launches of
// a few microseconds, and every Cauchy or search decision waits for the host.
// Here one 512-thread workgroup runs the whole method of solver.hip (same
// steps, constants and tests) inside a single launch: every pass walks the
// problem's 64-row slices with the workgroup's eight wavefronts, every
// reduction is a fixed-order workgroup reduction, and every decision is
// taken by all threads from the same reduced values, so control flow stays
// uniform and the only synchronisation is the workgroup barrier.  The work
// vectors stay in the caches for the sizes this path serves.
//
// The Cauchy search takes its trials one by one in the sequential order of
// the multi-block solver's rule (start at the previous step length,
// extrapolate x10 while the sufficient-decrease test holds, else interpolate
// x0.1 until it holds); the multi-block solver evaluates the same trials three
// at a time, which changes nothing but the cost.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nnqp_internal.hpp"
#include "rows.hpp"

namespace nnqp {

namespace {

constexpr double kMu0 = 0.01;       // sufficient-decrease constant
constexpr double kExtrap = 10.0;    // Cauchy extrapolation factor
constexpr double kInterp = 0.1;     // Cauchy interpolation factor
constexpr double kBack = 0.5;       // projected-search backtracking factor
constexpr int kMaxTrials = 60;

// report of one solve, written by thread 0 of the workgroup
struct SoloOut {
    double kkt_rel, kkt_nat_inf, min_c, norm_f, bytes;
    int outer_its, cg_its, spmvs, n_active, cauchy_trials, search_trials, status, pad;
};

struct SoloProb {
    int n, nsl;
    const int *so;          // [nsl + 1] slice offsets
    const int *sc;          // sliced-ELL columns
    const int *rp;          // CSR row pointers (row lengths for the byte model)
    const double *v;        // sliced-ELL values
    const double *diag;
    const double *f;
    double *c;              // in: start (c0_mode 1); out: solution
    uint8_t *active;        // out or null
    double *g, *w, *r, *z, *p, *q, *ks[2], *dm;
    uint8_t *mask;
    SoloOut *out;
};

struct SoloOpts {
    double tol, rtol2, c0v;
    int c0_mode, max_outer, max_cg;
};

// The workgroup: 512 threads, eight wavefronts (two per SIMD), so a
// wavefront may hold up to 256 registers and keep many slices in flight.
constexpr int kSoloBlock = 512;
constexpr int kSoloWaves = kSoloBlock / 64;
// Vectors in LDS: problems up to kSoloLdsRows rows keep c, g, z and w there
// (4 x 32 KiB); up to kSoloLdsRows5 rows also q (five vectors of 4,032 rows
// and the reduction buffer fill the 160 KiB of a CU; on the 64^2 square
// 6.31 -> 5.98 ms per solve).
constexpr int kSoloLdsRows = 4096;
constexpr int kSoloLdsRows5 = 4032;
// rows per LDS vector of the variant that keeps nv vectors there
__host__ __device__ constexpr int solo_lds_rows(int nv) { return nv == 5 ? kSoloLdsRows5 : kSoloLdsRows; }

// Reduced values of a pass, the same in every thread: wavefront shuffles,
// then the wavefronts' totals combined in wavefront order (a fixed order, so
// the result is reproducible).
#ifndef NNQP_SOLO_ONE_BARRIER
#define NNQP_SOLO_ONE_BARRIER 1
#endif
#if NNQP_SOLO_ONE_BARRIER
// One barrier per reduction: the totals go to one of two halves of sh,
// alternating between calls (parity, the same in every thread since every
// thread makes the same calls), and every thread combines them itself, so a
// half is written again only two reductions later, after the next barrier.
template <uint32_t OPS, int NV>
__device__ __forceinline__ void wg_reduce(double (&a)[NV], double *sh, int &parity)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_red<OPS, NV>(a);
    double *buf = sh + parity * (kSoloWaves * (kMaxRed + 1));
    parity ^= 1;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) buf[wid * (NV + 1) + k] = a[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const int op = (int)((OPS >> (2 * k)) & 3u);
        double v = buf[k];
#pragma unroll
        for (int w = 1; w < kSoloWaves; w++) v = red_comb(op, v, buf[w * (NV + 1) + k]);
        a[k] = v;
    }
}
#else
template <uint32_t OPS, int NV>
__device__ __forceinline__ void wg_reduce(double (&a)[NV], double *sh, int &)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_red<OPS, NV>(a);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wid * (NV + 1) + k] = a[k];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        const int op = (int)((OPS >> (2 * k)) & 3u);
        double v = sh[k];
#pragma nounroll
        for (int w = 1; w < kSoloWaves; w++) v = red_comb(op, v, sh[w * (NV + 1) + k]);
        sh[kSoloWaves * (NV + 1) + k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) a[k] = sh[kSoloWaves * (NV + 1) + k];
}
#endif

// Rows of the problem, slice by slice over the workgroup's wavefronts:
// body(i, act) for row i = 64 s + lane of every slice s of this wavefront.
template <class Body>
__device__ __forceinline__ void wg_rows(const SoloProb &P, Body body)
{
    const int lane = threadIdx.x & 63, wid = wave_id();
    for (int s = wid; s < P.nsl; s += kSoloWaves) {
        const int i = s * kSlice + lane;
        body(i, i < P.n);
    }
}

// Sliced-ELL product over the workgroup's slices: for each row i with
// mask[i] != 0 (every row without a mask), epi(i, sum over the row's entries
// of v * x(col), pre(i)).  The passes of a small problem are bound by memory
// round trips, not bytes (see wg_spmv).
template <int WMAX>
struct SliceEnt {
    int w;
    int cc[WMAX];
    double vv[WMAX];
};

// The entries of the slice whose first entry and width are off and w: raw
// words under wave-uniform guards (nothing here waits for them).
template <int WMAX>
__device__ __forceinline__ void load_slice(const SoloProb &P, int off, int w, SliceEnt<WMAX> &e)
{
    const int lane = threadIdx.x & 63;
    e.w = w;
#pragma unroll
    for (int k = 0; k < WMAX; k++) {
        if (k < w) {
            e.cc[k] = P.sc[off + k * kSlice + lane];
            e.vv[k] = P.v[off + k * kSlice + lane];
        } else {
            e.cc[k] = 0;
            e.vv[k] = 0.0;
        }
    }
}

// First entry and width of slice s (width 0 past the last slice), from two
// loads that need no guard.
__device__ __forceinline__ void slice_span(const SoloProb &P, int s, int &off, int &w)
{
    const int a = s < P.nsl ? s : P.nsl, b = s + 1 < P.nsl ? s + 1 : P.nsl;
    off = P.so[a];
    w = (P.so[b] - off) >> 6;
}

// Slices a wavefront loads ahead of the one it sums (slices up to 8 wide;
// wider ones one ahead, their entries take more registers).  On the 64^2
// square (3,969 rows, float64): one ahead 6.14 ms per solve, two 6.44 ms,
// three 6.66 ms.
#ifndef NNQP_SOLO_AHEAD
#define NNQP_SOLO_AHEAD 1
#endif

// mask: the free-row flags (null: every row).  A wavefront loads the slice
// offsets D + 1 slices ahead and the entries, own-row values and flags of the
// next D slices before it gathers and sums the current one; the own-row loads
// take a row every vector has (row 0 past the end) and keep the raw flag, so
// no load of a later slice is waited for before the current slice's sum.
template <int WMAX, class Pre, class X, class Epi>
__device__ __forceinline__ void wg_spmv(const SoloProb &P, const uint8_t *__restrict__ mask,
                                        Pre pre, X x, Epi epi)
{
    using PV = decltype(pre(0));
    constexpr int D = WMAX <= 8 ? NNQP_SOLO_AHEAD : 1;
    static_assert(D >= 1, "at least the next slice is loaded ahead");
    const int lane = threadIdx.x & 63, wid = wave_id();
    struct Own {
        bool in;
        uint8_t flag;
        PV pv;
    };
    auto own = [&](int s) {
        const int row = s * kSlice + lane;
        const bool in = s < P.nsl && row < P.n;
        const int r = in ? row : 0;
        return Own{in, mask ? mask[r] : (uint8_t)1, pre(r)};
    };
    SliceEnt<WMAX> ent[D + 1];
    Own ow[D + 1];
    int off, w;
#pragma unroll
    for (int t = 0; t < D; t++) {
        slice_span(P, wid + t * kSoloWaves, off, w);
        load_slice<WMAX>(P, off, w, ent[t]);
        ow[t] = own(wid + t * kSoloWaves);
    }
    slice_span(P, wid + D * kSoloWaves, off, w);   // the span of the next slice to load
    for (int s = wid; s < P.nsl; s += kSoloWaves) {
        int off2, w2;
        slice_span(P, s + (D + 1) * kSoloWaves, off2, w2);
        load_slice<WMAX>(P, off, w, ent[D]);
        ow[D] = own(s + D * kSoloWaves);
        const SliceEnt<WMAX> &cur = ent[0];
        const bool act_c = ow[0].in && ow[0].flag != 0;
        if (__ballot(act_c) != 0) {
            // every gather issued before the first product is added: a slot
            // past the slice's width has column 0 (a valid row) and its
            // product is not added (a select, the same fused multiply-adds in
            // the same order as a guarded sum)
            double xv[WMAX];
#pragma unroll
            for (int k = 0; k < WMAX; k++) xv[k] = x(cur.cc[k]);
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < WMAX; k++) {
                const double y = __builtin_fma(cur.vv[k], xv[k], acc);
                acc = k < cur.w ? y : acc;
            }
            if (cur.w > WMAX) {   // slices wider than the unrolled part
                int o, ww;
                slice_span(P, s, o, ww);
                for (int k = WMAX; k < ww; k++) {
                    const int e = o + k * kSlice + lane;
                    acc += P.v[e] * x(P.sc[e]);
                }
            }
            if (act_c) epi(s * kSlice + lane, acc, ow[0].pv);
        }
#pragma unroll
        for (int t = 0; t < D; t++) {
            ent[t] = ent[t + 1];
            ow[t] = ow[t + 1];
        }
        off = off2;
        w = w2;
    }
}

// Rows of the workgroup's slices in two phases, NR slices of a wavefront at a
// time: ld(i) loads a row's operands (i < n), then st(i, vals) computes and
// stores, so the loads of NR slices are in flight together.
template <int NR, class Ld, class St>
__device__ __forceinline__ void wg_rows2(const SoloProb &P, Ld ld, St st)
{
    using LV = decltype(ld(0));
    const int lane = threadIdx.x & 63, wid = wave_id();
    for (int s0 = wid; s0 < P.nsl; s0 += NR * kSoloWaves) {
        LV v[NR];
        bool in[NR];
#pragma unroll
        for (int t = 0; t < NR; t++) {
            const int i = (s0 + t * kSoloWaves) * kSlice + lane;
            in[t] = s0 + t * kSoloWaves < P.nsl && i < P.n;
            v[t] = in[t] ? ld(i) : LV();
        }
#pragma unroll
        for (int t = 0; t < NR; t++)
            if (in[t]) st((s0 + t * kSoloWaves) * kSlice + lane, v[t]);
    }
}

__device__ __forceinline__ bool ok_decrease(double gs, double sks)
{
    return gs < 0.0 && gs + 0.5 * sks <= kMu0 * gs;
}

// The whole solve of one problem by the calling workgroup.  LDSV = 4: the
// four vectors the passes gather (c, g, the CG vector z and the CG step w)
// live in the workgroup's LDS `lv` ([4][kSoloLdsRows]) for the whole solve,
// so a gather costs an LDS access instead of a cache round trip; c is read
// from and written back to global memory at the start and the end.  LDSV =
// 5: q as well ([5][kSoloLdsRows5]).  LDSV = 0: every vector in global memory.
template <int WMAX, int LDSV>
__device__ void solo_solve(const SoloProb &P, const SoloOpts &O, Box B, double *shbuf, double *lv)
{
    int par = 0;   // the half of shbuf the next reduction writes
    const int n = P.n;
    const double dn = n;
    SoloOut S = {};
    int status = NN_EMAXIT;
    double bytes = 0.0;
    const double spmv_b = 4.0 * (dn + 1) + 12.0 * (P.rp[n] - P.rp[0]) + 16.0 * dn;
    constexpr int LR = solo_lds_rows(LDSV);
    double *const C = LDSV ? lv : P.c;
    double *const G = LDSV ? lv + LR : P.g;
    double *const Z = LDSV ? lv + 2 * LR : P.z;
    double *const Wv = LDSV ? lv + 3 * LR : P.w;
    double *const Q = LDSV == 5 ? lv + 4 * LR : P.q;

    // ---- start point and load statistics
    {
        double a[4];
        red_init<OPS4(OP_SUM, OP_MAX, OP_SUM, OP_SUM), 4>(a);
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double fi = P.f[i];
            a[0] += fi * fi;
            a[1] = fmax(a[1], fi);
            a[2] += isfinite(fi) ? 0.0 : 1.0;
            if (O.c0_mode == 0) {
                C[i] = O.c0v;
            } else {
                const double cv = P.c[i];
                a[3] += isfinite(cv) ? 0.0 : 1.0;
                C[i] = proj_box(cv, B);
            }
        }
        wg_reduce<OPS4(OP_SUM, OP_MAX, OP_SUM, OP_SUM), 4>(a, shbuf, par);
        bytes += 16.0 * dn;
        S.norm_f = sqrt(a[0]);
        if (a[2] != 0.0 || a[3] != 0.0) {
            status = NN_ENONFINITE;
            goto finish;
        }
        if (B.lo == 0.0 && !(a[1] > 0.0)) {
            // f <= 0 with lower bound 0: c = 0 is the minimiser
            for (int i = threadIdx.x; i < n; i += blockDim.x) C[i] = 0.0;
            S.n_active = n;
            status = NN_OK;
            goto finish;
        }
    }
    {
        const double normf = S.norm_f;
        double t_cauchy = 1.0;
        for (int outer = 0;; outer++) {
            // ---- 1. gradient g = K c - f and the KKT report
            double a5[5];
            red_init<OPS5(OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM), 5>(a5);
            wg_spmv<WMAX>(P, nullptr, [&](int i) { return Two{C[i], P.f[i]}; },
                          [&](int j) { return C[j]; }, [&](int i, double s, Two cf) {
                const double gi = s - cf.b, cv = cf.a;
                G[i] = gi;
                const double pg = cv > B.lo ? (cv < B.hi ? gi : fmax(gi, 0.0)) : fmin(gi, 0.0);
                a5[0] += pg * pg;
                a5[1] += (isfinite(gi) && isfinite(cv)) ? 0.0 : 1.0;
                a5[2] = fmax(a5[2], fabs(fmax(cv - B.hi, fmin(gi, cv - B.lo))));
                a5[3] = fmin(a5[3], cv);
                a5[4] += (cv == B.lo || cv == B.hi) ? 1.0 : 0.0;
            });
            wg_reduce<OPS5(OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM), 5>(a5, shbuf, par);
            S.spmvs++;
            bytes += spmv_b + 16.0 * dn;
            if (a5[1] != 0.0) {
                status = NN_ENONFINITE;
                break;
            }
            S.kkt_rel = sqrt(a5[0]) / normf;
            S.kkt_nat_inf = a5[2];
            S.min_c = a5[3];
            S.n_active = (int)a5[4];
            S.outer_its = outer;
            if (S.kkt_rel <= O.tol) {
                status = NN_OK;
                break;
            }
            if (outer >= O.max_outer) break;   // NN_EMAXIT

            // ---- 2. Cauchy point: trials s = P(c - t g) - c, K s into ks[buf]
            auto trial = [&](double t, int buf, double &gs, double &sks) {
                auto sv = [&](int j) {
                    const double cj = C[j];
                    return proj_box(cj - t * G[j], B) - cj;
                };
                double a3[2] = {0.0, 0.0};
                wg_spmv<WMAX>(P, nullptr, [&](int i) { return Two{sv(i), G[i]}; }, sv,
                              [&](int i, double s, Two sg) {
                                  P.ks[buf][i] = s;
                                  a3[0] += sg.b * sg.a;
                                  a3[1] += sg.a * s;
                              });
                wg_reduce<OPS2(OP_SUM, OP_SUM), 2>(a3, shbuf, par);
                gs = a3[0];
                sks = a3[1];
                S.spmvs++;
                S.cauchy_trials++;
                bytes += spmv_b + 16.0 * dn;
            };
            double t = t_cauchy, gs, sks;
            int best = 0;
            trial(t, best, gs, sks);
            if (ok_decrease(gs, sks)) {
                for (int k = 0; k < 20; k++) {
                    double gs2, sks2;
                    trial(t * kExtrap, 1 - best, gs2, sks2);
                    if (!ok_decrease(gs2, sks2)) break;
                    const bool same = gs2 == gs && sks2 == sks;
                    t *= kExtrap;
                    best = 1 - best;
                    gs = gs2;
                    sks = sks2;
                    if (same) break;   // every moving variable has reached its bound
                }
            } else {
                int k = 0;
                for (;;) {
                    t *= kInterp;
                    trial(t, best, gs, sks);
                    if (ok_decrease(gs, sks) || !(++k < kMaxTrials && gs < 0.0)) break;
                }
                if (!ok_decrease(gs, sks)) break;   // rounding floor: NN_EMAXIT
            }
            t_cauchy = t;
            // c = P(c - t g)
            wg_rows(P, [&](int i, bool act) {
                if (act) C[i] = proj_box(C[i] - t * G[i], B);
            });
            bytes += 24.0 * dn;
            __syncthreads();

            // ---- 3. Jacobi-PCG on the free face of the Cauchy point
            double u[4] = {0.0, 0.0, 0.0, 0.0};
            const double *ksb = P.ks[best];
            struct SV {
                double g, ks, c, d;
                int len;
            };
            wg_rows2<4>(P, [&](int i) { return SV{G[i], ksb[i], C[i], P.diag[i], P.rp[i + 1] - P.rp[i]}; },
                        [&](int i, const SV &v) {
                            const double gi = v.g + v.ks;
                            G[i] = gi;
                            const double cv = v.c;
                            const bool fr = !((cv == B.lo && gi >= 0.0) || (cv == B.hi && gi <= 0.0));
                            const double dmi = fr ? 1.0 / v.d : 0.0;
                            const double ri = fr ? -gi : 0.0;
                            const double zi = dmi * ri;
                            P.mask[i] = fr ? 1 : 0;
                            P.dm[i] = dmi;
                            P.r[i] = ri;
                            Z[i] = zi;
                            P.p[i] = 0.0;
                            Q[i] = 0.0;
                            Wv[i] = 0.0;
                            u[0] += ri * zi;
                            u[1] += ri * ri;
                            u[2] += fr ? 1.0 : 0.0;
                            u[3] += fr ? (double)v.len : 0.0;
                        });
            wg_reduce<0u, 4>(u, shbuf, par);
            bytes += 88.0 * dn;
            double rz = u[0], rr = u[1], rz_prev = 0.0;
            const double nf = u[2], nzf = u[3], rr_stop = O.rtol2 * u[1];
            int it = 0;
            bool cg_fail = false;
            for (int j = 0;; j++) {
                if (!isfinite(rz) || !isfinite(rr)) {
                    status = NN_ENONFINITE;
                    cg_fail = true;
                    break;
                }
                if ((j == 0 && (rr == 0.0 || nf == 0.0)) || (j > 0 && rr <= rr_stop) ||
                    j >= O.max_cg || !(rz > 0.0))
                    break;
                const double beta = j == 0 ? 0.0 : rz / rz_prev;
                // p <- z + beta p, q <- K z + beta q on the free rows (K p by linearity)
                double pq[1] = {0.0};
                wg_spmv<WMAX>(P, P.mask, [&](int i) { return Three{P.p[i], Q[i], Z[i]}; },
                              [&](int jj) { return Z[jj]; }, [&](int i, double kz, Three x) {
                                  const double pi = fma(beta, x.a, x.c);
                                  const double qi = fma(beta, x.b, kz);
                                  P.p[i] = pi;
                                  Q[i] = qi;
                                  pq[0] += pi * qi;
                              });
                wg_reduce<0u, 1>(pq, shbuf, par);
                if (!(pq[0] > 0.0 && isfinite(pq[0]))) {
                    status = isfinite(pq[0]) ? NN_ENOTSPD : NN_ENONFINITE;
                    cg_fail = true;
                    break;
                }
                const double alpha = rz / pq[0];
                double a2[2] = {0.0, 0.0};
                struct UV {
                    double r, q, dm, p;
                    int m;
                };
                wg_rows2<4>(P, [&](int i) { return UV{P.r[i], Q[i], P.dm[i], P.p[i], P.mask[i]}; },
                            [&](int i, const UV &v) {
                                if (!v.m) return;
                                const double ri = v.r - alpha * v.q;
                                const double zi = v.dm * ri;
                                Wv[i] += alpha * v.p;
                                P.r[i] = ri;
                                Z[i] = zi;
                                a2[0] += ri * zi;
                                a2[1] += ri * ri;
                            });
                wg_reduce<0u, 2>(a2, shbuf, par);
                rz_prev = rz;
                rz = a2[0];
                rr = a2[1];
                it++;
                S.spmvs++;
                bytes += (dn + 4.0 * nf + 12.0 * nzf + 40.0 * nf) + (dn + 64.0 * nf);
            }
            S.cg_its += it;
            if (cg_fail) break;

            // ---- 4. projected search along w
            double b3[3];
            red_init<OPS3(OP_MIN, OP_SUM, OP_SUM), 3>(b3);
            wg_rows(P, [&](int i, bool act) {
                if (!act) return;
                const double wi = Wv[i], ci = C[i];
                if (wi < 0.0) b3[0] = fmin(b3[0], (ci - B.lo) / (-wi));
                else if (wi > 0.0) b3[0] = fmin(b3[0], (B.hi - ci) / wi);
                b3[1] += G[i] * wi;
                b3[2] += wi * wi;
            });
            wg_reduce<OPS3(OP_MIN, OP_SUM, OP_SUM), 3>(b3, shbuf, par);
            bytes += 24.0 * dn;
            const double bmin = b3[0], gw = b3[1], wn = sqrt(b3[2]);
            if (it > 0 && gw < 0.0 && wn > 0.0) {
                double ts = 1.0;
                if (bmin < 1.0) {
                    for (int k = 0; k < kMaxTrials; k++) {
                        auto sv = [&](int j) {
                            const double cj = C[j];
                            return proj_box(cj + ts * Wv[j], B) - cj;
                        };
                        double a3[2] = {0.0, 0.0};
                        wg_spmv<WMAX>(P, P.mask, [&](int i) { return Two{sv(i), G[i]}; }, sv,
                                      [&](int, double s, Two sg) {
                                          a3[0] += sg.b * sg.a;
                                          a3[1] += sg.a * s;
                                      });
                        wg_reduce<OPS2(OP_SUM, OP_SUM), 2>(a3, shbuf, par);
                        S.spmvs++;
                        S.search_trials++;
                        bytes += spmv_b + 16.0 * dn;
                        if (ok_decrease(a3[0], a3[1])) break;
                        ts *= kBack;
                        if (ts <= bmin) {
                            ts = bmin;   // no bound is crossed: decrease is guaranteed
                            break;
                        }
                    }
                }
                if (ts > 0.0) {
                    wg_rows(P, [&](int i, bool act) {
                        if (act) C[i] = proj_box(C[i] + ts * Wv[i], B);
                    });
                    bytes += 24.0 * dn;
                    __syncthreads();
                }
            }
        }
    }
finish:
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double ci = C[i];
        if (LDSV) P.c[i] = ci;
        if (P.active) P.active[i] = ci == B.lo ? 1 : (ci == B.hi ? 2 : 0);
    }
    if (threadIdx.x == 0) {
        S.status = status;
        S.bytes = bytes;
        *P.out = S;
    }
}

template <int WMAX, int LDSV>
__global__ __launch_bounds__(kSoloBlock) void k_solo(SoloProb P, SoloOpts O, Box B)
{
    __shared__ double shbuf[2 * kSoloWaves * (kMaxRed + 1)];
    if constexpr (LDSV > 0) {
        __shared__ double lv[LDSV * solo_lds_rows(LDSV)];
        solo_solve<WMAX, LDSV>(P, O, B, shbuf, lv);
    } else {
        solo_solve<WMAX, 0>(P, O, B, shbuf, nullptr);
    }
}

}  // namespace

bool solo_eligible(const nn_matrix *A, const nn_opts *o)
{
    return A->n > 0 && A->n < ((int64_t)1 << 31) / kSlice && o->method == NN_TRON &&
           o->precision == NN_FP64 && !(o->delta0 > 0.0) && o->precond_degree <= 1 &&
           o->subspace == 0 && o->verbose == 0;
}

nn_status solo_solve_impl(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *diag,
                          const double *f, const nn_opts *o, double *c, uint8_t *active,
                          nn_stats *st)
{
    const int64_t n = A->n;
    nn_status rc = ensure_workspace(ctx, n);
    if (rc != NN_OK) return rc;
    Workspace &W = ctx->ws;
    SoloProb P;
    P.n = (int)n;
    P.nsl = (int)A->nslices;
    P.so = A->sl_off;
    P.sc = A->sl_col;
    P.rp = A->rowptr;
    P.v = vals;
    P.diag = diag;
    P.f = f;
    P.c = c;
    P.active = active;
    P.g = W.g;
    P.w = W.w;
    P.r = W.r;
    P.z = W.z;
    P.p = W.p0;
    P.q = W.q;
    P.ks[0] = W.ks0;
    P.ks[1] = W.ks1;
    P.dm = W.dm;
    P.mask = W.mask;
    // the report goes through the reduction partials (free between calls)
    P.out = reinterpret_cast<SoloOut *>(ctx->partials);
    SoloOpts O;
    O.tol = o->tol;
    O.rtol2 = o->inner_rtol * o->inner_rtol;
    O.c0v = std::min(std::max(o->c0_value, o->lower), o->upper);
    O.c0_mode = o->c0_mode == 1 ? 1 : 0;
    O.max_outer = o->max_outer;
    O.max_cg = o->max_cg;
    Box box;
    box.lo = o->lower;
    box.hi = o->upper;
    NN_HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    const int lds = n <= kSoloLdsRows5 ? 5 : (n <= kSoloLdsRows ? 4 : 0);
#define NN_SOLO_LAUNCH(WM)                                                                       \
    do {                                                                                         \
        if (lds == 5)                                                                            \
            hipLaunchKernelGGL((k_solo<WM, 5>), dim3(1), dim3(kSoloBlock), 0, ctx->stream, P,    \
                               O, box);                                                          \
        else if (lds == 4)                                                                       \
            hipLaunchKernelGGL((k_solo<WM, 4>), dim3(1), dim3(kSoloBlock), 0, ctx->stream, P,    \
                               O, box);                                                          \
        else                                                                                     \
            hipLaunchKernelGGL((k_solo<WM, 0>), dim3(1), dim3(kSoloBlock), 0, ctx->stream, P,    \
                               O, box);                                                          \
    } while (0)
    if (A->wmax <= 8) NN_SOLO_LAUNCH(8);
    else if (A->wmax <= 16) NN_SOLO_LAUNCH(16);
    else NN_SOLO_LAUNCH(32);
#undef NN_SOLO_LAUNCH
    NN_HIP_TRY(ctx, hipGetLastError());
    SoloOut R;
    NN_HIP_TRY(ctx, hipMemcpyAsync(&R, P.out, sizeof(SoloOut), hipMemcpyDeviceToHost, ctx->stream));
    NN_HIP_TRY(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    NN_HIP_TRY(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    nn_stats S;
    std::memset(&S, 0, sizeof(S));
    S.kkt_rel = R.kkt_rel;
    S.kkt_nat_inf = R.kkt_nat_inf;
    S.min_c = R.min_c;
    S.norm_f = R.norm_f;
    S.outer_its = R.outer_its;
    S.cg_its = R.cg_its;
    S.spmvs = R.spmvs;
    S.n_active = R.n_active;
    S.cauchy_trials = R.cauchy_trials;
    S.search_trials = R.search_trials;
    S.status = R.status;
    S.bytes_moved = R.bytes;
    S.seconds = ms * 1e-3;
    if (st) *st = S;
    switch (R.status) {
    case NN_OK:
        ctx->err.clear();
        return NN_OK;
    case NN_EMAXIT:
        return fail(ctx, NN_EMAXIT, "outer iteration cap or rounding floor reached");
    case NN_ENONFINITE:
        return fail(ctx, NN_ENONFINITE, "non-finite value in the solve");
    case NN_ENOTSPD:
        return fail(ctx, NN_ENOTSPD, "non-positive curvature in CG");
    default:
        return fail(ctx, (nn_status)R.status, "solve failed");
    }
}

}  // namespace nnqp
