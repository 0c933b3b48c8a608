// Active-set projected-Newton / trust-region solver for
//     min 1/2 c.Kc - c.f  subject to  lo <= c <= hi
// (arXiv:1506.08435 Sec. 2.1.3, eq. non-negative: [0, inf); Sec. 2.2.2,
// eq. Eq:non-negative and the DMP Remark of Sec. 5: [c_min, c_max]), in the
// manner of TRON (Lin & More 1999), which the paper uses through TAO
// (Sec. 3.1, Sec. 5.1).  P below is the projection on [lo, hi].
//
// Outer iteration k (all vector work in kernels.hip; the host only sequences
// launches and reads a few scalars):
//   1. g = K c - f and the projected-gradient norm; stop at ||pg|| <= tol ||f||.
//   2. Cauchy point: projected search c(t) = P(c - t g) with the sufficient
//      decrease test q(c(t)) - q(c) <= mu0 g.(c(t) - c); t starts from the
//      previous iteration's value and is extrapolated (x10) while the test
//      holds, or interpolated (x0.1) until it holds.  Each trial is one
//      project-on-gather SpMV that returns g.s and s.Ks.
//   3. Free face at the Cauchy point: every variable except the binding ones,
//      c = lo with g >= 0 or c = hi with g <= 0 (a zero gradient counts as
//      binding).  Jacobi-PCG on
//      K_FF w = -g_F from w = 0 until ||r|| <= inner_rtol ||g_F|| (TRON's
//      inner tolerance, Sec. 5.1 TRON1/2/3), all scalars kept on the device.
//      With a finite trust radius the CG iterate is kept inside the ball of
//      the radius left after the steps already taken in this outer iteration
//      (Steihaug: the step that would leave it stops on its boundary).
//   4. Projected search along w from the Cauchy point: if no free variable
//      crosses a bound for a unit step the step is taken without a matrix pass
//      (CG from zero guarantees sufficient decrease along its own iterate);
//      otherwise P(c + t w) is tried for t = 1, 1/2, ... down to the first
//      breakpoint, where the step is again safe.
//   5. Subspace loop (TRON): when the search stopped on a new face (a free
//      variable reached its bound) and the CG did not stop on the trust-region
//      boundary, steps 3-4 repeat from the new point on its face: a fresh
//      gradient, no new Cauchy step, and the variables at a bound held there
//      (the CG face is the rows strictly inside the bounds, so it only
//      shrinks); until one of these fails or the projected gradient has
//      fallen to inner_rtol of its value at the Cauchy point.  Then the outer
//      iteration ends.
//   6. Trust region: the quadratic model is the objective, so the ratio of
//      actual to predicted reduction is one; the radius (unbounded unless the
//      caller gives one) grows by 4x whenever the outer iteration's step
//      reaches it.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "nnqp_internal.hpp"

namespace nnqp {

namespace {
constexpr double kMu0 = 0.01;       // sufficient-decrease constant
constexpr double kExtrap = 10.0;    // Cauchy extrapolation factor
constexpr double kInterp = 0.1;     // Cauchy interpolation factor
constexpr double kBack = 0.5;       // projected-search backtracking factor
constexpr int kMaxTrials = 60;
constexpr int kMaxSubspace = 100;   // subspace steps per outer iteration

struct Bytes {
    double n, nnz;
    double spmv() const { return 4.0 * (n + 1) + 12.0 * nnz + 16.0 * n; }
};
}  // namespace

// Chebyshev preconditioner set-up: lmax = Gershgorin bound of D^-1 A (valid
// for every face, a principal submatrix), interval [lmax / 30, lmax], the
// coefficients of the Chebyshev iteration (Saad, Iterative Methods for Sparse
// Linear Systems, Sec. 12.3), and its work vectors.  The polynomial q with
// z = q(D^-1 A) D^-1 r satisfies 1 - lambda q(lambda) = T_k(.)/T_k(sigma) in
// (-1, 1) on (0, lmax], so q > 0 there and the preconditioner is SPD.
nn_status cheb_prepare(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *diag,
                       int degree, Cheb *ch)
{
    *ch = Cheb();
    if (degree <= 1) return NN_OK;
    constexpr double kRatio = 30.0;
    Workspace &W = ctx->ws;
    const int64_t n = A->n;
    if (W.cheb_cap < n) {
        double **dv[] = {&W.cres, &W.cdz[0], &W.cdz[1]};
        float **fv[] = {&W.cres32, &W.cdz32[0], &W.cdz32[1]};
        for (double **v : dv) dev_free(ctx->al, *v), *v = nullptr;
        for (float **v : fv) dev_free(ctx->al, *v), *v = nullptr;
        W.cheb_cap = 0;
        for (double **v : dv)
            if (dev_malloc(ctx->al, v, sizeof(double) * std::max<int64_t>(n, 1)) != hipSuccess)
                return fail(ctx, NN_EOOM, "Chebyshev vectors");
        for (float **v : fv)
            if (dev_malloc(ctx->al, v, sizeof(float) * std::max<int64_t>(n, 1)) != hipSuccess)
                return fail(ctx, NN_EOOM, "Chebyshev vectors");
        W.cheb_cap = std::max<int64_t>(n, 1);
    }
    launch_gersh(ctx, A, vals, diag);
    static const int kMaxOp[1] = {OP_MAX};
    double lmax = 0.0;
    nn_status rc = host_reduce(ctx, n, 1, kMaxOp, &lmax);
    if (rc != NN_OK) return rc;
    if (!(lmax > 0.0) || !std::isfinite(lmax))
        return fail(ctx, NN_ENONFINITE, "no finite spectral bound for the Chebyshev preconditioner");
    const double lmin = lmax / kRatio;
    ch->degree = degree;
    ch->theta = 0.5 * (lmax + lmin);
    ch->delta = 0.5 * (lmax - lmin);
    const double sigma = ch->theta / ch->delta;
    double rho = 1.0 / sigma;
    for (int i = 1; i < degree; i++) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        ch->ca[i] = rn * rho;
        ch->cb[i] = 2.0 * rn / ch->delta;
        rho = rn;
    }
    return NN_OK;
}

// One synchronisation for the gradient report (5 values, host slot) and the
// Cauchy ladder (3 kLadder values from SLOT_U0 on); both combined in block order.
static nn_status read_grad_and_ladder(nn_ctx *ctx, int64_t n, double *grad, double *ladder)
{
    const Part P = make_part(n), PL = make_part(n, kLadderBlocks);
    double *h = ctx->h_multi;
    const size_t ng = (size_t)4 * kMaxBlocks + P.nb;
    const size_t nl = (size_t)(3 * kLadder - 1) * kMaxBlocks + PL.nb;
    NN_HIP_TRY(ctx, hipMemcpyAsync(h, ctx->partials, sizeof(double) * ng, hipMemcpyDeviceToHost,
                                   ctx->stream));
    const double *lsrc = ctx->partials + (size_t)SLOT_U0 * kMaxRed * kMaxBlocks;
    NN_HIP_TRY(ctx, hipMemcpyAsync(h + (size_t)5 * kMaxBlocks, lsrc, sizeof(double) * nl,
                                   hipMemcpyDeviceToHost, ctx->stream));
    NN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    static const int kGradOps[5] = {OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM};
    for (int k = 0; k < 5; k++) {
        const int op = kGradOps[k];
        double a = op == OP_SUM ? 0.0 : (op == OP_MIN ? INFINITY : -INFINITY);
        for (int b = 0; b < P.nb; b++) {
            const double v = h[(size_t)k * kMaxBlocks + b];
            a = op == OP_SUM ? a + v : (op == OP_MIN ? std::fmin(a, v) : std::fmax(a, v));
        }
        grad[k] = a;
    }
    for (int k = 0; k < 3 * kLadder; k++) {
        double a = 0.0;
        for (int b = 0; b < PL.nb; b++) a += h[(size_t)(5 + k) * kMaxBlocks + b];
        ladder[k] = a;
    }
    return NN_OK;
}

nn_status solve_impl(nn_ctx *ctx, const nn_matrix *A, const double *vals, const float *vals32,
                     const float *vals32q, const double *vals64p, const double *diag,
                     const double *f, const nn_opts *o, double *c, uint8_t *active, nn_stats *st)
{
    const int64_t n = A->n;
    nn_stats S;
    std::memset(&S, 0, sizeof(S));
    Box box;
    box.lo = o->lower;
    box.hi = o->upper;
    NN_HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    auto finish = [&](nn_status rc) -> nn_status {
        if (active && n > 0) launch_active(ctx, n, c, active, box);
        (void)hipEventRecord(ctx->ev1, ctx->stream);
        hipError_t e = hipEventSynchronize(ctx->ev1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        S.seconds = ms * 1e-3;
        prof_collect(ctx);
        if (e != hipSuccess) rc = fail(ctx, NN_EHIP, hipGetErrorString(e));
        S.status = (int32_t)rc;
        if (st) *st = S;
        return rc;
    };
    if (n == 0) return finish(NN_OK);
    nn_status rc = ensure_workspace(ctx, n);
    if (rc != NN_OK) return rc;
    Workspace &W = ctx->ws;
    DevScalars &H = *ctx->h_scal;
    const Bytes B{(double)n, (double)A->nnz};
    const double tol = o->tol;
    // Mixed precision: the searches and the inner CG use float32 values (and
    // float32 CG vectors); the gradient g = K c - f that decides convergence,
    // the KKT report and all reductions stay float64, so the fixed point is
    // the float64 KKT point.
    const bool mixed = vals32 != nullptr;
    Vals VS;
    if (mixed) {
        VS.v32 = vals32;
        VS.v32q = (vals32q && A->d16q) ? vals32q : nullptr;
    } else {
        VS.v64 = vals;
        VS.v64p = (vals64p && A->d16p) ? vals64p : nullptr;
    }
    const double vb = mixed ? 4.0 : 8.0;                  // bytes per vector entry in CG
    // index bytes of the search and CG passes: int16 column offsets when the
    // pass reads them (float32 values, or the paired float64 layout)
    const double ib = ((mixed && A->sl_d16) || VS.v64p) ? 2.0 : 4.0;
    const double spmv_s = 4.0 * (n + 1) + (ib + vb) * A->nnz + 16.0 * n;
    const double spmv_csr = spmv_s + (4.0 - ib) * A->nnz;   // 4-byte column indices
    Dir dir_g, dir_w;
    dir_g.f64 = W.g;
    if (mixed) dir_w.f32 = W.w32;
    else dir_w.f64 = W.w;

    static const int kInitOps[4] = {OP_SUM, OP_MAX, OP_SUM, OP_SUM};
    static const int kTrialOps[3] = {OP_SUM, OP_SUM, OP_SUM};
    static const int kBrkOps[3] = {OP_MIN, OP_SUM, OP_SUM};
    double red[kMaxRed];

    // ---- start point and load statistics
    prof_begin(ctx, KC_OTHER, 16.0 * n);
    // the start value is projected on the bounds
    const double c0v = std::min(std::max(o->c0_value, box.lo), box.hi);
    launch_init(ctx, n, c, f, o->c0_mode == 1 ? 1 : 0, c0v, box);
    prof_end(ctx);
    if ((rc = host_reduce(ctx, n, 4, kInitOps, red)) != NN_OK) return rc;
    S.bytes_moved += 16.0 * n;
    const double normf = std::sqrt(red[0]), fmax = red[1];
    S.norm_f = normf;
    if (red[2] != 0.0 || red[3] != 0.0)
        return finish(fail(ctx, NN_ENONFINITE, "non-finite value in f or the initial c"));
    if (box.lo == 0.0 && !(fmax > 0.0)) {
        // f <= 0 with lower bound 0: c = 0 satisfies c >= 0, g = -f >= 0, c.g = 0.
        NN_HIP_TRY(ctx, hipMemsetAsync(c, 0, sizeof(double) * n, ctx->stream));
        S.n_active = (int32_t)n;
        S.kkt_rel = 0.0;
        return finish(NN_OK);
    }

    Cheb cheb;
    if ((rc = cheb_prepare(ctx, A, vals, diag, o->precond_degree, &cheb)) != NN_OK)
        return finish(rc);
    const Cheb *chp = cheb.degree > 1 ? &cheb : nullptr;
    const int csteps = cheb.degree - 1;   // Chebyshev passes per CG iteration

    double t_cauchy = 1.0;
    double delta = o->delta0 > 0.0 ? o->delta0 : INFINITY;
    const bool tr = std::isfinite(delta);   // CG truncated at the trust-region boundary
    // CG iterations enqueued between convergence reads: a fixed chunk, or
    // (cg_chunk 0) a first chunk of at most 16 sized from the previous inner
    // solve's count, so a short inner solve enqueues fewer launches that find
    // it finished (each returns at once, but still costs a few microseconds)
    const int chunk = o->cg_chunk > 0 ? o->cg_chunk : 16;
    int cg_guess = chunk;   // iterations of the previous inner solve
    nn_status result = NN_EMAXIT;
    bool subspace = false;    // this iteration continues the subspace loop (no Cauchy step)
    int sub_run = 0;          // subspace steps taken in the current outer iteration
    double step_outer = 0.0;  // bound on |c - c_k| over the current outer iteration
    double pg_cauchy = 0.0;   // |pg| on the face of the outer iteration's Cauchy point
    // end of an outer iteration: radius update (exact model: ratio one)
    auto end_outer = [&]() {
        sub_run = 0;
        if (tr && step_outer >= 0.99 * delta) delta *= 4.0;
        step_outer = 0.0;
    };

    static_assert(kLadder == 3, "ladder buffers: ks0, ks1, ks2");
    double *const ladder_ks[kLadder] = {W.ks0, W.ks1, W.ks2};
    for (int outer = 0;; outer++) {
        // ---- 1. gradient and convergence test, with the Cauchy ladder around
        // the previous step length issued behind it (one synchronisation for
        // both; the ladder is unused on the last iteration and skipped on a
        // subspace step)
        // the float64 gradient reads the paired copy when the solve has one
        const double grad_b = (VS.v64p ? spmv_s : B.spmv()) + 16.0 * n;
        prof_begin(ctx, KC_GRAD, grad_b, B.spmv() + 16.0 * n);
        launch_grad(ctx, A, vals, VS.v64p, c, f, W.g, box);
        prof_end(ctx);
        S.spmvs++;
        S.bytes_moved += grad_b;
        // ladder ..., t_c / 10, t_c, 10 t_c, ... around the previous step
        // length, formed as the sequential search forms them (repeated x0.1
        // and x10)
        constexpr int kMid = kLadder / 2;
        double lt[kLadder];
        lt[kMid] = t_cauchy;
        for (int r = kMid - 1; r >= 0; r--) lt[r] = lt[r + 1] * kInterp;
        for (int r = kMid + 1; r < kLadder; r++) lt[r] = lt[r - 1] * kExtrap;
        double lres[3 * kLadder];
        if (subspace) {
            static const int kGradOps[5] = {OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM};
            if ((rc = host_reduce(ctx, n, 5, kGradOps, red)) != NN_OK) return rc;
            // the subspace loop also ends once the projected gradient has
            // fallen to inner_rtol of its value at the Cauchy point (the
            // inner tolerance applied to the whole subspace minimisation);
            // the outer iteration then starts here with its Cauchy step
            const double pgn = std::sqrt(red[0]);
            if (red[1] == 0.0 && pgn > tol * normf && pgn <= o->inner_rtol * pg_cauchy) {
                subspace = false;
                end_outer();
            }
        }
        if (!subspace) {
            prof_begin(ctx, KC_TRIAL, spmv_s + (16.0 + 8.0 * kLadder) * n,
                       spmv_csr + (16.0 + 8.0 * kLadder) * n);
            launch_ladder(ctx, A, VS, c, W.g, lt, ladder_ks, box);
            prof_end(ctx);
            // (after a subspace exit the gradient partials are read again)
            if ((rc = read_grad_and_ladder(ctx, n, red, lres)) != NN_OK) return rc;
        }
        if (red[1] != 0.0) return finish(fail(ctx, NN_ENONFINITE, "non-finite gradient"));
        S.kkt_rel = std::sqrt(red[0]) / normf;
        S.kkt_nat_inf = red[2];
        S.min_c = red[3];
        S.n_active = (int32_t)red[4];
        S.outer_its = outer;
        if (mixed) S.refinements = outer + 1;   // float64 residual evaluations
        if (S.kkt_rel <= tol) {
            result = NN_OK;
            break;
        }
        if (outer >= o->max_outer) {
            fail(ctx, NN_EMAXIT, "outer iteration cap reached");
            break;
        }
        const double *cg_ks = nullptr;   // Cauchy-step product added to g at the CG set-up
        if (subspace) {
            S.subspace_its++;
        } else {
            S.spmvs += kLadder;
            S.cauchy_trials += kLadder;
            S.bytes_moved += spmv_s + (16.0 + 8.0 * kLadder) * n;

            // ---- 2. Cauchy point along the projected steepest-descent path.
            // The decisions are those of the sequential search (start at t_c,
            // extrapolate x10 while the test holds, else interpolate x0.1 until
            // it holds), read off the ladder; a search that leaves the ladder
            // continues with single trials.
            double *best_ks = ladder_ks[kMid];
            auto scratch_for = [&](const double *busy) { return busy == W.ks0 ? W.ks1 : W.ks0; };
            auto trial_cauchy = [&](double t, double *ks, double &gs, double &sks, double &ss) -> nn_status {
                prof_begin(ctx, KC_TRIAL, spmv_s + 16.0 * n, spmv_csr + 16.0 * n);
                launch_trial(ctx, A, VS, c, dir_g, -t, W.g, nullptr, ks, box);
                prof_end(ctx);
                S.spmvs++;
                S.cauchy_trials++;
                S.bytes_moved += spmv_s + 16.0 * n;
                nn_status r2 = host_reduce(ctx, n, 3, kTrialOps, red);
                gs = red[0];
                sks = red[1];
                ss = red[2];
                return r2;
            };
            auto ok_decrease = [&](double gs, double sks, double ss) {
                return gs < 0.0 && gs + 0.5 * sks <= kMu0 * gs && std::sqrt(ss) <= delta;
            };
            auto lg = [&](int k) { return lres[3 * k]; };
            auto lk = [&](int k) { return lres[3 * k + 1]; };
            auto ls = [&](int k) { return lres[3 * k + 2]; };
            double t = lt[kMid], gs = lg(kMid), sks = lk(kMid), ss = ls(kMid);
            if (ok_decrease(gs, sks, ss)) {
                int k = 0;
                bool open_end = true;   // the chain may continue past the ladder
                for (int r = kMid + 1; r < kLadder; r++, k++) {
                    if (!ok_decrease(lg(r), lk(r), ls(r))) {
                        open_end = false;
                        break;
                    }
                    const bool same = lg(r) == gs && lk(r) == sks;
                    t = lt[r];
                    best_ks = ladder_ks[r];
                    gs = lg(r);
                    sks = lk(r);
                    ss = ls(r);
                    if (same) {   // every moving variable has reached its bound
                        open_end = false;
                        break;
                    }
                }
                for (; open_end && k < 20; k++) {
                    double gs2, sks2, ss2;
                    double *ks_try = scratch_for(best_ks);
                    if ((rc = trial_cauchy(t * kExtrap, ks_try, gs2, sks2, ss2)) != NN_OK) return rc;
                    if (!ok_decrease(gs2, sks2, ss2)) break;
                    const bool same = gs2 == gs && sks2 == sks;
                    t *= kExtrap;
                    best_ks = ks_try;
                    gs = gs2;
                    sks = sks2;
                    ss = ss2;
                    if (same) break;
                }
            } else {
                // t <- 0.1 t until the test holds, at most kMaxTrials times, while g.s < 0
                int k = 0, r = kMid - 1;
                for (;;) {
                    if (r >= 0) {
                        t = lt[r];
                        best_ks = ladder_ks[r];
                        gs = lg(r);
                        sks = lk(r);
                        ss = ls(r);
                        r--;
                    } else {
                        t *= kInterp;
                        best_ks = W.ks0;
                        if ((rc = trial_cauchy(t, best_ks, gs, sks, ss)) != NN_OK) return rc;
                    }
                    if (ok_decrease(gs, sks, ss) || !(++k < kMaxTrials && gs < 0.0)) break;
                }
                if (!ok_decrease(gs, sks, ss)) {
                    // no decrease possible along -g at this precision: stationary up to rounding
                    fail(ctx, NN_EMAXIT, "Cauchy search found no decrease (rounding floor)");
                    break;
                }
            }
            t_cauchy = t;
            prof_begin(ctx, KC_OTHER, 24.0 * n);
            launch_apply(ctx, n, c, dir_g, -t, box);
            prof_end(ctx);
            S.bytes_moved += 24.0 * n;
            step_outer = std::sqrt(ss);
            cg_ks = best_ks;
        }

        // ---- 3. masked Jacobi-PCG on the free face of the Cauchy point (or
        // of the current point on a subspace step), inside the radius left
        const double delta_rem = delta - step_outer;
        const double delta2 = tr ? std::max(delta_rem, 0.0) * std::max(delta_rem, 0.0) : INFINITY;
        prof_begin(ctx, KC_OTHER, 40.0 * n);
        launch_cg_setup(ctx, A, diag, c, W.g, cg_ks, mixed, box,
                        subspace ? FACE_INTERIOR : FACE_BINDING, chp);
        prof_end(ctx);
        S.bytes_moved += 88.0 * n;
        for (int st = 1; st <= csteps; st++) launch_cheb(ctx, A, VS, cheb, st, SLOT_U0);
        int it_seen = 0, j_next = 0;
        H.done = tr && !(delta_rem > 0.0) ? 2 : 0;   // no room left: no CG step
        for (int round = 0; !H.done; round++) {
            const size_t mark = ctx->prof_live.size();
            const int this_chunk = o->cg_chunk > 0 || round > 0
                                       ? chunk
                                       : std::max(2, std::min(chunk, cg_guess + 2));
            for (int k = 0; k < this_chunk; k++, j_next++) {
                ctx->prof_seq = k;
                prof_begin(ctx, KC_CG_SPMV, -1.0);
                launch_cg_spmv(ctx, A, VS, j_next, o->max_cg, o->inner_rtol, tr);
                prof_end(ctx);
                prof_begin(ctx, KC_CG_UPDATE, -1.0);
                launch_cg_update(ctx, n, j_next, mixed, chp, delta2);
                prof_end(ctx);
                const int slot = ((j_next + 1) & 1) ? SLOT_U1 : SLOT_U0;
                for (int st = 1; st <= csteps; st++) {
                    prof_begin(ctx, KC_OTHER, -1.0);
                    launch_cheb(ctx, A, VS, cheb, st, slot);
                    prof_end(ctx);
                }
            }
            ctx->prof_seq = -1;
            if ((rc = read_scalars(ctx)) != NN_OK) return rc;
            const int ran = H.it - it_seen;
            // byte model of the launches that did work; the rest exited at once
            const double nf = H.n_free, nzf = H.nnz_free;
            // matrix pass on the free rows (indices 4 or 2 B, values 8 or 4 B), z gathered,
            // p and q read and written (and w read in a trust-region solve); update:
            // p, q, dm, w, r read, w, r, z written
            const double b_spmv = n + 4.0 * nf + (ib + vb) * nzf + (tr ? 6.0 : 5.0) * vb * nf;
            const double b_upd = n + 8.0 * vb * nf + (chp ? 2.0 * vb * nf : 0.0);
            // Chebyshev pass: matrix on the free rows, dz gathered, res and z
            // read and written, dzp, dm, r read, dzn written
            const double b_cheb = n + 4.0 * nf + (ib + vb) * nzf + 8.0 * vb * nf;
            // the paper's CSR model of the same work: a masked SpMV (4-byte
            // columns, rowptr, gathered and written vector) plus the direction
            // update p = z + beta p as its own pass (read r, dinv, p; write p),
            // and the CG update as its unfused operands (read x, p, r, q, dinv;
            // write x, r)
            const double c_spmv = (4.0 + vb) * nzf + (4.0 + 2.0 * vb) * nf + 4.0 * vb * nf;
            const double c_upd = 7.0 * vb * nf;
            for (size_t e = mark; e < ctx->prof_live.size(); e++) {
                ProfEntry &P = ctx->prof_live[e];
                P.valid = P.seq >= 0 && P.seq < ran;   // the chunk's launches that did work
                P.bytes = P.cls == KC_CG_SPMV ? b_spmv : (P.cls == KC_OTHER ? b_cheb : b_upd);
                P.bytes_csr = P.cls == KC_CG_SPMV ? c_spmv : (P.cls == KC_OTHER ? b_cheb : c_upd);
            }
            S.bytes_moved += ran * (b_spmv + b_upd + csteps * b_cheb);
            S.spmvs += ran * (1 + csteps);
            it_seen = H.it;
        }
        S.cg_its += it_seen;
        if (H.done != 2 || it_seen > 0) cg_guess = it_seen;
        // |pg| on the CG face at the Cauchy point: r.r at the CG set-up, kept
        // on the device as rtol^2 r.r in the stop threshold
        if (!subspace && H.done != 2) pg_cauchy = std::sqrt(H.rr_stop) / o->inner_rtol;
        if (H.done == 4) return finish(fail(ctx, NN_ENONFINITE, "non-finite value in CG"));
        if (H.done == 3) return finish(fail(ctx, NN_ENOTSPD, "non-positive curvature in CG"));
        const bool on_boundary = H.done == 2;   // the CG step stopped on the trust region

        // ---- 4. projected search along w
        prof_begin(ctx, KC_OTHER, 24.0 * n);
        launch_breakpoint(ctx, n, c, dir_w, W.g, box);
        prof_end(ctx);
        S.bytes_moved += 24.0 * n;
        if ((rc = host_reduce(ctx, n, 3, kBrkOps, red)) != NN_OK) return rc;
        const double bmin = red[0], gw = red[1], wn = std::sqrt(red[2]);
        bool new_face = false;   // the step reached a bound the CG face did not hold
        if (it_seen > 0 && gw < 0.0 && wn > 0.0) {
            // |w| <= delta_rem up to rounding: the CG kept it in the ball
            double tmax = std::min(1.0, delta_rem / wn);
            double ts = tmax;
            if (bmin < tmax) {
                for (int k = 0; k < kMaxTrials; k++) {
                    prof_begin(ctx, KC_TRIAL, spmv_s + 16.0 * n, spmv_csr + 16.0 * n);
                    launch_trial(ctx, A, VS, c, dir_w, ts, W.g, W.mask, nullptr, box);
                    prof_end(ctx);
                    S.spmvs++;
                    S.search_trials++;
                    S.bytes_moved += spmv_s + 16.0 * n;
                    if ((rc = host_reduce(ctx, n, 3, kTrialOps, red)) != NN_OK) return rc;
                    const double g2 = red[0], s2 = red[1];
                    if (g2 < 0.0 && g2 + 0.5 * s2 <= kMu0 * g2) break;
                    ts *= kBack;
                    if (ts <= bmin) {
                        ts = bmin;   // no bound is crossed: decrease is guaranteed
                        break;
                    }
                }
            }
            if (ts > 0.0) {
                prof_begin(ctx, KC_OTHER, 24.0 * n);
                launch_apply(ctx, n, c, dir_w, ts, box);
                prof_end(ctx);
                S.bytes_moved += 24.0 * n;
                step_outer += ts * wn;
                new_face = bmin <= ts;
            }
        }
        if (o->verbose)
            std::fprintf(stderr,
                         "nnqp outer %3d %s kkt %.3e active %d free %.0f cauchy t %.3g cg %d "
                         "breakpoint %.3g step %.3e%s\n",
                         outer, subspace ? "subspace" : "cauchy  ", S.kkt_rel, S.n_active,
                         H.n_free, t_cauchy, it_seen, bmin, step_outer,
                         on_boundary ? " (trust-region boundary)" : "");
        if (on_boundary) S.radius_stops++;
        // ---- 5. subspace loop: another CG step on the new face, unless the
        // step stopped on the trust-region boundary (or the projected
        // gradient has fallen far enough, tested at the top)
        subspace = o->subspace && new_face && !on_boundary && sub_run < kMaxSubspace &&
                   !(tr && step_outer >= 0.99 * delta);
        if (subspace) {
            sub_run++;
            continue;
        }
        // ---- 6. radius update
        end_outer();
    }
    if (result == NN_OK) ctx->err.clear();
    return finish(result);
}

// Unconstrained Galerkin solve (Sec. 2.1.2, eq. Single_field_formulation):
// K c = f by Jacobi-PCG from c = 0, the baseline the paper runs with CG and a
// block Jacobi preconditioner (Sec. 5.1).  The same CG kernels as the inner
// solve run with every row free; the CG stops at ||r|| <= tol ||f|| on its
// recursive residual, and the report gives the true residual ||K c - f||,
// min c, max c and the number of negative entries (the DMP statistics of
// Table Tab:S5_cube_dmp).
nn_status galerkin_impl(nn_ctx *ctx, const nn_matrix *A, const double *f, const nn_opts *o,
                        double *c, nn_stats *st)
{
    const int64_t n = A->n;
    nn_stats S;
    std::memset(&S, 0, sizeof(S));
    NN_HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    auto finish = [&](nn_status rc) -> nn_status {
        (void)hipEventRecord(ctx->ev1, ctx->stream);
        hipError_t e = hipEventSynchronize(ctx->ev1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        S.seconds = ms * 1e-3;
        prof_collect(ctx);
        if (e != hipSuccess) rc = fail(ctx, NN_EHIP, hipGetErrorString(e));
        S.status = (int32_t)rc;
        if (st) *st = S;
        return rc;
    };
    if (n == 0) return finish(NN_OK);
    nn_status rc = ensure_workspace(ctx, n);
    if (rc != NN_OK) return rc;
    Workspace &W = ctx->ws;
    DevScalars &H = *ctx->h_scal;
    const Bytes B{(double)n, (double)A->nnz};
    static const int kInitOps[4] = {OP_SUM, OP_MAX, OP_SUM, OP_SUM};
    static const int kResidOps[5] = {OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM};
    double red[kMaxRed];

    prof_begin(ctx, KC_OTHER, 16.0 * n);
    const Box unbounded{-INFINITY, INFINITY};
    launch_init(ctx, n, c, f, 0, 0.0, unbounded);   // c = 0; ||f||, non-finite f
    prof_end(ctx);
    if ((rc = host_reduce(ctx, n, 4, kInitOps, red)) != NN_OK) return rc;
    S.bytes_moved += 16.0 * n;
    const double normf = std::sqrt(red[0]);
    S.norm_f = normf;
    if (red[2] != 0.0) return finish(fail(ctx, NN_ENONFINITE, "non-finite value in f"));
    if (normf == 0.0) return finish(NN_OK);   // c = 0 solves K c = 0

    // CG on K w = -g with every row free, then c += w and the true residual.
    // The matrix pass forms K p by the recurrence K p = K z + beta K p_old, so
    // CG's recursive residual drifts from f - K c by rounding; when the true
    // residual misses tol the solve restarts from c on f - K c (residual
    // replacement), at most kMaxRestarts times and while each restart gains.
    constexpr int kMaxRestarts = 8;
    Vals VS;
    VS.v64 = A->val;
    Cheb cheb;
    if ((rc = cheb_prepare(ctx, A, A->val, A->diag, o->precond_degree, &cheb)) != NN_OK)
        return finish(rc);
    const Cheb *chp = cheb.degree > 1 ? &cheb : nullptr;
    const int csteps = cheb.degree - 1;
    const int chunk = o->cg_chunk > 0 ? o->cg_chunk : 16;
    const double b_spmv = n + 4.0 * n + 12.0 * A->nnz + 40.0 * n;
    const double b_upd = n + 64.0 * n;
    double rel = 1.0;   // ||f - K c|| / ||f|| at c = 0
    for (int restart = 0;; restart++) {
        prof_begin(ctx, KC_GRAD, B.spmv() + 16.0 * n);
        launch_grad(ctx, A, A->val, A->val64p, c, f, W.g, unbounded);   // g = K c - f
        prof_end(ctx);
        S.spmvs++;
        S.bytes_moved += B.spmv() + 16.0 * n;
        prof_begin(ctx, KC_OTHER, 40.0 * n);
        launch_cg_setup(ctx, A, A->diag, c, W.g, nullptr, false, unbounded, FACE_ALL, chp);
        prof_end(ctx);
        S.bytes_moved += 88.0 * n;
        for (int st = 1; st <= csteps; st++) launch_cheb(ctx, A, VS, cheb, st, SLOT_U0);
        const double rtol = std::min(0.5, o->tol / rel);
        const int budget = o->max_cg - S.cg_its;
        int it_seen = 0, j_next = 0;
        for (;;) {
            const size_t mark = ctx->prof_live.size();
            for (int k = 0; k < chunk; k++, j_next++) {
                ctx->prof_seq = k;
                prof_begin(ctx, KC_CG_SPMV, -1.0);
                launch_cg_spmv(ctx, A, VS, j_next, budget, rtol);
                prof_end(ctx);
                prof_begin(ctx, KC_CG_UPDATE, -1.0);
                launch_cg_update(ctx, n, j_next, false, chp);
                prof_end(ctx);
                const int slot = ((j_next + 1) & 1) ? SLOT_U1 : SLOT_U0;
                for (int st = 1; st <= csteps; st++) {
                    prof_begin(ctx, KC_OTHER, -1.0);
                    launch_cheb(ctx, A, VS, cheb, st, slot);
                    prof_end(ctx);
                }
            }
            ctx->prof_seq = -1;
            if ((rc = read_scalars(ctx)) != NN_OK) return rc;
            const int ran = H.it - it_seen;
            const double b_cheb = n + 4.0 * n + 12.0 * A->nnz + 64.0 * n;
            const double c_spmv = 12.0 * A->nnz + 52.0 * n, c_upd = 56.0 * n;   // CSR model
            for (size_t e = mark; e < ctx->prof_live.size(); e++) {
                ProfEntry &P = ctx->prof_live[e];
                P.valid = P.seq >= 0 && P.seq < ran;   // the chunk's launches that did work
                P.bytes = P.cls == KC_CG_SPMV ? b_spmv : (P.cls == KC_OTHER ? b_cheb : b_upd);
                P.bytes_csr = P.cls == KC_CG_SPMV ? c_spmv : (P.cls == KC_OTHER ? b_cheb : c_upd);
            }
            S.bytes_moved += ran * (b_spmv + b_upd + csteps * b_cheb);
            S.spmvs += ran * (1 + csteps);
            it_seen = H.it;
            if (H.done) break;
        }
        S.cg_its += it_seen;
        if (H.done == 4) return finish(fail(ctx, NN_ENONFINITE, "non-finite value in CG"));
        if (H.done == 3) return finish(fail(ctx, NN_ENOTSPD, "non-positive curvature in CG"));

        prof_begin(ctx, KC_OTHER, 24.0 * n);
        launch_add(ctx, n, c, W.w);
        prof_end(ctx);
        S.bytes_moved += 24.0 * n;
        prof_begin(ctx, KC_OTHER, B.spmv() + 16.0 * n);
        launch_resid(ctx, A, A->val, c, f);
        prof_end(ctx);
        S.spmvs++;
        S.bytes_moved += B.spmv() + 16.0 * n;
        if ((rc = host_reduce(ctx, n, 5, kResidOps, red)) != NN_OK) return rc;
        if (red[1] != 0.0) return finish(fail(ctx, NN_ENONFINITE, "non-finite solution"));
        const double prev = rel;
        rel = std::sqrt(red[0]) / normf;
        S.kkt_rel = rel;
        S.max_c = red[2];
        S.min_c = red[3];
        S.n_negative = (int32_t)red[4];
        S.refinements = restart;
        if (o->verbose)
            std::fprintf(stderr,
                         "nnqp galerkin pass %d cg %d residual %.3e min c %.6g max c %.6g "
                         "negative %d\n",
                         restart, it_seen, rel, S.min_c, S.max_c, S.n_negative);
        if (rel <= o->tol) break;
        if (S.cg_its >= o->max_cg)
            return finish(fail(ctx, NN_EMAXIT, "CG iteration cap reached"));
        if (restart >= kMaxRestarts || !(rel < 0.5 * prev))
            return finish(fail(ctx, NN_EMAXIT, "true residual stalled above tol (rounding floor)"));
    }
    ctx->err.clear();
    return finish(NN_OK);
}

}  // namespace nnqp
