// Bounded limited-memory variable-metric (BLMVM) solver for
//     min 1/2 c.Kc - c.f  subject to  lo <= c <= hi
// the gradient-only method the paper runs beside TRON through TAO (Sec. 3.1,
// Sec. 5.1; the objective and gradient callbacks of eq. S3_tao_objective and
// eq. S3_tao_gradient are all it uses).  The method is that of Benson & More
// (2001): an L-BFGS inverse-Hessian approximation H built from the steps s and
// the differences y of projected gradients, search direction d = -H pg, and a
// projected line search.  Here, for the quadratic objective:
//
//   1. Pair pass (one kernel over the rows): pg at the current point, the new
//      y = pg - pg_prev when a step was just taken, and every inner product
//      the compact representation needs (s_j.pg, y_j.pg, s_j.y, y_j.y, s.s).
//   2. Coefficient kernel (one wavefront): accepts the new pair when
//      s.y > 1e-12 |s| |y| (else drops it; a full memory then loses its
//      oldest pair), sets gamma = s.y / y.y, and solves the small triangular
//      systems of the compact form (Byrd, Nocedal & Schnabel 1994)
//          H v = gamma v + S t - gamma Y p,  p = R^-1 S'v,
//          t = R^-T ((D + gamma Y'Y) p - gamma Y'v),
//      R the upper triangle of S'Y and D its diagonal (pairs oldest first).
//   3. Direction pass: d = -H pg from those coefficients, with every
//      component that points out of the box at a bound set to zero (the
//      projection would cancel it for any step), the first bound crossing
//      along d, g.d and d.d.
//   4. Line search: when no bound is crossed up to t = 1, one trial at t = 1
//      gives K d, and the step is the exact minimiser of the quadratic along
//      d (capped at the first crossing); otherwise projected backtracking
//      c(t) = P(c + t d), t = 1, 1/2, ..., until the sufficient-decrease test
//      holds, finishing with the exact step on the segment [0, crossing] if t
//      reaches it.  Each trial is one matrix pass that gathers P(c + t d) and
//      returns the gradient K c(t) - f at the trial point.
//   5. Step: c <- c(t), s stored in the next pair slot, g updated; done by
//      the next iteration's pair pass (one pass over the rows fewer), or by a
//      step kernel when a gradient refresh comes first.
// g is refreshed with a plain gradient pass every 50 iterations that did not
// end on a freshly computed gradient, and before convergence is accepted.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "nnqp_internal.hpp"
#include "rows.hpp"

namespace nnqp {

namespace {

constexpr int kLmMax = 8;                  // pair slots supported
constexpr int kLmNV = 4 * kLmMax + 3;      // values of the pair pass at kLmMax
static_assert(kLmMax * kLmMax <= 64, "one lane per table entry in the coefficient kernel");
constexpr double kLmMu = 0.01;             // sufficient-decrease constant
constexpr double kLmCurv = 1e-12;          // pair acceptance: s.y > kLmCurv |s| |y|
constexpr int kLmRefresh = 50;             // iterations between gradient refreshes
constexpr int kLmMaxTrials = 60;

struct LmState {
    int count;        // stored pairs
    int head;         // slot the next pair is written to
    int pending;      // a step was taken: its s is in slot head, its y is formed next
    int accepted;     // pairs accepted / rejected so far
    int rejected;
    double gamma;     // H0 = gamma I
    double pg2;       // |pg|^2 at the current point
    double nonfinite; // non-finite c or g entries at the current point
    double sy[kLmMax][kLmMax];   // s_a . y_b by slot (used for a older than or equal to b)
    double yy[kLmMax][kLmMax];   // y_a . y_b by slot
    double sc[kLmMax];           // coefficient of s_slot in H pg
    double yc[kLmMax];           // coefficient of y_slot in H pg
    double bmin, gd;             // direction: first bound crossing, g.d
    double gs, sks;              // trial at t = 1: g.s, s.(gn - g)
};

// slot j is live in the pair pass: a stored pair, or the pair being formed
__device__ __forceinline__ bool lm_live(int j, int M, int count, int head, int pending)
{
    const int age = (head - j + M) % M;   // 1 = newest stored pair, ..., M = oldest when full
    return (pending && j == head) || (age >= 1 && age <= count) || (count == M && j == head);
}

// Block total of NV sums (fixed order: butterfly within the wavefront, waves
// in order) stored as this block's partial part[k * kMaxBlocks + block].
template <int NV>
__device__ __forceinline__ void block_sums(double (&a)[NV], double *part)
{
    __shared__ double sh[kWaves][NV];
    const int lane = threadIdx.x & 63, wid = wave_id();
#pragma unroll
    for (int k = 0; k < NV; k++)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) a[k] += __shfl_xor(a[k], o, 64);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wid][k] = a[k];
    __syncthreads();
    for (int k = threadIdx.x; k < NV; k += kBlock) {
        double v = sh[0][k];
        for (int w = 1; w < kWaves; w++) v += sh[w][k];
        part[k * kMaxBlocks + blockIdx.x] = v;
    }
}

// 1. pair pass (see the file comment); values: |pg|^2, #non-finite,
// s_j.pg, y_j.pg, s_j.y, y_j.y (j = 0..M-1 by slot), s.s.
// With `apply` the step of the previous iteration is taken here first (the
// step kernel fused in): c <- P(c + t d), s = c_new - c into slot head,
// g <- g + gscale (gn - g) (gscale = 1: gn itself), and the pair is formed
// from that s.
template <int M>
__global__ __launch_bounds__(kBlock) void kl_pairs(Part P, double *__restrict__ c,
                                                   double *__restrict__ g,
                                                   double *__restrict__ pg,
                                                   double *__restrict__ S,
                                                   double *__restrict__ Y, int64_t ld,
                                                   const LmState *__restrict__ st, Box B,
                                                   double *part, int apply,
                                                   const double *__restrict__ d, double t,
                                                   const double *__restrict__ gn, double gscale)
{
    constexpr int NV = 4 * M + 3;
    const int count = st->count, head = st->head, pending = apply || st->pending;
    bool live[M];
#pragma unroll
    for (int j = 0; j < M; j++) live[j] = lm_live(j, M, count, head, pending);
    double a[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) a[k] = 0.0;
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        double ci = c[i], gi = g[i], sn = 0.0;
        if (apply) {
            const double cn = proj_box(ci + t * d[i], B);
            sn = cn - ci;
            ci = cn;
            gi = gscale == 1.0 ? gn[i] : gi + gscale * (gn[i] - gi);
            c[i] = ci;
            g[i] = gi;
            S[head * ld + i] = sn;
        } else if (pending) {
            sn = S[head * ld + i];
        }
        const double pgi = ci > B.lo ? (ci < B.hi ? gi : fmax(gi, 0.0)) : fmin(gi, 0.0);
        a[0] += pgi * pgi;
        a[1] += (isfinite(ci) && isfinite(gi)) ? 0.0 : 1.0;
        double yn = 0.0;
        if (pending) {
            yn = pgi - pg[i];
            Y[head * ld + i] = yn;
            a[2 + 4 * M] += sn * sn;
        }
        pg[i] = pgi;
#pragma unroll
        for (int j = 0; j < M; j++) {
            if (!live[j]) continue;
            const bool fresh = pending && j == head;
            const double sj = fresh ? sn : S[j * ld + i];
            const double yj = fresh ? yn : Y[j * ld + i];
            a[2 + j] += sj * pgi;
            a[2 + M + j] += yj * pgi;
            if (pending) {
                a[2 + 2 * M + j] += sj * yn;
                a[2 + 3 * M + j] += yj * yn;
            }
        }
    });
    block_sums<NV>(a, part);
}

// 2. coefficient kernel: one wavefront.  The lanes combine the block
// partials (lane-strided sums, then a butterfly: fixed order) and stage the
// S'Y and Y'Y tables in LDS; lane 0 does the small algebra.
template <int M>
__global__ __launch_bounds__(64) void kl_coef(int nb, LmState *st, const double *part, int applied)
{
    constexpr int NV = 4 * M + 3;
    __shared__ double t[NV];
    __shared__ double sy[M][M], yy[M][M];
    const int lane = threadIdx.x;
    // every load is issued before the first use (the state scalars, the
    // tables and the partials), so their latencies overlap
    const int count0 = st->count, head0 = st->head, pend0 = st->pending;
    const double gam0 = st->gamma;
    double tsy = 0.0, tyy = 0.0;
    if (lane < M * M) {
        tsy = st->sy[lane / M][lane % M];
        tyy = st->yy[lane / M][lane % M];
    }
    {
        double acc[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) acc[k] = 0.0;
        // nb <= kMaxBlocks = 512: at most eight blocks per lane
#pragma unroll
        for (int r = 0; r < kMaxBlocks / 64; r++) {
            const int b = lane + 64 * r;
            if (b < nb)
#pragma unroll
                for (int k = 0; k < NV; k++) acc[k] += part[k * kMaxBlocks + b];
        }
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double v = acc[k];
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) t[k] = v;
        }
    }
    if (lane < M * M) {
        sy[lane / M][lane % M] = tsy;
        yy[lane / M][lane % M] = tyy;
    }
    __syncthreads();
    if (lane == 0) {
        int count = count0, head = head0;
        double gam = gam0;
        st->pg2 = t[0];
        st->nonfinite = t[1];
        if (pend0 || applied) {
            const double sny = t[2 + 2 * M + head], yny = t[2 + 3 * M + head], ss = t[2 + 4 * M];
            const bool ok = isfinite(sny) && isfinite(yny) && yny > 0.0 &&
                            sny > kLmCurv * sqrt(ss) * sqrt(yny);
            if (ok) {
                // column `head` of S'Y and Y'Y against every pair that stays
                for (int j = 0; j < M; j++) {
                    if (!lm_live(j, M, count, head, 1)) continue;
                    sy[j][head] = t[2 + 2 * M + j];
                    yy[j][head] = t[2 + 3 * M + j];
                    yy[head][j] = t[2 + 3 * M + j];
                }
                count = count < M ? count + 1 : M;
                head = (head + 1) % M;
                gam = sny / yny;
                st->accepted++;
            } else {
                if (count == M) count = M - 1;   // its oldest pair was overwritten
                st->rejected++;
            }
            st->pending = 0;
        }
        st->count = count;
        st->head = head;
        st->gamma = gam;
        // compact-form coefficients over the pairs, oldest first
        int sl[M];
        double u[M], w[M], p[M], z[M], tp[M];
        for (int k = 0; k < count; k++) {
            sl[k] = (head - count + k + 2 * M) % M;
            u[k] = t[2 + sl[k]];
            w[k] = t[2 + M + sl[k]];
        }
        for (int a = count - 1; a >= 0; a--) {
            double v = u[a];
            for (int b = a + 1; b < count; b++) v -= sy[sl[a]][sl[b]] * p[b];
            p[a] = v / sy[sl[a]][sl[a]];
        }
        for (int a = 0; a < count; a++) {
            double v = sy[sl[a]][sl[a]] * p[a] - gam * w[a];
            for (int b = 0; b < count; b++) v += gam * yy[sl[a]][sl[b]] * p[b];
            z[a] = v;
        }
        for (int a = 0; a < count; a++) {
            double v = z[a];
            for (int b = 0; b < a; b++) v -= sy[sl[b]][sl[a]] * tp[b];
            tp[a] = v / sy[sl[a]][sl[a]];
        }
        double sc[M], yc[M];
        for (int j = 0; j < M; j++) {
            sc[j] = 0.0;
            yc[j] = 0.0;
        }
        for (int a = 0; a < count; a++) {
            sc[sl[a]] = tp[a];
            yc[sl[a]] = -gam * p[a];
        }
        for (int j = 0; j < M; j++) {
            st->sc[j] = sc[j];
            st->yc[j] = yc[j];
        }
    }
    __syncthreads();
    if (lane < M * M) {
        st->sy[lane / M][lane % M] = sy[lane / M][lane % M];
        st->yy[lane / M][lane % M] = yy[lane / M][lane % M];
    }
}

// Line-search summary for the host: combines the direction pass partials
// (SLOT_Q: first crossing, g.d) and the trial's (host slot: g.s, s.(gn - g))
// into the state, so one small copy returns everything.
__global__ __launch_bounds__(64) void kl_summary(int nb, LmState *st, double *partials)
{
    const double *q = slot_ptr(partials, SLOT_Q), *h = slot_ptr(partials, SLOT_HOST);
    double bm = INFINITY, gd = 0.0, gs = 0.0, sks = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) {
        bm = fmin(bm, q[b]);
        gd += q[kMaxBlocks + b];
        gs += h[b];
        sks += h[kMaxBlocks + b];
    }
    for (int o = 32; o >= 1; o >>= 1) {
        bm = fmin(bm, __shfl_xor(bm, o, 64));
        gd += __shfl_xor(gd, o, 64);
        gs += __shfl_xor(gs, o, 64);
        sks += __shfl_xor(sks, o, 64);
    }
    if (threadIdx.x == 0) {
        st->bmin = bm;
        st->gd = gd;
        st->gs = gs;
        st->sks = sks;
    }
}

// drop every stored pair (before the coefficients are formed again)
__global__ void kl_forget(LmState *st) { st->count = 0; }

__global__ void kl_state_init(LmState *st, double gamma)
{
    st->count = 0;
    st->head = 0;
    st->pending = 0;
    st->accepted = 0;
    st->rejected = 0;
    st->gamma = gamma;
}

// 3. direction pass: d = -H pg, outward components at a bound zeroed;
// first crossing (min), g.d, d.d
template <int M>
__global__ __launch_bounds__(kBlock) void kl_dir(Part P, const double *__restrict__ c,
                                                 const double *__restrict__ g,
                                                 const double *__restrict__ pg,
                                                 const double *__restrict__ S,
                                                 const double *__restrict__ Y, int64_t ld,
                                                 const LmState *__restrict__ st, Box B,
                                                 double *__restrict__ d, double *partials)
{
    const int count = st->count, head = st->head;
    const double gam = st->gamma;
    bool live[M];
    double sc[M], yc[M];
#pragma unroll
    for (int j = 0; j < M; j++) {
        live[j] = lm_live(j, M, count, head, 0) && count > 0;
        sc[j] = st->sc[j];
        yc[j] = st->yc[j];
    }
    constexpr uint32_t kOps = OPS3(OP_MIN, OP_SUM, OP_SUM);
    double a[3];
    red_init<kOps, 3>(a);
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        double di = -gam * pg[i];
#pragma unroll
        for (int j = 0; j < M; j++)
            if (live[j]) di -= sc[j] * S[j * ld + i] + yc[j] * Y[j * ld + i];
        const double ci = c[i];
        if ((ci <= B.lo && di < 0.0) || (ci >= B.hi && di > 0.0)) di = 0.0;
        d[i] = di;
        if (di < 0.0) a[0] = fmin(a[0], (ci - B.lo) / (-di));
        else if (di > 0.0) a[0] = fmin(a[0], (B.hi - ci) / di);
        a[1] += g[i] * di;
        a[2] += di * di;
    });
    block_partial<kOps, 3>(a, slot_ptr(partials, SLOT_Q));
}

// 4. trial: gathers c(t) = P(c + t d), writes gn = K c(t) - f; g.s, s.(gn - g), s.s
// with s = c(t) - c
template <int WMAX, class Cols>
__global__ __launch_bounds__(kBlock) void kl_trial(Part P, const int *__restrict__ so, Cols cols,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ c,
                                                   const double *__restrict__ d, double t,
                                                   const double *__restrict__ f,
                                                   const double *__restrict__ g,
                                                   double *__restrict__ gn, Box B,
                                                   double *partials)
{
    auto ct = [&](int j) { return proj_box(c[j] + t * d[j], B); };
    constexpr uint32_t kOps = OPS3(OP_SUM, OP_SUM, OP_SUM);
    double a[3];
    red_init<kOps, 3>(a);
    sell_rows<WMAX>(P, so, cols, v, AllRows(),
                    [&](int i) { return Three{ct(i) - c[i], f[i], g[i]}; }, ct,
                    [&](int i, double kc, Three x) {
                        const double gni = kc - x.b;
                        gn[i] = gni;
                        a[0] += x.c * x.a;
                        a[1] += x.a * (gni - x.c);
                        a[2] += x.a * x.a;
                    });
    block_partial<kOps, 3>(a, slot_ptr(partials, SLOT_HOST));
}

// 5. step: c <- P(c + t d), s -> slot head, g <- g + gscale (gn - g)
// (gscale = 1: the trial's gradient itself)
__global__ __launch_bounds__(kBlock) void kl_step(Part P, double *__restrict__ c,
                                                  const double *__restrict__ d, double t,
                                                  double *__restrict__ g,
                                                  const double *__restrict__ gn, double gscale,
                                                  double *__restrict__ S, int64_t ld,
                                                  LmState *st, Box B)
{
    const int head = st->head;
    for_rows(P, [&](int i, bool act) {
        if (!act) return;
        const double ci = c[i];
        const double cn = proj_box(ci + t * d[i], B);
        S[head * ld + i] = cn - ci;
        c[i] = cn;
        g[i] = gscale == 1.0 ? gn[i] : g[i] + gscale * (gn[i] - g[i]);
    });
    if (blockIdx.x == 0 && threadIdx.x == 0) st->pending = 1;
}

// The pair pass holds 4M + 3 accumulators per lane (95 VGPRs at M = 5), so
// one 1024-thread block fits a CU: it runs one block per CU and walks more
// slices per wavefront instead of queueing a second round of blocks.
constexpr int kPairBlocks = 256;

// Pair pass and coefficients; with apply, the pending step (t, gscale) is
// taken inside the pair pass.
template <int M>
void launch_pairs_coef(nn_ctx *ctx, const Part &P, double *c, double *g, Box B, bool apply,
                       double t, double gscale)
{
    LmWork &L = ctx->lm;
    const Part P1 = make_part(P.n, kPairBlocks);
    kl_pairs<M><<<P1.nb, kBlock, 0, ctx->stream>>>(P1, c, g, L.pg, L.S, L.Y, L.cap,
                                                   (const LmState *)L.state, B, L.part,
                                                   apply ? 1 : 0, L.d, t, L.gn, gscale);
    kl_coef<M><<<1, 64, 0, ctx->stream>>>(P1.nb, (LmState *)L.state, L.part, apply ? 1 : 0);
}

template <int M>
void launch_coef(nn_ctx *ctx, const Part &P)
{
    const Part P1 = make_part(P.n, kPairBlocks);
    kl_coef<M><<<1, 64, 0, ctx->stream>>>(P1.nb, (LmState *)ctx->lm.state, ctx->lm.part, 0);
}

template <int M>
void launch_dir(nn_ctx *ctx, const Part &P, const double *c, const double *g, Box B)
{
    LmWork &L = ctx->lm;
    kl_dir<M><<<P.nb, kBlock, 0, ctx->stream>>>(P, c, g, L.pg, L.S, L.Y, L.cap,
                                                (const LmState *)L.state, B, L.d, ctx->partials);
}

#define NN_LM_DISPATCH(m, fn, ...)                  \
    switch (m) {                                    \
    case 1: fn<1>(__VA_ARGS__); break;              \
    case 2: fn<2>(__VA_ARGS__); break;              \
    case 3: fn<3>(__VA_ARGS__); break;              \
    case 4: fn<4>(__VA_ARGS__); break;              \
    case 5: fn<5>(__VA_ARGS__); break;              \
    case 6: fn<6>(__VA_ARGS__); break;              \
    case 7: fn<7>(__VA_ARGS__); break;              \
    default: fn<8>(__VA_ARGS__); break;             \
    }

nn_status ensure_lm(nn_ctx *ctx, int64_t n, int m)
{
    LmWork &L = ctx->lm;
    if (L.state && L.cap >= n && L.m >= m) return NN_OK;
    lm_release(ctx);
    const int64_t cap = std::max<int64_t>(n, 64);
    hipError_t e = dev_malloc(ctx->al, &L.S, sizeof(double) * cap * m);
    if (e == hipSuccess) e = dev_malloc(ctx->al, &L.Y, sizeof(double) * cap * m);
    if (e == hipSuccess) e = dev_malloc(ctx->al, &L.pg, sizeof(double) * cap);
    if (e == hipSuccess) e = dev_malloc(ctx->al, &L.d, sizeof(double) * cap);
    if (e == hipSuccess) e = dev_malloc(ctx->al, &L.gn, sizeof(double) * cap);
    if (e == hipSuccess) e = dev_malloc(ctx->al, &L.part, sizeof(double) * kLmNV * kMaxBlocks);
    if (e == hipSuccess) e = dev_malloc(ctx->al, &L.state, sizeof(LmState));
    if (e == hipSuccess) e = hipHostMalloc(&L.h_state, sizeof(LmState), hipHostMallocDefault);
    if (e != hipSuccess) {
        lm_release(ctx);
        return fail(ctx, NN_EOOM, std::string("BLMVM workspace: ") + hipGetErrorString(e));
    }
    // stale slots are never read as pairs, but keep them finite
    e = hipMemsetAsync(L.S, 0, sizeof(double) * cap * m, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L.Y, 0, sizeof(double) * cap * m, ctx->stream);
    if (e != hipSuccess) return fail(ctx, NN_EHIP, hipGetErrorString(e));
    L.cap = cap;
    L.m = m;
    return NN_OK;
}

}  // namespace

void lm_release(nn_ctx *ctx)
{
    LmWork &L = ctx->lm;
    double *bufs[] = {L.S, L.Y, L.pg, L.d, L.gn, L.part};
    for (double *b : bufs) dev_free(ctx->al, b);
    dev_free(ctx->al, L.state);
    if (L.h_state) (void)hipHostFree(L.h_state);
    L = LmWork();
}

nn_status blmvm_impl(nn_ctx *ctx, const nn_matrix *A, const double *vals, const double *f,
                     const nn_opts *o, double *c, uint8_t *active, nn_stats *st)
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
    const int M = std::min(std::max(o->lmm_vectors, 1), kLmMax);
    nn_status rc = ensure_workspace(ctx, n);
    if (rc != NN_OK) return rc;
    if ((rc = ensure_lm(ctx, n, M)) != NN_OK) return rc;
    Workspace &W = ctx->ws;
    LmWork &L = ctx->lm;
    LmState &H = *(LmState *)L.h_state;
    const Part P = make_part(n);
    const double nd = (double)n, nnz = (double)A->nnz;
    const double b_grad = 4.0 * (nd + 1) + 12.0 * nnz + 32.0 * nd;
    const double b_trial = 4.0 * (nd + 1) + 12.0 * nnz + 40.0 * nd;
    static const int kInitOps[4] = {OP_SUM, OP_MAX, OP_SUM, OP_SUM};
    static const int kGradOps[5] = {OP_SUM, OP_SUM, OP_MAX, OP_MIN, OP_SUM};
    static const int kTrialOps[3] = {OP_SUM, OP_SUM, OP_SUM};
    double red[kMaxRed];

    // ---- start point, load statistics, first gradient
    const double c0v = std::min(std::max(o->c0_value, box.lo), box.hi);
    prof_begin(ctx, KC_OTHER, 16.0 * n);
    launch_init(ctx, n, c, f, o->c0_mode == 1 ? 1 : 0, c0v, box);
    prof_end(ctx);
    if ((rc = host_reduce(ctx, n, 4, kInitOps, red)) != NN_OK) return rc;
    S.bytes_moved += 16.0 * n;
    const double normf = std::sqrt(red[0]), fmax = red[1];
    S.norm_f = normf;
    if (red[2] != 0.0 || red[3] != 0.0)
        return finish(fail(ctx, NN_ENONFINITE, "non-finite value in f or the initial c"));
    if (box.lo == 0.0 && !(fmax > 0.0)) {
        NN_HIP_TRY(ctx, hipMemsetAsync(c, 0, sizeof(double) * n, ctx->stream));
        S.n_active = (int32_t)n;
        return finish(NN_OK);
    }
    // gradient pass with the KKT report; true when the point is converged
    auto refresh = [&](bool &conv) -> nn_status {
        prof_begin(ctx, KC_GRAD, b_grad);
        launch_grad(ctx, A, vals, nullptr, c, f, W.g, box);
        prof_end(ctx);
        S.spmvs++;
        S.bytes_moved += b_grad;
        nn_status r2 = host_reduce(ctx, n, 5, kGradOps, red);
        if (r2 != NN_OK) return r2;
        if (red[1] != 0.0) return fail(ctx, NN_ENONFINITE, "non-finite gradient");
        S.kkt_rel = std::sqrt(red[0]) / normf;
        S.kkt_nat_inf = red[2];
        S.min_c = red[3];
        S.n_active = (int32_t)red[4];
        conv = S.kkt_rel <= o->tol;
        return NN_OK;
    };
    bool conv = false;
    if ((rc = refresh(conv)) != NN_OK) return finish(rc);
    if (conv) return finish(NN_OK);
    kl_state_init<<<1, 1, 0, ctx->stream>>>((LmState *)L.state, 1.0);
    std::memset(L.h_state, 0, sizeof(LmState));

    const double vp = 8.0 * n;   // bytes of one vector pass
    // Trial at step t along d: gathers P(c + t d), writes K c(t) - f; the
    // partials (g.s, s.(gn - g), s.s) stay in the host slot.
    auto launch_trial_t = [&](double t) {
        prof_begin(ctx, KC_TRIAL, b_trial);
        NN_DISPATCH_W(A->wmax, (kl_trial<WM, ColsI32>), P.nb, P, A->sl_off, ColsI32{A->sl_col},
                      vals, c, L.d, t, f, W.g, L.gn, box, ctx->partials);
        prof_end(ctx);
        S.spmvs++;
        S.search_trials++;
        S.bytes_moved += b_trial;
    };
    auto read_trial = [&](double &gs, double &sks) -> nn_status {
        nn_status r2 = host_reduce(ctx, n, 3, kTrialOps, red);
        gs = red[0];
        sks = red[1];
        return r2;
    };
    // Direction pass (partials in SLOT_Q) and, without waiting for it, the
    // first trial t = 1 (both line searches start there); one synchronisation
    // returns the state, the direction summary and the trial.
    double bmin = INFINITY, gd = 0.0, gs1 = 0.0, sks1 = 0.0;
    auto direction_and_first_trial = [&]() -> nn_status {
        const double live = std::min(H.count + 1, M);
        prof_begin(ctx, KC_OTHER, vp * (4.0 + 2.0 * live));
        NN_LM_DISPATCH(M, launch_dir, ctx, P, c, W.g, box);
        prof_end(ctx);
        launch_trial_t(1.0);
        kl_summary<<<1, 64, 0, ctx->stream>>>(P.nb, (LmState *)L.state, ctx->partials);
        NN_HIP_TRY(ctx, hipMemcpyAsync(L.h_state, L.state, sizeof(LmState),
                                       hipMemcpyDeviceToHost, ctx->stream));
        NN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        bmin = H.bmin;
        gd = H.gd;
        gs1 = H.gs;
        sks1 = H.sks;
        return NN_OK;
    };
    bool fresh = true;
    int since_fresh = 0;
    // the step of an iteration is taken by the next pair pass unless a
    // gradient refresh comes in between
    bool step_pending = false;
    double step_t = 0.0, step_gscale = 1.0;
    nn_status result = NN_EMAXIT;
    for (int it = 0;; it++) {
        // ---- 1-3. (pending step,) pairs, coefficients, direction (+ first trial)
        const double live = std::min(it, M);
        const double b_pairs = vp * (5.0 + 2.0 * live) + (step_pending ? vp * 3.0 : 0.0);
        prof_begin(ctx, KC_OTHER, b_pairs);
        NN_LM_DISPATCH(M, launch_pairs_coef, ctx, P, c, W.g, box, step_pending, step_t,
                       step_gscale);
        prof_end(ctx);
        S.bytes_moved += b_pairs + vp * (4.0 + 2.0 * live);
        step_pending = false;
        if ((rc = direction_and_first_trial()) != NN_OK) return finish(rc);
        if (H.nonfinite != 0.0) return finish(fail(ctx, NN_ENONFINITE, "non-finite iterate"));
        S.outer_its = it;
        const double rel = std::sqrt(H.pg2) / normf;
        if (rel <= o->tol) {
            if (fresh) {
                S.kkt_rel = rel;
                result = NN_OK;
                break;
            }
            if ((rc = refresh(conv)) != NN_OK) return finish(rc);
            fresh = true;
            since_fresh = 0;
            if (conv) {
                result = NN_OK;
                break;
            }
            continue;   // pairs and direction again from the fresh gradient
        }
        if (it >= o->max_lm_its) {
            fail(ctx, NN_EMAXIT, "BLMVM iteration cap reached");
            break;
        }
        if (!(gd < 0.0)) {
            // not a descent direction: forget the pairs, d = -gamma pg
            kl_forget<<<1, 1, 0, ctx->stream>>>((LmState *)L.state);
            NN_LM_DISPATCH(M, launch_coef, ctx, P);
            S.bytes_moved += vp * 4.0;
            S.refinements++;   // memory resets
            if ((rc = direction_and_first_trial()) != NN_OK) return finish(rc);
            if (!(gd < 0.0)) {
                fail(ctx, NN_EMAXIT, "no descent direction above the tolerance (rounding floor)");
                break;
            }
        }
        // ---- 4. line search (the trial at t = 1 is in gs1, sks1)
        double t, gscale, gs = gs1, sks = sks1;
        if (bmin >= 1.0) {
            if (!(sks > 0.0))
                return finish(fail(ctx, NN_ENOTSPD, "non-positive curvature along the direction"));
            t = std::min(-gs / sks, bmin);
            gscale = t;
        } else {
            t = 1.0;
            gscale = 1.0;
            for (int k = 0;; k++) {
                if (gs < 0.0 && gs + 0.5 * sks <= kLmMu * gs) break;
                t *= 0.5;
                if (t <= bmin || k + 1 >= kLmMaxTrials) {
                    // exact step on the segment before the first crossing
                    t = bmin;
                    launch_trial_t(t);
                    if ((rc = read_trial(gs, sks)) != NN_OK) return finish(rc);
                    if (!(sks > 0.0))
                        return finish(fail(ctx, NN_ENOTSPD, "non-positive curvature along the direction"));
                    gscale = std::min(-gs / sks, 1.0);
                    t *= gscale;
                    break;
                }
                launch_trial_t(t);
                if ((rc = read_trial(gs, sks)) != NN_OK) return finish(rc);
            }
        }
        // ---- 5. step: taken by the next pair pass, or here before a refresh
        fresh = gscale == 1.0;
        since_fresh = fresh ? 0 : since_fresh + 1;
        if (since_fresh >= kLmRefresh) {
            prof_begin(ctx, KC_OTHER, 56.0 * n);
            kl_step<<<P.nb, kBlock, 0, ctx->stream>>>(P, c, L.d, t, W.g, L.gn, gscale, L.S,
                                                      L.cap, (LmState *)L.state, box);
            prof_end(ctx);
            S.bytes_moved += 56.0 * n;
            if ((rc = refresh(conv)) != NN_OK) return finish(rc);
            fresh = true;
            since_fresh = 0;
        } else {
            step_pending = true;
            step_t = t;
            step_gscale = gscale;
        }
        if (o->verbose)
            std::fprintf(stderr, "nnqp blmvm %5d |pg|/|f| %.3e pairs %d gamma %.3g crossing %.3g step %.3g\n",
                         it, rel, H.count, H.gamma, bmin, t);
    }
    // final report from a fresh gradient
    if ((rc = refresh(conv)) != NN_OK) return finish(rc);
    if (result == NN_OK && !conv) result = NN_EMAXIT;
    if (result == NN_OK) ctx->err.clear();
    return finish(result);
}

}  // namespace nnqp
