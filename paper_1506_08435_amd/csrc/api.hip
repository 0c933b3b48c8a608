// C ABI entry points (include/nnqp.h): argument checks, object lifetime,
// workspace, profiling, and dispatch to the assembly and solver code.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "nnqp_internal.hpp"

namespace nnqp {

nn_status fail(nn_ctx *ctx, nn_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

hipError_t dev_malloc_raw(const DevAlloc &a, void **p, size_t bytes)
{
    *p = nullptr;
    if (!a.alloc) return hipMalloc(p, bytes);
    *p = a.alloc(bytes > 0 ? bytes : 8, a.user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(const DevAlloc &a, void *p)
{
    if (!p) return;
    if (a.free_) a.free_(p, a.user);
    else (void)hipFree(p);
}

nn_status ensure_workspace(nn_ctx *ctx, int64_t n)
{
    Workspace &W = ctx->ws;
    if (W.cap >= n && W.g) return NN_OK;
    double **vecs[] = {&W.g,   &W.w,   &W.r,  &W.z,  &W.q,   &W.p0,  &W.p1,
                       &W.ks0, &W.ks1, &W.dm, &W.ft, &W.ks2};
    for (double **v : vecs)
        if (*v) {
            dev_free(ctx->al, *v);
            *v = nullptr;
        }
    float **fv[] = {&W.w32, &W.r32, &W.z32, &W.q32, &W.p32, &W.dm32};
    for (float **v : fv)
        if (*v) {
            dev_free(ctx->al, *v);
            *v = nullptr;
        }
    dev_free(ctx->al, W.mask);
    W.mask = nullptr;
    W.cap = 0;
    const int64_t cap = std::max<int64_t>(n, 1);
    for (double **v : vecs) {
        hipError_t e = dev_malloc(ctx->al, v, sizeof(double) * cap);
        if (e != hipSuccess) return fail(ctx, NN_EOOM, "workspace allocation failed");
    }
    if (dev_malloc(ctx->al, &W.mask, cap) != hipSuccess) return fail(ctx, NN_EOOM, "workspace allocation failed");
    float **fvecs[] = {&W.w32, &W.r32, &W.z32, &W.q32, &W.p32, &W.dm32};
    for (float **v : fvecs) {
        hipError_t e = dev_malloc(ctx->al, v, sizeof(float) * cap);
        if (e != hipSuccess) return fail(ctx, NN_EOOM, "workspace allocation failed");
    }
    W.cap = cap;
    return NN_OK;
}

nn_status host_reduce(nn_ctx *ctx, int64_t n, int nv, const int *ops, double *out)
{
    const Part P = make_part(n);
    // partials are laid out [value][block]: copy the first nv rows
    const size_t count = (size_t)(nv - 1) * kMaxBlocks + P.nb;
    NN_HIP_TRY(ctx, hipMemcpyAsync(ctx->h_part, ctx->partials, sizeof(double) * count,
                                   hipMemcpyDeviceToHost, ctx->stream));
    NN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < nv; k++) {
        double a = ops[k] == OP_SUM ? 0.0 : (ops[k] == OP_MIN ? INFINITY : -INFINITY);
        for (int b = 0; b < P.nb; b++) {
            const double v = ctx->h_part[(size_t)k * kMaxBlocks + b];
            a = ops[k] == OP_SUM ? a + v : (ops[k] == OP_MIN ? std::fmin(a, v) : std::fmax(a, v));
        }
        out[k] = a;
    }
    return NN_OK;
}

nn_status read_scalars(nn_ctx *ctx)
{
    NN_HIP_TRY(ctx, hipMemcpyAsync(ctx->h_scal, ctx->scal, sizeof(DevScalars), hipMemcpyDeviceToHost,
                                   ctx->stream));
    NN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return NN_OK;
}

static hipEvent_t pool_event(nn_ctx *ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void prof_begin(nn_ctx *ctx, int cls, double bytes, double bytes_csr)
{
    ctx->prof_open = false;
    ctx->prof_attach = false;
    if (!ctx->prof || !((ctx->prof_mask >> cls) & 1)) return;
    const bool cg = cls == KC_CG_SPMV || cls == KC_CG_UPDATE;
    if (cg && ctx->prof_every > 1) {
        // a pseudo-random one in prof_every: a fixed stride would keep hitting
        // the same place in every chunk of CG launches (the first launch after
        // a host read starts on an idle GPU and runs long)
        const uint32_t h = (uint32_t)ctx->prof_calls[cls]++ * 2654435761u;
        if ((h >> 16) % (uint32_t)ctx->prof_every != 0) return;
    }
    ProfEntry p;
    p.cls = cls;
    p.seq = ctx->prof_seq;
    p.a = pool_event(ctx);
    p.b = pool_event(ctx);
    p.bytes = bytes;
    p.bytes_csr = std::isnan(bytes_csr) ? bytes : bytes_csr;
    p.valid = 1;
    (void)hipEventRecord(p.a, ctx->stream);
    ctx->prof_live.push_back(p);
    ctx->prof_open = true;
    ctx->prof_attach = cg;
}

void prof_end(nn_ctx *ctx)
{
    ctx->prof_attach = false;
    if (!ctx->prof_open || ctx->prof_live.empty()) return;
    (void)hipEventRecord(ctx->prof_live.back().b, ctx->stream);
    ctx->prof_open = false;
}

bool prof_kernel_events(nn_ctx *ctx, hipEvent_t *a, hipEvent_t *b)
{
    if (!ctx->prof_attach || !ctx->prof_open || ctx->prof_live.empty()) return false;
    ProfEntry &p = ctx->prof_live.back();
    p.ka = pool_event(ctx);
    p.kb = pool_event(ctx);
    ctx->prof_attach = false;   // one kernel per entry
    if (!p.ka || !p.kb) return false;
    *a = p.ka;
    *b = p.kb;
    return true;
}

void prof_add(nn_ctx *ctx, int cls, double ms, double bytes, double bytes_csr)
{
    if (std::isnan(bytes_csr)) bytes_csr = bytes;
    ctx->prof_count[cls]++;
    ctx->prof_ms[cls] += ms;
    ctx->prof_bytes[cls] += bytes > 0 ? bytes : 0.0;
    ctx->prof_bytes_csr[cls] += bytes_csr > 0 ? bytes_csr : 0.0;
}

void prof_collect(nn_ctx *ctx)
{
    if (ctx->prof_live.empty()) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (ProfEntry &p : ctx->prof_live) {
        if (p.valid) {
            float ms = 0.f;
            const bool own = p.ka && p.kb;   // the kernel's own begin and end
            if (hipEventElapsedTime(&ms, own ? p.ka : p.a, own ? p.kb : p.b) == hipSuccess) {
                ctx->prof_count[p.cls]++;
                ctx->prof_ms[p.cls] += ms;
                ctx->prof_bytes[p.cls] += p.bytes > 0 ? p.bytes : 0.0;
                ctx->prof_bytes_csr[p.cls] += p.bytes_csr > 0 ? p.bytes_csr : 0.0;
            }
        }
        ctx->ev_pool.push_back(p.a);
        ctx->ev_pool.push_back(p.b);
        if (p.ka) ctx->ev_pool.push_back(p.ka);
        if (p.kb) ctx->ev_pool.push_back(p.kb);
    }
    ctx->prof_live.clear();
}

}  // namespace nnqp

namespace nnqp {

// Copies of K that the single-problem passes read: with f64, the paired
// int16 offsets and float64 values; when the float32 values exist, the quad
// int16 offsets and float32 values.
#ifndef NNQP_PAIR_F64
#define NNQP_PAIR_F64 1   // float64 solves read the paired layout when it exists
#endif

// The paired int16 offsets (nn_matrix::d16p) that every float64 paired copy
// is read with.
static nn_status ensure_d16p(nn_ctx *ctx, nn_matrix *K)
{
    if (K->d16p || !K->sl_d16 || K->n == 0) return NN_OK;
    const size_t m = (size_t)std::max<int64_t>(K->nsell, 1);
    if (dev_malloc(K->al, &K->d16p, sizeof(short) * m) != hipSuccess)
        return fail(ctx, NN_EOOM, "paired offsets allocation");
    launch_pair_d16(ctx, K, K->sl_d16, K->d16p);
    return NN_OK;
}

nn_status ensure_paired(nn_ctx *ctx, nn_matrix *K, bool f64)
{
    if (!K->sl_d16 || K->n == 0) return NN_OK;
    const size_t m = (size_t)std::max<int64_t>(K->nsell, 1);
    if (f64 && ensure_d16p(ctx, K) != NN_OK) return NN_EOOM;
    if (K->val32 && !K->val32q) {
        if (!K->d16q) {
            if (dev_malloc(K->al, &K->d16q, sizeof(short) * m) != hipSuccess)
                return fail(ctx, NN_EOOM, "quad offsets allocation");
            launch_quad_d16(ctx, K, K->sl_d16, K->d16q);
        }
        if (dev_malloc(K->al, &K->val32q, sizeof(float) * m) != hipSuccess)
            return fail(ctx, NN_EOOM, "quad float32 allocation");
        launch_quad_f32(ctx, K, K->val32, K->val32q);
    }
    if (f64 && !K->val64p) {
        if (dev_malloc(K->al, &K->val64p, sizeof(double) * m) != hipSuccess)
            return fail(ctx, NN_EOOM, "paired float64 allocation");
        launch_pair_f64(ctx, K, K->val, K->val64p);
    }
    NN_HIP_TRY(ctx, hipGetLastError());
    return NN_OK;
}

// M/dt + K values for a backward-Euler step (formed once per dt, kept with K).
// `paired`: the single-problem solver will read the paired copy for this
// precision (the batched solver reads the column-major values only).  Every
// copy that exists is re-formed when dt changes.
nn_status ensure_transient(nn_ctx *ctx, nn_matrix *K, double dt, bool mixed, bool paired)
{
    const int64_t n = K->n;
    if (n == 0) return NN_OK;
    const size_t m = (size_t)std::max<int64_t>(K->nsell, 1);
    const bool want32q = paired && mixed && K->sl_d16;
    const bool want64p = paired && !mixed && NNQP_PAIR_F64 && K->sl_d16;
    const bool fresh = K->kt && K->kt_dt == dt;
    if (fresh && (!mixed || K->kt32) && (!want32q || K->kt32q) && (!want64p || K->kt64p))
        return NN_OK;
    // each buffer is guarded on its own: a call that got one of them and was
    // refused the other leaves the first in place, and a later call takes
    // only the missing one (the values are formed below whenever kt_dt != dt)
    if (!K->kt && dev_malloc(K->al, &K->kt, sizeof(double) * m) != hipSuccess)
        return fail(ctx, NN_EOOM, "transient matrix allocation");
    if (!K->kt_diag && dev_malloc(K->al, &K->kt_diag, sizeof(double) * n) != hipSuccess)
        return fail(ctx, NN_EOOM, "transient diagonal allocation");
    if (mixed && !K->kt32 && dev_malloc(K->al, &K->kt32, sizeof(float) * m) != hipSuccess)
        return fail(ctx, NN_EOOM, "transient float32 allocation");
    if (want64p && ensure_d16p(ctx, K) != NN_OK) return NN_EOOM;
    if (want32q && !K->d16q) {
        if (dev_malloc(K->al, &K->d16q, sizeof(short) * m) != hipSuccess)
            return fail(ctx, NN_EOOM, "quad offsets allocation");
        launch_quad_d16(ctx, K, K->sl_d16, K->d16q);
    }
    if (want32q && !K->kt32q && dev_malloc(K->al, &K->kt32q, sizeof(float) * m) != hipSuccess)
        return fail(ctx, NN_EOOM, "transient float32 allocation");
    if (want64p && !K->kt64p && dev_malloc(K->al, &K->kt64p, sizeof(double) * m) != hipSuccess)
        return fail(ctx, NN_EOOM, "transient paired float64 allocation");
    launch_axpby_vals(ctx, K->nsell, K->mval, dt, K->val, K->kt);
    launch_diag(ctx, K, K->kt, K->kt_diag);
    if (K->kt32) launch_to_f32(ctx, K->nsell, K->kt, K->kt32);
    if (K->kt32 && K->kt32q) launch_quad_f32(ctx, K, K->kt32, K->kt32q);
    if (K->kt64p) launch_pair_f64(ctx, K, K->kt, K->kt64p);
    NN_HIP_TRY(ctx, hipGetLastError());
    K->kt_dt = dt;
    return NN_OK;
}

}  // namespace nnqp

using namespace nnqp;

#define NN_CHECK_CTX(ctx)                               \
    do {                                                \
        if (!(ctx)) return NN_EINVAL;                   \
        if (hipSetDevice((ctx)->device) != hipSuccess)  \
            return fail((ctx), NN_EHIP, "hipSetDevice"); \
    } while (0)

static nn_status create_impl(nn_ctx **out, int device, void *hip_stream, const DevAlloc &al)
{
    if (!out) return NN_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NN_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return NN_EHIP;
    noalloc_attach(device);
    nn_ctx *ctx = new (std::nothrow) nn_ctx();
    if (!ctx) return NN_EOOM;
    ctx->al = al;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    const size_t part_bytes = sizeof(double) * kSlots * kMaxBlocks * kMaxRed;
    bool ok = dev_malloc(ctx->al, &ctx->partials, part_bytes) == hipSuccess &&
              hipHostMalloc(&ctx->h_part, sizeof(double) * kMaxBlocks * kMaxRed,
                            hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&ctx->h_multi, sizeof(double) * kMaxBlocks * (5 + 3 * kLadder),
                            hipHostMallocDefault) == hipSuccess &&
              dev_malloc(ctx->al, &ctx->scal, sizeof(DevScalars)) == hipSuccess &&
              hipHostMalloc(&ctx->h_scal, sizeof(DevScalars), hipHostMallocDefault) == hipSuccess &&
              hipEventCreate(&ctx->ev0) == hipSuccess && hipEventCreate(&ctx->ev1) == hipSuccess;
    if (ok) {
        ok = hipMemsetAsync(ctx->partials, 0, part_bytes, ctx->stream) == hipSuccess &&
             hipMemsetAsync(ctx->scal, 0, sizeof(DevScalars), ctx->stream) == hipSuccess &&
             hipStreamSynchronize(ctx->stream) == hipSuccess;
    }
    if (!ok) {
        nn_destroy(ctx);
        return NN_EOOM;
    }
    *out = ctx;
    return NN_OK;
}

nn_status nnqp::check_opts(nn_ctx *ctx, const nn_opts *o)
{
    if (!o) return fail(ctx, NN_EINVAL, "null options");
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(ctx, NN_EINVAL, "tol must be > 0");
    if (!(o->inner_rtol > 0.0 && o->inner_rtol < 1.0))
        return fail(ctx, NN_EINVAL, "inner_rtol must be in (0, 1)");
    if (o->max_outer < 0 || o->max_cg < 1) return fail(ctx, NN_EINVAL, "bad iteration caps");
    if (o->precision != NN_FP64 && o->precision != NN_MIXED)
        return fail(ctx, NN_EINVAL, "unknown precision");
    if (o->c0_mode != 0 && o->c0_mode != 1) return fail(ctx, NN_EINVAL, "unknown c0_mode");
    if (o->c0_mode == 0 && !std::isfinite(o->c0_value))
        return fail(ctx, NN_EINVAL, "c0_value must be finite");
    if (!std::isfinite(o->lower) || std::isnan(o->upper) || !(o->upper > o->lower))
        return fail(ctx, NN_EINVAL, "bounds must satisfy lower finite, upper > lower");
    if (o->method != NN_TRON && o->method != NN_BLMVM) return fail(ctx, NN_EINVAL, "unknown method");
    if (o->precond_degree < 0 || o->precond_degree > 8)
        return fail(ctx, NN_EINVAL, "precond_degree must be in 0..8");
    if (o->subspace != 0 && o->subspace != 1) return fail(ctx, NN_EINVAL, "subspace must be 0 or 1");
    if (o->engine < 0 || o->engine > 2) return fail(ctx, NN_EINVAL, "engine must be 0, 1 or 2");
    if (o->method == NN_BLMVM) {
        if (o->lmm_vectors < 1 || o->lmm_vectors > 8)
            return fail(ctx, NN_EINVAL, "lmm_vectors must be in 1..8");
        if (o->max_lm_its < 0) return fail(ctx, NN_EINVAL, "bad iteration cap");
        if (o->precision != NN_FP64) return fail(ctx, NN_EINVAL, "BLMVM runs in float64 only");
    }
    return NN_OK;
}

extern "C" {

nn_status nn_create(nn_ctx **out, int device, void *hip_stream)
{
    return create_impl(out, device, hip_stream, DevAlloc{});
}

nn_status nn_create_ex(nn_ctx **out, int device, void *hip_stream, nn_alloc_fn alloc,
                       nn_free_fn free_, void *user)
{
    if (out) *out = nullptr;
    if (!alloc || !free_) return NN_EINVAL;
    DevAlloc a;
    a.alloc = alloc;
    a.free_ = free_;
    a.user = user;
    return create_impl(out, device, hip_stream, a);
}


void nn_destroy(nn_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    Workspace &W = ctx->ws;
    double *vecs[] = {W.g,   W.w,   W.r,  W.z,  W.q,   W.p0,  W.p1,
                      W.ks0, W.ks1, W.dm, W.ft, W.ks2};
    for (double *v : vecs)
        dev_free(ctx->al, v);
    float *fvecs[] = {W.w32, W.r32, W.z32, W.q32, W.p32, W.dm32};
    for (float *v : fvecs)
        dev_free(ctx->al, v);
    dev_free(ctx->al, W.mask);
    double *cv[] = {W.cres, W.cdz[0], W.cdz[1]};
    for (double *v : cv)
        dev_free(ctx->al, v);
    float *cf[] = {W.cres32, W.cdz32[0], W.cdz32[1]};
    for (float *v : cf)
        dev_free(ctx->al, v);
    lm_release(ctx);
    dev_free(ctx->al, ctx->partials);
    if (ctx->h_part) (void)hipHostFree(ctx->h_part);
    if (ctx->h_multi) (void)hipHostFree(ctx->h_multi);
    dev_free(ctx->al, ctx->scal);
    if (ctx->h_scal) (void)hipHostFree(ctx->h_scal);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (ProfEntry &p : ctx->prof_live) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
        if (p.ka) (void)hipEventDestroy(p.ka);
        if (p.kb) (void)hipEventDestroy(p.kb);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

const char *nn_last_error(const nn_ctx *ctx)
{
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

nn_status nn_default_opts(nn_opts *o)
{
    if (!o) return NN_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->inner_rtol = 1e-1;
    o->max_outer = 500;
    o->max_cg = 5000;
    o->precision = NN_FP64;
    o->c0_mode = 0;
    o->c0_value = 1e-8;
    o->delta0 = 0.0;
    o->cg_chunk = 16;
    o->lower = 0.0;
    o->upper = INFINITY;
    o->method = NN_TRON;
    o->lmm_vectors = 5;
    o->max_lm_its = 20000;
    o->subspace = 0;
    return NN_OK;
}

nn_status nn_assemble(nn_ctx *ctx, const nn_mesh *mesh, const double *D, int64_t nD,
                      const double *kscale, const double *f_elem, const uint8_t *dirichlet,
                      const double *dirichlet_values, int with_mass, nn_matrix **K_out,
                      double *F_dev, int64_t *dof_of_node)
{
    NN_CHECK_CTX(ctx);
    if (K_out) *K_out = nullptr;
    return assemble_impl(ctx, mesh, D, nD, kscale, f_elem, dirichlet, dirichlet_values, with_mass,
                         K_out, F_dev, dof_of_node);
}

nn_status nn_matrix_from_csr(nn_ctx *ctx, int64_t n, const int64_t *rowptr, const int32_t *col,
                             const double *val, const double *mval, nn_matrix **out)
{
    NN_CHECK_CTX(ctx);
    if (!out || n < 0 || !rowptr || (n > 0 && (!col || !val)))
        return fail(ctx, NN_EINVAL, "null argument to nn_matrix_from_csr");
    *out = nullptr;
    if (n >= ((int64_t)1 << 31)) return fail(ctx, NN_EINVAL, "n too large");
    if (rowptr[0] != 0) return fail(ctx, NN_EINVAL, "rowptr[0] must be 0");
    const int64_t nnz = rowptr[n];
    if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(ctx, NN_EINVAL, "nnz out of range");
    std::vector<int> rp32(n + 1);
    for (int64_t i = 0; i < n; i++) {
        if (rowptr[i + 1] < rowptr[i]) return fail(ctx, NN_EINVAL, "rowptr not monotone");
        bool has_diag = false;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) {
            if (col[k] < 0 || col[k] >= n) return fail(ctx, NN_EINVAL, "column index out of range");
            if (k > rowptr[i] && col[k] <= col[k - 1])
                return fail(ctx, NN_EINVAL, "columns must be strictly ascending within a row");
            if (!std::isfinite(val[k]) || (mval && !std::isfinite(mval[k])))
                return fail(ctx, NN_ENONFINITE, "non-finite matrix value");
            if (col[k] == i) has_diag = true;
        }
        if (!has_diag) return fail(ctx, NN_EINVAL, "missing diagonal entry");
        rp32[i] = (int)rowptr[i];
    }
    rp32[n] = (int)nnz;
    nn_matrix *M = new (std::nothrow) nn_matrix();
    if (!M) return fail(ctx, NN_EOOM, "host allocation");
    M->al = ctx->al;
    M->n = n;
    M->nnz = nnz;
    const size_t nz = (size_t)std::max<int64_t>(nnz, 1);
    double *d_val = nullptr, *d_mval = nullptr;
    auto release = [&]() {
        dev_free(ctx->al, d_val);
        dev_free(ctx->al, d_mval);
    };
    bool ok = dev_malloc(M->al, &M->rowptr, sizeof(int) * (n + 1)) == hipSuccess &&
              dev_malloc(M->al, &M->col, sizeof(int) * nz) == hipSuccess &&
              dev_malloc(ctx->al, &d_val, sizeof(double) * nz) == hipSuccess &&
              (!mval || dev_malloc(ctx->al, &d_mval, sizeof(double) * nz) == hipSuccess);
    if (!ok) {
        release();
        nn_matrix_free(ctx, M);
        return fail(ctx, NN_EOOM, "matrix allocation failed");
    }
    hipStream_t s = ctx->stream;
    ok = hipMemcpyAsync(M->rowptr, rp32.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok && nnz > 0) {
        ok = hipMemcpyAsync(M->col, col, sizeof(int) * nnz, hipMemcpyHostToDevice, s) == hipSuccess &&
             hipMemcpyAsync(d_val, val, sizeof(double) * nnz, hipMemcpyHostToDevice, s) == hipSuccess &&
             (!mval || hipMemcpyAsync(d_mval, mval, sizeof(double) * nnz, hipMemcpyHostToDevice, s) == hipSuccess);
    }
    if (!ok || hipStreamSynchronize(s) != hipSuccess) {
        release();
        nn_matrix_free(ctx, M);
        return fail(ctx, NN_EHIP, "matrix upload failed");
    }
    int mr = 0;
    for (int64_t i = 0; i < n; i++) mr = std::max<int>(mr, (int)(rowptr[i + 1] - rowptr[i]));
    M->max_row = mr;
    nn_status st = sell_build(ctx, M, rowptr, d_val, d_mval);
    release();
    if (st == NN_OK) st = finish_matrix(ctx, M);
    if (st != NN_OK) {
        nn_matrix_free(ctx, M);
        return st;
    }
    *out = M;
    return NN_OK;
}

nn_status nn_matrix_info(const nn_matrix *A, int64_t *n, int64_t *nnz, int *has_mass)
{
    if (!A) return NN_EINVAL;
    if (n) *n = A->n;
    if (nnz) *nnz = A->nnz;
    if (has_mass) *has_mass = A->mval != nullptr;
    return NN_OK;
}

nn_status nn_matrix_export(nn_ctx *ctx, const nn_matrix *A, int64_t *rowptr, int32_t *col,
                           double *val, double *mval)
{
    NN_CHECK_CTX(ctx);
    if (!A) return fail(ctx, NN_EINVAL, "null matrix");
    if (mval && !A->mval) return fail(ctx, NN_EINVAL, "matrix has no capacity values");
    hipStream_t s = ctx->stream;
    std::vector<int> rp(A->n + 1);
    NN_HIP_TRY(ctx, hipMemcpyAsync(rp.data(), A->rowptr, sizeof(int) * (A->n + 1),
                                   hipMemcpyDeviceToHost, s));
    NN_HIP_TRY(ctx, hipStreamSynchronize(s));
    std::vector<int64_t> rp64(rp.begin(), rp.end());
    if (rowptr)
        for (int64_t i = 0; i <= A->n; i++) rowptr[i] = rp64[i];
    if (A->nnz > 0) {
        if (col) NN_HIP_TRY(ctx, hipMemcpyAsync(col, A->col, sizeof(int) * A->nnz, hipMemcpyDeviceToHost, s));
        // values live in sliced-ELL order: entry k of row i sits at off[i/64] + 64 k + i%64
        std::vector<int64_t> off;
        int wmax = 0;
        sell_offsets(rp64.data(), A->n, off, wmax);
        std::vector<double> buf(A->nsell);
        const double *srcs[2] = {A->val, A->mval};
        double *dsts[2] = {val, mval};
        for (int t = 0; t < 2; t++) {
            if (!dsts[t]) continue;
            NN_HIP_TRY(ctx, hipMemcpyAsync(buf.data(), srcs[t], sizeof(double) * A->nsell,
                                           hipMemcpyDeviceToHost, s));
            NN_HIP_TRY(ctx, hipStreamSynchronize(s));
            for (int64_t i = 0; i < A->n; i++)
                for (int64_t k = 0; k < rp64[i + 1] - rp64[i]; k++)
                    dsts[t][rp64[i] + k] = buf[off[i / kSlice] + k * kSlice + i % kSlice];
        }
    }
    NN_HIP_TRY(ctx, hipStreamSynchronize(s));
    return NN_OK;
}

nn_status nn_matrix_bytes(const nn_matrix *A, int precision, size_t *bytes)
{
    if (!A || !bytes) return NN_EINVAL;
    const double n = (double)A->n, nnz = (double)A->nnz, ns = (double)A->nsell;
    double b = 4.0 * (n + 1) + 4.0 * nnz;                   // CSR pattern
    b += 4.0 * (A->nslices + 1) + 12.0 * ns + 8.0 * n;      // sliced-ELL columns, values, diag
    if (A->sl_d16) b += 2.0 * ns;                           // int16 column offsets
    if (A->mval) b += 16.0 * ns + 8.0 * n;                  // capacity + transient values, diag
    b += 11.0 * 8.0 * n + n;                                // solver work vectors + mask
    if (precision == NN_MIXED) b += 4.0 * ns + 40.0 * n;    // float32 values and vectors
    // paired copies already made by single-problem solves
    if (A->d16p) b += 2.0 * ns;
    if (A->d16q) b += 2.0 * ns;
    if (A->val32q) b += 4.0 * ns;
    if (A->kt32q) b += 4.0 * ns;
    if (A->val64p) b += 8.0 * ns;
    if (A->kt64p) b += 8.0 * ns;
    *bytes = (size_t)b;
    return NN_OK;
}

void nn_matrix_free(nn_ctx *ctx, nn_matrix *A)
{
    if (!A) return;
    if (ctx) (void)hipSetDevice(ctx->device);
    int *iv[] = {A->rowptr, A->col, A->sl_off, A->sl_col};
    for (int *p : iv)
        dev_free(A->al, p);
    dev_free(A->al, A->sl_d16);
    dev_free(A->al, A->d16p);
    dev_free(A->al, A->d16q);
    dev_free(A->al, A->val64p);
    dev_free(A->al, A->kt64p);
    double *dv[] = {A->val, A->mval, A->diag, A->kt, A->kt_diag};
    for (double *p : dv)
        dev_free(A->al, p);
    float *fv[] = {A->val32, A->kt32, A->val32q, A->kt32q};
    for (float *p : fv)
        dev_free(A->al, p);
    delete A;
}

nn_status nn_matvec(nn_ctx *ctx, const nn_matrix *A, int which, const double *x_dev, double *y_dev)
{
    NN_CHECK_CTX(ctx);
    if (!A || (A->n > 0 && (!x_dev || !y_dev)) || (which != 0 && which != 1))
        return fail(ctx, NN_EINVAL, "bad argument to nn_matvec");
    if (which == 1 && !A->mval) return fail(ctx, NN_EINVAL, "matrix has no capacity values");
    launch_matvec(ctx, A, which == 0 ? A->val : A->mval, x_dev, y_dev);
    NN_HIP_TRY(ctx, hipGetLastError());
    return NN_OK;
}


// NN_OK: run the solve in one workgroup; NN_EMAXIT: run the multi-block
// passes; NN_EINVAL: engine 2 asked for a solve one workgroup cannot run.
static nn_status choose_solo(nn_ctx *ctx, const nn_matrix *K, const nn_opts *o)
{
    const bool ok = solo_eligible(K, o);
    if (o->engine == 2) {
        if (!ok)
            return fail(ctx, NN_EINVAL,
                        "engine 2 (one workgroup) runs float64 TRON without a trust radius, "
                        "subspace loop, Chebyshev preconditioner or trace");
        return NN_OK;
    }
    return (o->engine == 0 && ok && K->n <= kSoloMaxRows) ? NN_OK : NN_EMAXIT;
}

nn_status nn_solve_nonneg(nn_ctx *ctx, nn_matrix *K, const double *f_dev,
                          const nn_opts *opts, double *c_dev, uint8_t *active_dev, nn_stats *stats)
{
    NN_CHECK_CTX(ctx);
    if (!K || (K->n > 0 && (!f_dev || !c_dev))) return fail(ctx, NN_EINVAL, "null argument");
    nn_status st = check_opts(ctx, opts);
    if (st != NN_OK) return st;
    if (opts->method == NN_BLMVM)
        return blmvm_impl(ctx, K, K->val, f_dev, opts, c_dev, active_dev, stats);
    if ((st = choose_solo(ctx, K, opts)) == NN_OK)
        return solo_solve_impl(ctx, K, K->val, K->diag, f_dev, opts, c_dev, active_dev, stats);
    if (st != NN_EMAXIT) return st;   // (NN_EMAXIT: the multi-block passes)
    const float *v32 = nullptr;
    if (opts->precision == NN_MIXED && K->n > 0) {
        if (!K->val32) {
            if (dev_malloc(K->al, &K->val32, sizeof(float) * std::max<int64_t>(K->nsell, 1)) != hipSuccess)
                return fail(ctx, NN_EOOM, "float32 value allocation");
            launch_to_f32(ctx, K->nsell, K->val, K->val32);
            NN_HIP_TRY(ctx, hipGetLastError());
        }
        v32 = K->val32;
    }
    // paired copies for the CG and search passes (when the int16 offsets exist)
    const bool pair64 = NNQP_PAIR_F64 && v32 == nullptr;
    if ((v32 || pair64) && (st = ensure_paired(ctx, K, pair64)) != NN_OK) return st;
    return solve_impl(ctx, K, K->val, v32, v32 ? K->val32q : nullptr, v32 ? nullptr : K->val64p,
                      K->diag, f_dev, opts, c_dev, active_dev, stats);
}

nn_status nn_solve_galerkin(nn_ctx *ctx, nn_matrix *K, const double *f_dev, const nn_opts *opts,
                            double *c_dev, nn_stats *stats)
{
    NN_CHECK_CTX(ctx);
    if (!K || (K->n > 0 && (!f_dev || !c_dev))) return fail(ctx, NN_EINVAL, "null argument");
    nn_status st = check_opts(ctx, opts);
    if (st != NN_OK) return st;
    if (opts->precision != NN_FP64)
        return fail(ctx, NN_EINVAL, "the Galerkin solve runs in float64 only");
    return galerkin_impl(ctx, K, f_dev, opts, c_dev, stats);
}

nn_status nn_step_transient(nn_ctx *ctx, nn_matrix *K, double dt, const double *f_dev,
                            const nn_opts *opts, double *c_dev, uint8_t *active_dev,
                            nn_stats *stats)
{
    NN_CHECK_CTX(ctx);
    if (!K || (K->n > 0 && (!f_dev || !c_dev))) return fail(ctx, NN_EINVAL, "null argument");
    if (!K->mval) return fail(ctx, NN_EINVAL, "matrix has no capacity values (assemble with_mass)");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, NN_EINVAL, "dt must be > 0");
    nn_status st = check_opts(ctx, opts);
    if (st != NN_OK) return st;
    const int64_t n = K->n;
    const bool mixed = opts->precision == NN_MIXED;
    if (n == 0) return solve_impl(ctx, K, K->val, nullptr, nullptr, nullptr, K->diag, f_dev, opts,
                                    c_dev, active_dev, stats);
    if ((st = ensure_transient(ctx, K, dt, mixed, true)) != NN_OK) return st;
    if ((st = ensure_workspace(ctx, n)) != NN_OK) return st;
    launch_transient_rhs(ctx, K, c_dev, f_dev, dt, ctx->ws.ft);
    nn_opts o = *opts;
    o.c0_mode = 1;   // warm start from c^(n)
    if (o.method == NN_BLMVM) return blmvm_impl(ctx, K, K->kt, ctx->ws.ft, &o, c_dev, active_dev, stats);
    if ((st = choose_solo(ctx, K, &o)) == NN_OK)
        return solo_solve_impl(ctx, K, K->kt, K->kt_diag, ctx->ws.ft, &o, c_dev, active_dev, stats);
    if (st != NN_EMAXIT) return st;
    return solve_impl(ctx, K, K->kt, mixed ? K->kt32 : nullptr, mixed ? K->kt32q : nullptr,
                      mixed ? nullptr : K->kt64p, K->kt_diag, ctx->ws.ft, &o, c_dev, active_dev,
                      stats);
}

// Shared checks of the batched entry points: arguments, options, and that
// no two members' solution buffers overlap (they are written concurrently).
static nn_status check_batch(nn_ctx *ctx, int32_t nprob, nn_matrix *const *K,
                             const double *const *f_dev, const nn_opts *opts,
                             double *const *c_dev, bool need_mass)
{
    if (nprob < 0) return fail(ctx, NN_EINVAL, "nprob must be >= 0");
    if (nprob > 0 && (!K || !f_dev || !c_dev)) return fail(ctx, NN_EINVAL, "null argument");
    nn_status st = check_opts(ctx, opts);
    if (st != NN_OK) return st;
    if (opts->method != NN_TRON) return fail(ctx, NN_EINVAL, "the batched solver runs TRON only");
    if (opts->precond_degree > 1)
        return fail(ctx, NN_EINVAL, "the batched solver uses the Jacobi preconditioner only");
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    for (int p = 0; p < nprob; p++) {
        if (!K[p]) return fail(ctx, NN_EINVAL, "null matrix in batch");
        if (need_mass && !K[p]->mval)
            return fail(ctx, NN_EINVAL, "batch member has no capacity values (assemble with_mass)");
        if (K[p]->n > 0 && (!f_dev[p] || !c_dev[p]))
            return fail(ctx, NN_EINVAL, "null f or c in batch");
        if (K[p]->n > 0)
            spans.push_back({(uintptr_t)c_dev[p], (uintptr_t)c_dev[p] + sizeof(double) * K[p]->n});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); k++)
        if (spans[k].first < spans[k - 1].second)
            return fail(ctx, NN_EINVAL, "solution buffers of two batch members overlap");
    return NN_OK;
}

// A failure of a batched call itself (invalid arguments, an allocation
// refused, a HIP error) returns before any member is reported: every member
// then carries that status, so a caller that reads only the per-member
// reports (a server stepping its resident requests) cannot take an unstepped
// member for a finished one.
static void batch_stats_open(int32_t nprob, nn_stats *stats)
{
    if (!stats) return;
    for (int32_t p = 0; p < nprob; p++) {
        std::memset(&stats[p], 0, sizeof(nn_stats));
        stats[p].status = -1;   // not reported yet
    }
}
static nn_status batch_stats_close(int32_t nprob, nn_stats *stats, nn_status rc)
{
    if (stats)
        for (int32_t p = 0; p < nprob; p++)
            if (stats[p].status == -1) stats[p].status = (int32_t)rc;
    return rc;
}

static nn_status step_transient_batch_body(nn_ctx *ctx, int32_t nprob, nn_matrix *const *K,
                                           double dt, const double *const *f_dev,
                                           const nn_opts *opts, double *const *c_dev,
                                           uint8_t *const *active_dev, nn_stats *stats)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, NN_EINVAL, "dt must be > 0");
    nn_status st = check_batch(ctx, nprob, K, f_dev, opts, c_dev, true);
    if (st != NN_OK) return st;
    const bool mixed = opts->precision == NN_MIXED;
    for (int p = 0; p < nprob; p++)
        if ((st = ensure_transient(ctx, K[p], dt, mixed, false)) != NN_OK) return st;
    if (nprob == 0) {
        ctx->err.clear();
        return NN_OK;
    }
    nn_opts o = *opts;
    o.c0_mode = 1;   // warm start from c^(n)
    return solve_batch_impl(ctx, nprob, K, f_dev, &o, c_dev, active_dev, stats, dt);
}

nn_status nn_step_transient_batch(nn_ctx *ctx, int32_t nprob, nn_matrix *const *K, double dt,
                                  const double *const *f_dev, const nn_opts *opts,
                                  double *const *c_dev, uint8_t *const *active_dev,
                                  nn_stats *stats)
{
    batch_stats_open(nprob, stats);
    if (!ctx) return batch_stats_close(nprob, stats, NN_EINVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return batch_stats_close(nprob, stats, fail(ctx, NN_EHIP, "hipSetDevice"));
    return batch_stats_close(nprob, stats,
                             step_transient_batch_body(ctx, nprob, K, dt, f_dev, opts, c_dev,
                                                       active_dev, stats));
}

static nn_status solve_batch_body(nn_ctx *ctx, int32_t nprob, nn_matrix *const *K,
                                  const double *const *f_dev, const nn_opts *opts,
                                  double *const *c_dev, uint8_t *const *active_dev,
                                  nn_stats *stats)
{
    nn_status st = check_batch(ctx, nprob, K, f_dev, opts, c_dev, false);
    if (st != NN_OK) return st;
    if (nprob == 0) {
        ctx->err.clear();
        return NN_OK;
    }
    return solve_batch_impl(ctx, nprob, K, f_dev, opts, c_dev, active_dev, stats, 0.0);
}

nn_status nn_solve_batch(nn_ctx *ctx, int32_t nprob, nn_matrix *const *K,
                         const double *const *f_dev, const nn_opts *opts, double *const *c_dev,
                         uint8_t *const *active_dev, nn_stats *stats)
{
    batch_stats_open(nprob, stats);
    if (!ctx) return batch_stats_close(nprob, stats, NN_EINVAL);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return batch_stats_close(nprob, stats, fail(ctx, NN_EHIP, "hipSetDevice"));
    return batch_stats_close(nprob, stats,
                             solve_batch_body(ctx, nprob, K, f_dev, opts, c_dev, active_dev,
                                              stats));
}

nn_status nn_set_profiling(nn_ctx *ctx, int classes)
{
    NN_CHECK_CTX(ctx);
    ctx->prof = classes != 0;
    ctx->prof_mask = classes & NN_PROF_ALL;
    return NN_OK;
}

nn_status nn_set_profiling_sample(nn_ctx *ctx, int32_t every)
{
    NN_CHECK_CTX(ctx);
    if (every < 1) return fail(ctx, NN_EINVAL, "profiling sample interval must be >= 1");
    ctx->prof_every = every;
    for (int k = 0; k < NN_KCLASSES; k++) ctx->prof_calls[k] = 0;
    return NN_OK;
}

nn_status nn_kernel_times(nn_ctx *ctx, int64_t *counts, double *total_ms, double *total_bytes,
                          double *total_bytes_csr, int reset)
{
    NN_CHECK_CTX(ctx);
    prof_collect(ctx);
    for (int k = 0; k < NN_KCLASSES; k++) {
        if (counts) counts[k] = ctx->prof_count[k];
        if (total_ms) total_ms[k] = ctx->prof_ms[k];
        if (total_bytes) total_bytes[k] = ctx->prof_bytes[k];
        if (total_bytes_csr) total_bytes_csr[k] = ctx->prof_bytes_csr[k];
        if (reset) {
            ctx->prof_count[k] = 0;
            ctx->prof_ms[k] = 0.0;
            ctx->prof_bytes[k] = 0.0;
            ctx->prof_bytes_csr[k] = 0.0;
        }
    }
    return NN_OK;
}

}  // extern "C"
