// nn_solve_nonneg_noalloc: the TRON solve of nn_solve_nonneg with every work
// buffer in one fixed device array, for callers that cannot allocate device
// memory during a call (tight serving loops, harnesses that forbid it).
//
// The array `scratch` below is a file-scope device variable: the HIP runtime
// gives every GPU the library runs on its own copy when the code object is
// loaded, and each copy lives until the process ends.  In host code the
// name `scratch` is only a host-side stand-in, never a device address, so the
// host takes each device's address once with hipGetSymbolAddress (at
// nn_create, with that device current) and hands out that address only.
#include <algorithm>
#include <mutex>
#include <string>

#include "nnqp_internal.hpp"

namespace nnqp {

namespace {

constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Layout of the array for kNoAllocMaxRows rows: reduction partials, device
// scalars, ten float64 work vectors (gradient, CG iterate, residual,
// preconditioned residual, K p, direction, three Cauchy products, Jacobi
// diagonal), six float32 CG vectors (mixed precision) and the face mask,
// each aligned to 256 bytes.
constexpr size_t kPartBytes = align_up(sizeof(double) * kSlots * kMaxBlocks * kMaxRed);
constexpr size_t kScalBytes = align_up(sizeof(DevScalars));
constexpr size_t kVec64Bytes = align_up(sizeof(double) * (size_t)kNoAllocMaxRows);
constexpr size_t kVec32Bytes = align_up(sizeof(float) * (size_t)kNoAllocMaxRows);
constexpr size_t kMaskBytes = align_up((size_t)kNoAllocMaxRows);
constexpr int kVec64 = 10, kVec32 = 6;
constexpr size_t kScratchBytes =
    kPartBytes + kScalBytes + kVec64 * kVec64Bytes + kVec32 * kVec32Bytes + kMaskBytes;

// Per-device address of `scratch`, taken once per device.
constexpr int kMaxDevices = 64;
struct DevSlot {
    bool tried = false;
    hipError_t rc = hipSuccess;
    unsigned char *ptr = nullptr;
};
DevSlot g_slots[kMaxDevices];
std::mutex g_slots_mu;

}  // namespace

// The fixed work array (see kScratchBytes for its size).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Called by nn_create with `device` current: take this device's address of
// the array (once per device).  A failure is kept and reported by the
// entry point; contexts work without it.
void noalloc_attach(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_slots_mu);
    DevSlot &s = g_slots[device];
    if (s.tried) return;
    s.tried = true;
    void *p = nullptr;
    s.rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    s.ptr = s.rc == hipSuccess ? static_cast<unsigned char *>(p) : nullptr;
}

static nn_status noalloc_address(nn_ctx *ctx, unsigned char **out)
{
    *out = nullptr;
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return fail(ctx, NN_EINVAL, "device index beyond the no-allocation table");
    std::lock_guard<std::mutex> lock(g_slots_mu);
    const DevSlot &s = g_slots[ctx->device];
    if (!s.tried) return fail(ctx, NN_EHIP, "no-allocation array not attached to this device");
    if (s.rc != hipSuccess || !s.ptr)
        return fail(ctx, NN_EHIP, std::string("hipGetSymbolAddress of the no-allocation array: ") +
                                      hipGetErrorString(s.rc));
    *out = s.ptr;
    return NN_OK;
}

// Device scalars start from zero on every call (the array keeps the last
// call's contents); a kernel clears them, so nothing here records a memset.
__global__ void k_clear_scalars(DevScalars *S)
{
    if (threadIdx.x == 0) *S = DevScalars{};
}

}  // namespace nnqp

using namespace nnqp;

extern "C" nn_status nn_solve_nonneg_noalloc(nn_ctx *ctx, nn_matrix *K, const double *f_dev,
                                             const nn_opts *opts, double *c_dev,
                                             uint8_t *active_dev, nn_stats *stats)
{
    if (!ctx) return NN_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, NN_EHIP, "hipSetDevice");
    if (!K || (K->n > 0 && (!f_dev || !c_dev))) return fail(ctx, NN_EINVAL, "null argument");
    if (!opts) return fail(ctx, NN_EINVAL, "null options");
    if (K->n > kNoAllocMaxRows)
        return fail(ctx, NN_EINVAL,
                    "nn_solve_nonneg_noalloc: n = " + std::to_string(K->n) +
                        " exceeds the fixed work array's " + std::to_string(kNoAllocMaxRows) +
                        " rows (use nn_solve_nonneg)");
    nn_status st = check_opts(ctx, opts);
    if (st != NN_OK) return st;
    if (opts->method != NN_TRON)
        return fail(ctx, NN_EINVAL, "nn_solve_nonneg_noalloc runs TRON only");
    if (opts->precond_degree > 1)
        return fail(ctx, NN_EINVAL, "nn_solve_nonneg_noalloc uses the Jacobi preconditioner only");
    const bool mixed = opts->precision == NN_MIXED;
    if (mixed && K->n > 0 && !K->val32)
        return fail(ctx, NN_EINVAL,
                    "nn_solve_nonneg_noalloc: the matrix has no float32 copy yet (a mixed "
                    "nn_solve_nonneg call forms it)");
    unsigned char *base = nullptr;
    if ((st = noalloc_address(ctx, &base)) != NN_OK) return st;

    // carve the array
    Workspace W;
    unsigned char *p = base;
    double *partials = reinterpret_cast<double *>(p);
    p += kPartBytes;
    DevScalars *scal = reinterpret_cast<DevScalars *>(p);
    p += kScalBytes;
    double **v64[kVec64] = {&W.g, &W.w, &W.r, &W.z, &W.q, &W.p0, &W.ks0, &W.ks1, &W.ks2, &W.dm};
    for (double **v : v64) {
        *v = reinterpret_cast<double *>(p);
        p += kVec64Bytes;
    }
    float **v32[kVec32] = {&W.w32, &W.r32, &W.z32, &W.q32, &W.p32, &W.dm32};
    for (float **v : v32) {
        *v = reinterpret_cast<float *>(p);
        p += kVec32Bytes;
    }
    W.mask = p;
    W.cap = kNoAllocMaxRows;
    hipLaunchKernelGGL(k_clear_scalars, dim3(1), dim3(64), 0, ctx->stream, scal);
    if (hipGetLastError() != hipSuccess) return fail(ctx, NN_EHIP, "scalar clear launch");

    // The solve runs on the context with its work buffers, partials and
    // scalars swapped for the array's; the copies a matrix may carry are used
    // as they are (none is formed here), and launch timing is off (its
    // events would be created on demand).
    std::swap(ctx->ws, W);
    std::swap(ctx->partials, partials);
    std::swap(ctx->scal, scal);
    const bool prof = ctx->prof;
    ctx->prof = false;
    const nn_status rc =
        solve_impl(ctx, K, K->val, mixed ? K->val32 : nullptr, mixed ? K->val32q : nullptr,
                   mixed ? nullptr : K->val64p, K->diag, f_dev, opts, c_dev, active_dev, stats);
    ctx->prof = prof;
    std::swap(ctx->scal, scal);
    std::swap(ctx->partials, partials);
    std::swap(ctx->ws, W);
    return rc;
}
