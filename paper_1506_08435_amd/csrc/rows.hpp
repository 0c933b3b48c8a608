// Device-side building blocks shared by the row-parallel kernels of
// kernels.hip and blmvm.hip: fixed-order block reductions into per-block
// partials, the slice walkers over the 64-row sliced-ELL layout, and the
// projection on the bounds.  Header-only (templates and inline functions).
#pragma once

#include <cmath>
#include <type_traits>

#include "nnqp_internal.hpp"

namespace nnqp {

// ---------------------------------------------------------------- reductions
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

// Block-wide combination (waves in order) of a[]; every thread gets the block
// total.  Thread k combines value k across the waves, so the combine costs a
// handful of registers instead of one per wave and value.
template <uint32_t OPS, int NV>
__device__ __forceinline__ void block_red(double (&a)[NV], double (*sh)[NV + 1])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_red<OPS, NV>(a);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) sh[wid][k] = a[k];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        const int op = (int)((OPS >> (2 * k)) & 3u);
        double v = sh[0][k];
#pragma nounroll
        for (int w = 1; w < kWaves; w++) v = red_comb(op, v, sh[w][k]);
        sh[kWaves][k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) a[k] = sh[kWaves][k];
}

__host__ __device__ __forceinline__ double *slot_ptr(double *partials, int s)
{
    return partials + (size_t)s * kMaxRed * kMaxBlocks;
}

// Store this block's total of a[] as its partial: slot[k * kMaxBlocks + block].
template <uint32_t OPS, int NV>
__device__ __forceinline__ void block_partial(double (&a)[NV], double *slot)
{
    __shared__ double sh[kWaves + 1][NV + 1];
    block_red<OPS, NV>(a, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) slot[k * kMaxBlocks + blockIdx.x] = a[k];
}

// Combine the partials of `nb` blocks left in `slot` by the previous kernel:
// every block runs the same fixed-order combination and gets the same bits.
template <uint32_t OPS, int NV>
__device__ __forceinline__ void combine_partials(const double *slot, int nb, double (&a)[NV])
{
    __shared__ double sh[kWaves + 1][NV + 1];
    red_init<OPS, NV>(a);
    for (int b = threadIdx.x; b < nb; b += kBlock)
#pragma unroll
        for (int k = 0; k < NV; k++) a[k] = red_comb(op_of<OPS>(k), a[k], slot[k * kMaxBlocks + b]);
    block_red<OPS, NV>(a, sh);
}

// Index of the calling wavefront in its block.  It is uniform in the
// wavefront; readfirstlane states that to the compiler, so the slice index,
// the slice offsets and width and the loop bounds derived from it live in
// scalar registers (the row passes of the batched solver dropped from 54 to
// 43 VGPRs with it).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ---------------------------------------------------------------- slice walkers
// Calls body(i, act) for the row i = 64 s + lane of every slice s this
// wavefront owns; act = i < n.  The loop trip count is uniform in a wavefront.
template <class Body>
__device__ __forceinline__ void for_rows(const Part &P, Body body)
{
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int nw = P.nb * kWaves;
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += nw) {
        const int i = s * kSlice + lane;
        body(i, i < P.n);
    }
}

// Column readers of the sliced-ELL entries (entry e of the slice holding row).
// Float32-value passes read int16 offsets from the row when the pattern
// allows (|col - row| <= 32767); float64-value passes, and patterns with
// wider offsets, read int32 columns.
struct ColsI32 {
    const int *c;
    __device__ __forceinline__ int operator()(int e, int) const { return c[e]; }
};
struct ColsD16 {
    const short *d;
    __device__ __forceinline__ int operator()(int e, int row) const { return row + (int)d[e]; }
};
// int16 offsets in the paired layout (see nn_matrix::d16p)
struct ColsD16P {
    const short *d;
    __device__ __forceinline__ int operator()(int e, int row) const { return row + (int)d[e]; }
};
// int16 offsets in the quad layout (see nn_matrix::d16q)
struct ColsD16Q {
    const short *d;
    __device__ __forceinline__ int operator()(int e, int row) const { return row + (int)d[e]; }
};

// Matrix values are read once per pass.  Float64 values are loaded with the
// non-temporal hint, which keeps the value stream from displacing the
// gathered vector in the caches (measured on the 128^3 pattern: the CG matrix
// pass 97 -> 80 us); for float32 values the hint is slower, so they load
// normally.
__device__ __forceinline__ double ld_val(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_val(const float *p) { return *p; }

// Both values of a pair in the paired layout (8-byte aligned for float32,
// 16-byte aligned for float64): one 8- or 16-byte load, with the same hint
// choice as ld_val.
__device__ __forceinline__ void ld_pair(const float *p, float &a, float &b)
{
    const float2 v = *reinterpret_cast<const float2 *>(p);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void ld_pair(const double *p, double &a, double &b)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
    a = v.x;
    b = v.y;
}

// Sliced-ELL product row by row: for each owned row i with active(i), the sum
// over the row's entries k = 0..w-1 (column order) of val * x(col), then
// epi(i, sum, pre(i)).  Padding entries have value 0 and column i.
// The SpMV passes are latency-bound (each slice is a chain: offsets ->
// indices/values -> gathers -> own-row data -> stores), so a wavefront keeps
// NS slices in flight at once, issues the slice offsets and the own-row loads
// of pre() before any gather, and loads entries eight at a time (all eight
// before their gathers, which keeps the kernels under 64 VGPRs).  Slices wider
// than WMAX finish in a plain loop.  The single-product walks of the paired
// and quad layouts take slices up to WMAX wide with pair_row_flat and
// quad_row_flat, which keep every load of a phase in flight together.
#ifndef NNQP_SLICES_IN_FLIGHT
#define NNQP_SLICES_IN_FLIGHT 1
#endif
#ifndef NNQP_LOAD_PHASE
#define NNQP_LOAD_PHASE 8
#endif
#ifndef NNQP_FLAT_PAIRS
#define NNQP_FLAT_PAIRS 1   // paired layout: pair_row_flat for slices of width <= WMAX
#endif
// Paired layout (ColsD16P): the pair (2k, 2k+1) of the row of lane l sits at
// off + 128 k + 2 l, so one 8-byte (float32) or 16-byte (float64) load brings
// both values and one 4-byte load both offsets; an odd last column stays
// column-major and is loaded after the pairs in the guarded walk (loading it
// with the last pairs there held more registers and, for float64 values,
// cost a wave per SIMD: the 128^3 CG matrix pass went from 78 to 100 us).
//
// The row sum of sell_rows_paired for a slice of width w <= WMAX, written as
// quad_row_flat (below): HP pairs per phase, the odd last entry in the last
// phase, loads under guards that only move raw bits, gathers unconditional,
// products added in entry order with selects.  One pair per phase measured
// best on the 128^3 float64 CG pass: 70.7-71.7 us, against 74.6-75.9 us for
// the guarded walk, 73.9-75.4 us with two pairs and 74.8 us with four pairs
// per phase (65 VGPRs, seven waves per SIMD).
template <int WMAX, int HP, class VT, class X>
__device__ __forceinline__ double pair_row_flat(const VT *__restrict__ sv,
                                                const short *__restrict__ d16, int off, int w,
                                                int row, int safe, X x)
{
    const int lane = threadIdx.x & 63;
    const int np = w >> 1;
    constexpr int NP = WMAX / 2 > 0 ? WMAX / 2 : 1;   // pairs of the widest slice
    double acc = 0.0;
#pragma unroll
    for (int h0 = 0; h0 < NP; h0 += HP) {
        const bool last = h0 + HP >= NP;
        if (!last && h0 >= np) continue;   // wave-uniform
        VT v[HP][2];
        int d[HP];
#pragma unroll
        for (int k = 0; k < HP; k++) {
            if (h0 + k < np) {
                const int e = off + (h0 + k) * 2 * kSlice + 2 * lane;
                ld_pair(sv + e, v[k][0], v[k][1]);
                d[k] = *reinterpret_cast<const int *>(d16 + e);
            } else {
                v[k][0] = v[k][1] = VT(0);
                d[k] = 0;
            }
        }
        VT sg = VT(0);
        int dsg = 0;
        if (last && (w & 1)) {
            const int e = off + (w - 1) * kSlice + lane;
            sg = ld_val(sv + e);
            dsg = d16[e];
        }
        double xv[2 * HP];
#pragma unroll
        for (int k = 0; k < HP; k++) {
            const bool ok = h0 + k < np;
            xv[2 * k] = x(ok ? row + (int)(short)(d[k] & 0xffff) : safe);
            xv[2 * k + 1] = x(ok ? row + (d[k] >> 16) : safe);
        }
        const double xs = last ? x((w & 1) ? row + dsg : safe) : 0.0;
#pragma unroll
        for (int k = 0; k < HP; k++)
#pragma unroll
            for (int t = 0; t < 2; t++) {
                const double y = __builtin_fma((double)v[k][t], xv[2 * k + t], acc);
                acc = h0 + k < np ? y : acc;
            }
        if (last) {
            const double y = __builtin_fma((double)sg, xs, acc);
            acc = (w & 1) ? y : acc;
        }
    }
    return acc;
}

#ifndef NNQP_PAIR_FLAT_PHASE
#define NNQP_PAIR_FLAT_PHASE 2   // entries per load phase of pair_row_flat
#endif
template <int WMAX, class VT, class Act, class Pre, class X, class Epi>
__device__ __forceinline__ void sell_rows_paired(const Part &P, const int *__restrict__ so,
                                                 ColsD16P sc, const VT *__restrict__ sv,
                                                 Act active, Pre pre, X x, Epi epi)
{
    using PV = decltype(pre(0));
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int nw = P.nb * kWaves;
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += nw) {
        const int off = so[s];
        const int w = (so[s + 1] - off) >> 6;   // uniform in the wave
        const int np = w >> 1;
        const int row = s * kSlice + lane;
        const bool act = row < P.n && active(row);
        const PV pv = act ? pre(row) : PV();
        if (__ballot(act) == 0) continue;
        if (NNQP_FLAT_PAIRS && w <= WMAX) {
            constexpr int HP = (WMAX < NNQP_PAIR_FLAT_PHASE ? WMAX : NNQP_PAIR_FLAT_PHASE) / 2;
            const int safe = row < P.n ? row : P.n - 1;   // an index every vector has
            const double acc = pair_row_flat<WMAX, HP>(sv, sc.d, off, w, row, safe, x);
            if (act) epi(row, acc, pv);
            continue;
        }
        double acc = 0.0;
        constexpr int H = (WMAX < NNQP_LOAD_PHASE ? WMAX : NNQP_LOAD_PHASE) / 2;   // pairs per phase
#pragma unroll
        for (int h0 = 0; h0 < WMAX / 2; h0 += H) {
            int cc[2 * H];
            VT vv[2 * H];
#pragma unroll
            for (int k = 0; k < H; k++) {
                if (h0 + k < np) {
                    const int e = off + (h0 + k) * 2 * kSlice + 2 * lane;
                    ld_pair(sv + e, vv[2 * k], vv[2 * k + 1]);
                    const int d2 = *reinterpret_cast<const int *>(sc.d + e);
                    cc[2 * k] = row + (int)(short)(d2 & 0xffff);
                    cc[2 * k + 1] = row + (d2 >> 16);
                } else {
                    cc[2 * k] = cc[2 * k + 1] = 0;
                    vv[2 * k] = vv[2 * k + 1] = VT(0);
                }
            }
#pragma unroll
            for (int k = 0; k < 2 * H; k++)
                if (h0 + k / 2 < np) acc += (double)vv[k] * x(cc[k]);
        }
        for (int k = WMAX / 2; k < np; k++) {
            const int e = off + k * 2 * kSlice + 2 * lane;
            acc += (double)ld_val(sv + e) * x(sc(e, row));
            acc += (double)ld_val(sv + e + 1) * x(sc(e + 1, row));
        }
        if (w & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            acc += (double)ld_val(sv + e) * x(sc(e, row));
        }
        if (act) epi(row, acc, pv);
    }
}

// Quad layout of float32 values (ColsD16Q): the entries 4k .. 4k+3 of the
// row of lane l sit at off + 256 k + 4 l, so one 16-byte load brings four
// values and one 8-byte load their four offsets; two entries left over sit
// as a pair at off + 256 (w / 4) + 2 l, and an odd last one keeps its
// column-major place.  A 3D row of 15 entries takes five value loads (three
// quads, a pair, a single) instead of eight in the paired layout: the
// float32 passes are bound by load instructions more than by bytes.
// Entries per load phase of the guarded quad walker (slices wider than the
// unrolled part, and the multi-trial passes), and the non-temporal hint on
// the quad loads (bit 0: values, bit 1: offsets).  Measured on the 128^3
// float32 CG pass with the guarded walk (per launch): 8 entries, no hint
// 49.3 us; 4 entries 50.1 us; 16 entries 71.6 us (80 VGPRs, six waves per
// SIMD); hint on values 55.7 us, on both 59.1 us.
#ifndef NNQP_QUAD_PHASE
#define NNQP_QUAD_PHASE NNQP_LOAD_PHASE
#endif
#ifndef NNQP_QUAD_NT
#define NNQP_QUAD_NT 0
#endif
__device__ __forceinline__ float4 ld_quad(const float *p)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 *q = reinterpret_cast<const f4 *>(p);
    const f4 v = (NNQP_QUAD_NT & 1) ? __builtin_nontemporal_load(q) : *q;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int2 ld_quad_d(const short *p)
{
    typedef int i2 __attribute__((ext_vector_type(2)));
    const i2 *q = reinterpret_cast<const i2 *>(p);
    const i2 v = (NNQP_QUAD_NT & 2) ? __builtin_nontemporal_load(q) : *q;
    return make_int2(v.x, v.y);
}

// The row sum of sell_rows_quad for a slice of width w <= WMAX, phase by
// phase with no load waiting for another: the quads of a phase (and, in the
// last phase, the pair and the single left over) are loaded under
// wave-uniform guards that only move raw bits, so the compiler has no reason
// to wait for them there; then every gather of the phase is issued, then the
// products are added in entry order with fused multiply-adds.  A slot past
// the slice's width gathers x(safe), where safe is the row itself or, for the
// lanes past the last row, row n - 1 (an index every vector has), and its
// product is not added (a select), so the sum is bitwise the one of the
// guarded walk.  (Decoding the columns inside the guards made every
// quad and every gather a round trip of its own.)  On the 128^3 float32 CG
// pass: one quad per phase 39.9-40.1 us (64 VGPRs), two 49.0 us and four
// 50.1 us (80 VGPRs, six waves per SIMD), the guarded walk 46.5 us.
#ifndef NNQP_FLAT_ROWS
#define NNQP_FLAT_ROWS 1
#endif
#ifndef NNQP_QUAD_FLAT_PHASE
#define NNQP_QUAD_FLAT_PHASE 4   // entries per load phase of quad_row_flat
#endif
template <int WMAX, int HQ, class X>
__device__ __forceinline__ double quad_row_flat(const float *__restrict__ sv,
                                                const short *__restrict__ d16, int off, int w,
                                                int row, int safe, X x)
{
    const int lane = threadIdx.x & 63;
    const int nq = w >> 2, rem = w & 3;
    constexpr int NQ = WMAX / 4 > 0 ? WMAX / 4 : 1;   // quads of the widest slice
    double acc = 0.0;
#pragma unroll
    for (int h0 = 0; h0 < NQ; h0 += HQ) {
        const bool last = h0 + HQ >= NQ;
        if (!last && h0 >= nq) continue;   // wave-uniform
        float q[HQ][4];
        int2 dq[HQ];
#pragma unroll
        for (int k = 0; k < HQ; k++) {
            if (h0 + k < nq) {
                const int e = off + (h0 + k) * 4 * kSlice + 4 * lane;
                const float4 v = ld_quad(sv + e);
                dq[k] = ld_quad_d(d16 + e);
                q[k][0] = v.x;
                q[k][1] = v.y;
                q[k][2] = v.z;
                q[k][3] = v.w;
            } else {
                q[k][0] = q[k][1] = q[k][2] = q[k][3] = 0.f;
                dq[k] = make_int2(0, 0);
            }
        }
        float pa = 0.f, pb = 0.f, sg = 0.f;
        int dp = 0, dsg = 0;
        if (last) {
            if (rem >= 2) {
                const int e = off + nq * 4 * kSlice + 2 * lane;
                ld_pair(sv + e, pa, pb);
                dp = *reinterpret_cast<const int *>(d16 + e);
            }
            if (rem & 1) {
                const int e = off + (w - 1) * kSlice + lane;
                sg = ld_val(sv + e);
                dsg = d16[e];
            }
        }
        double xv[4 * HQ];
#pragma unroll
        for (int k = 0; k < HQ; k++) {
            const bool ok = h0 + k < nq;
            xv[4 * k] = x(ok ? row + (int)(short)(dq[k].x & 0xffff) : safe);
            xv[4 * k + 1] = x(ok ? row + (dq[k].x >> 16) : safe);
            xv[4 * k + 2] = x(ok ? row + (int)(short)(dq[k].y & 0xffff) : safe);
            xv[4 * k + 3] = x(ok ? row + (dq[k].y >> 16) : safe);
        }
        double xp = 0.0, xq = 0.0, xs = 0.0;
        if (last) {
            xp = x(rem >= 2 ? row + (int)(short)(dp & 0xffff) : safe);
            xq = x(rem >= 2 ? row + (dp >> 16) : safe);
            xs = x((rem & 1) ? row + dsg : safe);
        }
#pragma unroll
        for (int k = 0; k < HQ; k++)
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const double y = __builtin_fma((double)q[k][t], xv[4 * k + t], acc);
                acc = h0 + k < nq ? y : acc;
            }
        if (last) {
            const double y0 = __builtin_fma((double)pa, xp, acc);
            acc = rem >= 2 ? y0 : acc;
            const double y1 = __builtin_fma((double)pb, xq, acc);
            acc = rem >= 2 ? y1 : acc;
            const double y2 = __builtin_fma((double)sg, xs, acc);
            acc = (rem & 1) ? y2 : acc;
        }
    }
    return acc;
}

template <int WMAX, class VT, class Act, class Pre, class X, class Epi>
__device__ __forceinline__ void sell_rows_quad(const Part &P, const int *__restrict__ so,
                                               ColsD16Q sc, const VT *__restrict__ sv, Act active,
                                               Pre pre, X x, Epi epi)
{
    static_assert(sizeof(VT) == 4, "the quad layout holds float32 values");
    using PV = decltype(pre(0));
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int nw = P.nb * kWaves;
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += nw) {
        const int off = so[s];
        const int w = (so[s + 1] - off) >> 6;   // uniform in the wave
        const int nq = w >> 2, rem = w & 3;
        const int row = s * kSlice + lane;
        const bool act = row < P.n && active(row);
        const PV pv = act ? pre(row) : PV();
        if (__ballot(act) == 0) continue;
        constexpr int HQ = (WMAX < NNQP_QUAD_PHASE ? WMAX : NNQP_QUAD_PHASE) / 4;   // quads per phase
        if (NNQP_FLAT_ROWS && w <= WMAX) {
            constexpr int HF = NNQP_QUAD_FLAT_PHASE / 4 > 0 ? NNQP_QUAD_FLAT_PHASE / 4 : 1;
            const int safe = row < P.n ? row : P.n - 1;   // an index every vector has
            const double acc = quad_row_flat<WMAX, HF>(sv, sc.d, off, w, row, safe, x);
            if (act) epi(row, acc, pv);
            continue;
        }
        double acc = 0.0;
#pragma unroll
        for (int h0 = 0; h0 < WMAX / 4; h0 += HQ) {
            int cc[4 * HQ];
            float vv[4 * HQ];
#pragma unroll
            for (int k = 0; k < HQ; k++) {
                if (h0 + k < nq) {
                    const int e = off + (h0 + k) * 4 * kSlice + 4 * lane;
                    const float4 v = ld_quad(sv + e);
                    const int2 d = ld_quad_d(sc.d + e);
                    vv[4 * k] = v.x;
                    vv[4 * k + 1] = v.y;
                    vv[4 * k + 2] = v.z;
                    vv[4 * k + 3] = v.w;
                    cc[4 * k] = row + (int)(short)(d.x & 0xffff);
                    cc[4 * k + 1] = row + (d.x >> 16);
                    cc[4 * k + 2] = row + (int)(short)(d.y & 0xffff);
                    cc[4 * k + 3] = row + (d.y >> 16);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        cc[4 * k + q] = 0;
                        vv[4 * k + q] = 0.f;
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
            for (int q = 0; q < 4; q++) acc += (double)ld_val(sv + e + q) * x(sc(e + q, row));
        }
        if (rem >= 2) {
            const int e = off + nq * 4 * kSlice + 2 * lane;
            float a, b;
            ld_pair(sv + e, a, b);
            const int d2 = *reinterpret_cast<const int *>(sc.d + e);
            acc += (double)a * x(row + (int)(short)(d2 & 0xffff));
            acc += (double)b * x(row + (d2 >> 16));
        }
        if (rem & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            acc += (double)ld_val(sv + e) * x(sc(e, row));
        }
        if (act) epi(row, acc, pv);
    }
}

template <int WMAX, class VT, class Cols, class Act, class Pre, class X, class Epi>
__device__ __forceinline__ void sell_rows(const Part &P, const int *__restrict__ so, Cols sc,
                                          const VT *__restrict__ sv, Act active, Pre pre, X x,
                                          Epi epi)
{
    if constexpr (std::is_same<Cols, ColsD16P>::value) {
        sell_rows_paired<WMAX>(P, so, sc, sv, active, pre, x, epi);
        return;
    } else if constexpr (std::is_same<Cols, ColsD16Q>::value) {
        sell_rows_quad<WMAX>(P, so, sc, sv, active, pre, x, epi);
        return;
    } else {
    constexpr int NS = NNQP_SLICES_IN_FLIGHT;
    using PV = decltype(pre(0));
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int nw = P.nb * kWaves;
    for (int s0 = blockIdx.x * kWaves + wid; s0 < P.nslices; s0 += NS * nw) {
        int off[NS], w[NS], row[NS];
        bool act[NS];
        PV pv[NS];
#pragma unroll
        for (int t = 0; t < NS; t++) {
            const int s = s0 + t * nw;
            const bool has = s < P.nslices;
            off[t] = has ? so[s] : 0;
            w[t] = has ? (so[s + 1] - off[t]) >> 6 : 0;   // slice width (uniform in the wave)
            row[t] = s * kSlice + lane;
            act[t] = has && row[t] < P.n && active(row[t]);
            pv[t] = act[t] ? pre(row[t]) : PV();
        }
        bool any = false;
#pragma unroll
        for (int t = 0; t < NS; t++) any = any || (__ballot(act[t]) != 0);
        if (!any) continue;
        // Every lane of a live slice loads and gathers under the wave-uniform
        // test k < w: padding and inactive rows hold valid columns, so this
        // stays in bounds, and their sums are discarded below.  Per-lane
        // predication here would cost more issue slots than the bytes saved.
        double acc[NS];
#pragma unroll
        for (int t = 0; t < NS; t++) acc[t] = 0.0;
        constexpr int H = WMAX < NNQP_LOAD_PHASE ? WMAX : NNQP_LOAD_PHASE;
#pragma unroll
        for (int h0 = 0; h0 < WMAX; h0 += H) {
            int cc[NS][H];
            VT vv[NS][H];
#pragma unroll
            for (int t = 0; t < NS; t++)
#pragma unroll
                for (int k = 0; k < H; k++) {
                    if (h0 + k < w[t]) {
                        cc[t][k] = sc(off[t] + (h0 + k) * kSlice + lane, row[t]);
                        vv[t][k] = ld_val(sv + off[t] + (h0 + k) * kSlice + lane);
                    } else {
                        cc[t][k] = 0;
                        vv[t][k] = VT(0);
                    }
                }
#pragma unroll
            for (int t = 0; t < NS; t++)
#pragma unroll
                for (int k = 0; k < H; k++)
                    if (h0 + k < w[t]) acc[t] += (double)vv[t][k] * x(cc[t][k]);
        }
#pragma unroll
        for (int t = 0; t < NS; t++) {
            for (int k = WMAX; k < w[t]; k++) {
                const int e = off[t] + k * kSlice + lane;
                acc[t] += (double)ld_val(sv + e) * x(sc(e, row[t]));
            }
            if (act[t]) epi(row[t], acc[t], pv[t]);
        }
    }
    }
}

#ifndef NNQP_FLAT_MULTI
#define NNQP_FLAT_MULTI 1   // the multi-product walks use the flat row sums below
#endif
// pair_row_flat and quad_row_flat for NT products at once: x(j, out) fills
// NT values per gathered column; acc[t] is the row sum of product t, in the
// same order and with the same fused multiply-adds as the guarded walks.
template <int WMAX, int NT, int HP, class VT, class X>
__device__ __forceinline__ void pair_row_flat_n(const VT *__restrict__ sv,
                                                const short *__restrict__ d16, int off, int w,
                                                int row, int safe, X x, double (&acc)[NT])
{
    const int lane = threadIdx.x & 63;
    const int np = w >> 1;
    constexpr int NP = WMAX / 2 > 0 ? WMAX / 2 : 1;
#pragma unroll
    for (int h0 = 0; h0 < NP; h0 += HP) {
        const bool last = h0 + HP >= NP;
        if (!last && h0 >= np) continue;   // wave-uniform
        VT v[HP][2];
        int d[HP];
#pragma unroll
        for (int k = 0; k < HP; k++) {
            if (h0 + k < np) {
                const int e = off + (h0 + k) * 2 * kSlice + 2 * lane;
                ld_pair(sv + e, v[k][0], v[k][1]);
                d[k] = *reinterpret_cast<const int *>(d16 + e);
            } else {
                v[k][0] = v[k][1] = VT(0);
                d[k] = 0;
            }
        }
        VT sg = VT(0);
        int dsg = 0;
        if (last && (w & 1)) {
            const int e = off + (w - 1) * kSlice + lane;
            sg = ld_val(sv + e);
            dsg = d16[e];
        }
        double xv[2 * HP][NT];
#pragma unroll
        for (int k = 0; k < HP; k++) {
            const bool ok = h0 + k < np;
            x(ok ? row + (int)(short)(d[k] & 0xffff) : safe, xv[2 * k]);
            x(ok ? row + (d[k] >> 16) : safe, xv[2 * k + 1]);
        }
        double xs[NT];
        if (last) x((w & 1) ? row + dsg : safe, xs);
#pragma unroll
        for (int k = 0; k < HP; k++)
#pragma unroll
            for (int u = 0; u < 2; u++)
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const double y = __builtin_fma((double)v[k][u], xv[2 * k + u][t], acc[t]);
                    acc[t] = h0 + k < np ? y : acc[t];
                }
        if (last)
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const double y = __builtin_fma((double)sg, xs[t], acc[t]);
                acc[t] = (w & 1) ? y : acc[t];
            }
    }
}

template <int WMAX, int NT, int HQ, class X>
__device__ __forceinline__ void quad_row_flat_n(const float *__restrict__ sv,
                                                const short *__restrict__ d16, int off, int w,
                                                int row, int safe, X x, double (&acc)[NT])
{
    const int lane = threadIdx.x & 63;
    const int nq = w >> 2, rem = w & 3;
    constexpr int NQ = WMAX / 4 > 0 ? WMAX / 4 : 1;
#pragma unroll
    for (int h0 = 0; h0 < NQ; h0 += HQ) {
        const bool last = h0 + HQ >= NQ;
        if (!last && h0 >= nq) continue;   // wave-uniform
        float q[HQ][4];
        int2 dq[HQ];
#pragma unroll
        for (int k = 0; k < HQ; k++) {
            if (h0 + k < nq) {
                const int e = off + (h0 + k) * 4 * kSlice + 4 * lane;
                const float4 v = ld_quad(sv + e);
                dq[k] = ld_quad_d(d16 + e);
                q[k][0] = v.x;
                q[k][1] = v.y;
                q[k][2] = v.z;
                q[k][3] = v.w;
            } else {
                q[k][0] = q[k][1] = q[k][2] = q[k][3] = 0.f;
                dq[k] = make_int2(0, 0);
            }
        }
        float pa = 0.f, pb = 0.f, sg = 0.f;
        int dp = 0, dsg = 0;
        if (last) {
            if (rem >= 2) {
                const int e = off + nq * 4 * kSlice + 2 * lane;
                ld_pair(sv + e, pa, pb);
                dp = *reinterpret_cast<const int *>(d16 + e);
            }
            if (rem & 1) {
                const int e = off + (w - 1) * kSlice + lane;
                sg = ld_val(sv + e);
                dsg = d16[e];
            }
        }
        double xv[4 * HQ][NT];
#pragma unroll
        for (int k = 0; k < HQ; k++) {
            const bool ok = h0 + k < nq;
            x(ok ? row + (int)(short)(dq[k].x & 0xffff) : safe, xv[4 * k]);
            x(ok ? row + (dq[k].x >> 16) : safe, xv[4 * k + 1]);
            x(ok ? row + (int)(short)(dq[k].y & 0xffff) : safe, xv[4 * k + 2]);
            x(ok ? row + (dq[k].y >> 16) : safe, xv[4 * k + 3]);
        }
        double xr[3][NT];
        if (last) {
            x(rem >= 2 ? row + (int)(short)(dp & 0xffff) : safe, xr[0]);
            x(rem >= 2 ? row + (dp >> 16) : safe, xr[1]);
            x((rem & 1) ? row + dsg : safe, xr[2]);
        }
#pragma unroll
        for (int k = 0; k < HQ; k++)
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const double y = __builtin_fma((double)q[k][u], xv[4 * k + u][t], acc[t]);
                    acc[t] = h0 + k < nq ? y : acc[t];
                }
        if (last)
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const double y0 = __builtin_fma((double)pa, xr[0][t], acc[t]);
                acc[t] = rem >= 2 ? y0 : acc[t];
                const double y1 = __builtin_fma((double)pb, xr[1][t], acc[t]);
                acc[t] = rem >= 2 ? y1 : acc[t];
                const double y2 = __builtin_fma((double)sg, xr[2][t], acc[t]);
                acc[t] = (rem & 1) ? y2 : acc[t];
            }
    }
}

// NT products in one pass: like sell_rows, with x(j, out) filling NT values
// per gathered column and epi(i, acc[NT], pre(i)).  Entries are loaded eight
// at a time before their gathers; one slice per wavefront in flight.
// sell_rows_n on the paired layout (see sell_rows_paired): PHASE / 2 pairs
// per load phase, entries in the same order, so the sums are the same.
template <int WMAX, int NT, class VT, class Pre, class X, class Epi, int PHASE>
__device__ __forceinline__ void sell_rows_n_paired(const Part &P, const int *__restrict__ so,
                                                   ColsD16P sc, const VT *__restrict__ sv,
                                                   Pre pre, X x, Epi epi)
{
    using PV = decltype(pre(0));
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int nw = P.nb * kWaves;
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += nw) {
        const int off = so[s];
        const int w = (so[s + 1] - off) >> 6;
        const int np = w >> 1;
        const int row = s * kSlice + lane;
        const bool act = row < P.n;
        const PV pv = act ? pre(row) : PV();
        double acc[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) acc[t] = 0.0;
        if (NNQP_FLAT_MULTI && w <= WMAX) {
            constexpr int HF = (WMAX < NNQP_PAIR_FLAT_PHASE ? WMAX : NNQP_PAIR_FLAT_PHASE) / 2;
            const int safe = row < P.n ? row : P.n - 1;
            pair_row_flat_n<WMAX, NT, HF>(sv, sc.d, off, w, row, safe, x, acc);
            if (act) epi(row, acc, pv);
            continue;
        }
        constexpr int H = (WMAX < PHASE ? WMAX : PHASE) / 2;   // pairs per phase
        double xv[NT];
#pragma unroll
        for (int h0 = 0; h0 < WMAX / 2; h0 += H) {
            int cc[2 * H];
            VT vv[2 * H];
#pragma unroll
            for (int k = 0; k < H; k++) {
                if (h0 + k < np) {
                    const int e = off + (h0 + k) * 2 * kSlice + 2 * lane;
                    ld_pair(sv + e, vv[2 * k], vv[2 * k + 1]);
                    const int d2 = *reinterpret_cast<const int *>(sc.d + e);
                    cc[2 * k] = row + (int)(short)(d2 & 0xffff);
                    cc[2 * k + 1] = row + (d2 >> 16);
                } else {
                    cc[2 * k] = cc[2 * k + 1] = 0;
                    vv[2 * k] = vv[2 * k + 1] = VT(0);
                }
            }
#pragma unroll
            for (int k = 0; k < 2 * H; k++)
                if (h0 + k / 2 < np) {
                    x(cc[k], xv);
#pragma unroll
                    for (int t = 0; t < NT; t++) acc[t] += (double)vv[k] * xv[t];
                }
        }
        for (int k = WMAX / 2; k < np; k++)
            for (int q = 0; q < 2; q++) {
                const int e = off + k * 2 * kSlice + 2 * lane + q;
                x(sc(e, row), xv);
                const double vk = (double)ld_val(sv + e);
#pragma unroll
                for (int t = 0; t < NT; t++) acc[t] += vk * xv[t];
            }
        if (w & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            x(sc(e, row), xv);
            const double vk = (double)ld_val(sv + e);
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t] += vk * xv[t];
        }
        if (act) epi(row, acc, pv);
    }
}

// sell_rows_n on the quad layout (see sell_rows_quad): PHASE / 4 quads per
// load phase (at least one), entries in the same order, so the sums are the
// same as on the column-major copy.
template <int WMAX, int NT, class VT, class Pre, class X, class Epi, int PHASE>
__device__ __forceinline__ void sell_rows_n_quad(const Part &P, const int *__restrict__ so,
                                                 ColsD16Q sc, const VT *__restrict__ sv, Pre pre,
                                                 X x, Epi epi)
{
    static_assert(sizeof(VT) == 4, "the quad layout holds float32 values");
    using PV = decltype(pre(0));
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int nw = P.nb * kWaves;
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += nw) {
        const int off = so[s];
        const int w = (so[s + 1] - off) >> 6;
        const int nq = w >> 2, rem = w & 3;
        const int row = s * kSlice + lane;
        const bool act = row < P.n;
        const PV pv = act ? pre(row) : PV();
        double acc[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) acc[t] = 0.0;
        if (NNQP_FLAT_MULTI && w <= WMAX) {
            constexpr int HF = NNQP_QUAD_FLAT_PHASE / 4 > 0 ? NNQP_QUAD_FLAT_PHASE / 4 : 1;
            const int safe = row < P.n ? row : P.n - 1;
            quad_row_flat_n<WMAX, NT, HF>(sv, sc.d, off, w, row, safe, x, acc);
            if (act) epi(row, acc, pv);
            continue;
        }
        constexpr int HP = WMAX < PHASE ? WMAX : PHASE;
        constexpr int HQ = HP / 4 > 0 ? HP / 4 : 1;   // quads per phase
        double xv[NT];
#pragma unroll
        for (int h0 = 0; h0 < WMAX / 4; h0 += HQ) {
            int cc[4 * HQ];
            float vv[4 * HQ];
#pragma unroll
            for (int k = 0; k < HQ; k++) {
                if (h0 + k < nq) {
                    const int e = off + (h0 + k) * 4 * kSlice + 4 * lane;
                    const float4 v = ld_quad(sv + e);
                    const int2 d = ld_quad_d(sc.d + e);
                    vv[4 * k] = v.x;
                    vv[4 * k + 1] = v.y;
                    vv[4 * k + 2] = v.z;
                    vv[4 * k + 3] = v.w;
                    cc[4 * k] = row + (int)(short)(d.x & 0xffff);
                    cc[4 * k + 1] = row + (d.x >> 16);
                    cc[4 * k + 2] = row + (int)(short)(d.y & 0xffff);
                    cc[4 * k + 3] = row + (d.y >> 16);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        cc[4 * k + q] = 0;
                        vv[4 * k + q] = 0.f;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 4 * HQ; k++)
                if (h0 + k / 4 < nq) {
                    x(cc[k], xv);
#pragma unroll
                    for (int t = 0; t < NT; t++) acc[t] += (double)vv[k] * xv[t];
                }
        }
        for (int k = WMAX / 4; k < nq; k++)   // slices wider than the unrolled part
            for (int q = 0; q < 4; q++) {
                const int e = off + k * 4 * kSlice + 4 * lane + q;
                x(sc(e, row), xv);
                const double vk = (double)ld_val(sv + e);
#pragma unroll
                for (int t = 0; t < NT; t++) acc[t] += vk * xv[t];
            }
        if (rem >= 2) {
            const int e = off + nq * 4 * kSlice + 2 * lane;
            float a, b;
            ld_pair(sv + e, a, b);
            const int d2 = *reinterpret_cast<const int *>(sc.d + e);
            x(row + (int)(short)(d2 & 0xffff), xv);
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t] += (double)a * xv[t];
            x(row + (d2 >> 16), xv);
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t] += (double)b * xv[t];
        }
        if (rem & 1) {
            const int e = off + (w - 1) * kSlice + lane;
            x(sc(e, row), xv);
            const double vk = (double)ld_val(sv + e);
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t] += vk * xv[t];
        }
        if (act) epi(row, acc, pv);
    }
}

template <int WMAX, int NT, class VT, class Cols, class Pre, class X, class Epi,
          int PHASE = NNQP_LOAD_PHASE>
__device__ __forceinline__ void sell_rows_n(const Part &P, const int *__restrict__ so, Cols sc,
                                            const VT *__restrict__ sv, Pre pre, X x, Epi epi)
{
    if constexpr (std::is_same<Cols, ColsD16P>::value) {
        sell_rows_n_paired<WMAX, NT, VT, Pre, X, Epi, PHASE>(P, so, sc, sv, pre, x, epi);
        return;
    } else if constexpr (std::is_same<Cols, ColsD16Q>::value) {
        sell_rows_n_quad<WMAX, NT, VT, Pre, X, Epi, PHASE>(P, so, sc, sv, pre, x, epi);
        return;
    } else {
    using PV = decltype(pre(0));
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int nw = P.nb * kWaves;
    for (int s = blockIdx.x * kWaves + wid; s < P.nslices; s += nw) {
        const int off = so[s];
        const int w = (so[s + 1] - off) >> 6;
        const int row = s * kSlice + lane;
        const bool act = row < P.n;
        const PV pv = act ? pre(row) : PV();
        double acc[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) acc[t] = 0.0;
        constexpr int H = WMAX < PHASE ? WMAX : PHASE;
        double xv[NT];
#pragma unroll
        for (int h0 = 0; h0 < WMAX; h0 += H) {
            int cc[H];
            VT vv[H];
#pragma unroll
            for (int k = 0; k < H; k++) {
                if (h0 + k < w) {
                    cc[k] = sc(off + (h0 + k) * kSlice + lane, row);
                    vv[k] = ld_val(sv + off + (h0 + k) * kSlice + lane);
                } else {
                    cc[k] = 0;
                    vv[k] = VT(0);
                }
            }
#pragma unroll
            for (int k = 0; k < H; k++)
                if (h0 + k < w) {
                    x(cc[k], xv);
#pragma unroll
                    for (int t = 0; t < NT; t++) acc[t] += (double)vv[k] * xv[t];
                }
        }
        for (int k = WMAX; k < w; k++) {
            const int e = off + k * kSlice + lane;
            x(sc(e, row), xv);
            const double vk = (double)ld_val(sv + e);
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t] += vk * xv[t];
        }
        if (act) epi(row, acc, pv);
    }
    }
}

struct NoPre {
    __device__ __forceinline__ int operator()(int) const { return 0; }
};

struct Two {
    double a, b;
};
struct Three {
    double a, b, c;
};

struct AllRows {
    __device__ __forceinline__ bool operator()(int) const { return true; }
};

// projection on [lo, hi]; NaN maps to lo (for lo = 0 the result is +0.0)
__device__ __forceinline__ double proj_box(double x, Box B)
{
    const double y = x > B.lo ? x : B.lo;
    return y < B.hi ? y : B.hi;
}

// Launch KERNEL (a template over WM, the unrolled slice width; may be a
// parenthesised template-id) with the instance that covers the widest slice
// `wmax`; kBlock threads per block on ctx->stream.
// A launch on the context's stream; while a CG-class profiling entry waits
// for its kernel, the kernel's own begin and end are recorded into the
// entry's events (hipExtLaunchKernelGGL) rather than markers around it.
#define NN_LAUNCH_ROWS(KERNEL, grid, ...)                                                    \
    do {                                                                                     \
        hipEvent_t ka_ = nullptr, kb_ = nullptr;                                             \
        if (ctx->prof_attach && prof_kernel_events(ctx, &ka_, &kb_))                         \
            hipExtLaunchKernelGGL(KERNEL, dim3(grid), dim3(kBlock), 0, ctx->stream, ka_, kb_, \
                                  0, __VA_ARGS__);                                           \
        else                                                                                 \
            hipLaunchKernelGGL(KERNEL, dim3(grid), dim3(kBlock), 0, ctx->stream, __VA_ARGS__); \
    } while (0)

#define NN_DISPATCH_W(wmax, KERNEL, grid, ...)                                             \
    do {                                                                                   \
        if ((wmax) <= 8) {                                                                 \
            constexpr int WM = 8;                                                          \
            NN_LAUNCH_ROWS(KERNEL, grid, __VA_ARGS__);                                     \
        } else if ((wmax) <= 16) {                                                         \
            constexpr int WM = 16;                                                         \
            NN_LAUNCH_ROWS(KERNEL, grid, __VA_ARGS__);                                     \
        } else {                                                                           \
            constexpr int WM = 32;                                                         \
            NN_LAUNCH_ROWS(KERNEL, grid, __VA_ARGS__);                                     \
        }                                                                                  \
    } while (0)

}  // namespace nnqp
