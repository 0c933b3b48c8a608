// P1 assembly of the stiffness matrix K, capacity matrix M and load F.
//
// Host: validation and the symbolic phase (free-DOF numbering, node-to-element
// incidence, CSR pattern of the free rows), split over host threads.
// Device: a row-gather numeric phase.  One thread owns one free row i and
// walks the elements incident to its node in increasing element order; for
// each it forms the P1 gradients and adds the row's element entries
//     K^e_ab = |e| grad phi_a . D_e grad phi_b,
//     M^e_ab = |e| (1 + delta_ab) / ((d+1)(d+2)),   F^e_a = |e| f_e / (d+1)
// (bilinear form B and functional L of Sec. 2.1.2; capacity matrix of
// Sec. 2.2.2) into the row's own slots.  No two threads write the same slot,
// so no atomics are needed and the result is reproducible; the stiffness
// entry is evaluated with a form symmetric in (a, b), so K is bitwise
// symmetric.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "nnqp_internal.hpp"

namespace nnqp {

namespace {

template <class F>
void parallel_for(int64_t n, F &&fn)
{
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 32) nt = 32;
    if (n < 4096) nt = 1;
    if (nt == 1) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    int64_t per = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; t++) {
        int64_t a = (int64_t)t * per, b = std::min<int64_t>(n, a + per);
        if (a >= b) break;
        th.emplace_back([&, a, b, t] { fn(a, b, (int)t); });
    }
    for (auto &x : th) x.join();
}

// A scratch device buffer of one call, taken from and returned to the
// context's allocator.
struct DevBuf {
    const nnqp::DevAlloc &al;
    void *p = nullptr;
    explicit DevBuf(const nnqp::DevAlloc &a) : al(a) {}
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { nnqp::dev_free(al, p); }
};

}  // namespace

// ---------------------------------------------------------------- device side
struct AsmArgs {
    int dim;
    int nfree;
    const int *free_node;   // [nfree] node id of each free row
    const int64_t *inc_ptr; // [n_nodes + 1]
    const int *inc_elem;    // incident elements, ascending per node
    const int *elems;       // [ne * (dim+1)]
    const double *coords;   // [nn * dim]
    const double *D;        // [nD * dim * dim]
    int per_elem_D;
    const double *kscale;   // [ne] or null
    const double *f;        // [ne]
    const double *dval;     // [nn] Dirichlet values or null (homogeneous)
    const int *dof;         // [nn]
    const int *rowptr;
    const int *col;
    double *val;
    double *mval;           // or null
    double *F;
};

// K^e_ab without contraction and in an order symmetric in (a, b).
__device__ __forceinline__ double stiff_entry(int dim, const double *Dm, const double *ga,
                                             const double *gb)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int k = 0; k < dim; k++) s += Dm[k * dim + k] * (ga[k] * gb[k]);
    for (int k = 0; k < dim; k++)
        for (int l = k + 1; l < dim; l++) s += Dm[k * dim + l] * (ga[k] * gb[l] + ga[l] * gb[k]);
    return s;
}

__global__ __launch_bounds__(kBlock) void k_assemble(AsmArgs A)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= A.nfree) return;
    const int dim = A.dim, nv = dim + 1;
    const int node = A.free_node[row];
    const int s0 = A.rowptr[row], s1 = A.rowptr[row + 1];
    double Frow = 0.0;
    for (int64_t t = A.inc_ptr[node]; t < A.inc_ptr[node + 1]; t++) {
        const int e = A.inc_elem[t];
        int vid[4];
        double x[4][3];
        for (int a = 0; a < nv; a++) {
            vid[a] = A.elems[(int64_t)e * nv + a];
            for (int k = 0; k < dim; k++) x[a][k] = A.coords[(int64_t)vid[a] * dim + k];
        }
        // gradients of the barycentric functions from the edge vectors e_k = x_k - x_0
        double gr[4][3];
        double vol;
        if (dim == 2) {
            const double e1x = x[1][0] - x[0][0], e1y = x[1][1] - x[0][1];
            const double e2x = x[2][0] - x[0][0], e2y = x[2][1] - x[0][1];
            const double det = e1x * e2y - e1y * e2x;
            gr[1][0] = e2y / det;
            gr[1][1] = -e2x / det;
            gr[2][0] = -e1y / det;
            gr[2][1] = e1x / det;
            gr[0][0] = -(gr[1][0] + gr[2][0]);
            gr[0][1] = -(gr[1][1] + gr[2][1]);
            vol = fabs(det) * 0.5;
        } else {
            double ev[3][3];
            for (int a = 0; a < 3; a++)
                for (int k = 0; k < 3; k++) ev[a][k] = x[a + 1][k] - x[0][k];
            // cross products e2 x e3, e3 x e1, e1 x e2
            double cr[3][3];
            for (int a = 0; a < 3; a++) {
                const double *u = ev[(a + 1) % 3], *w = ev[(a + 2) % 3];
                cr[a][0] = u[1] * w[2] - u[2] * w[1];
                cr[a][1] = u[2] * w[0] - u[0] * w[2];
                cr[a][2] = u[0] * w[1] - u[1] * w[0];
            }
            const double det = ev[0][0] * cr[0][0] + ev[0][1] * cr[0][1] + ev[0][2] * cr[0][2];
            for (int k = 0; k < 3; k++) {
                gr[1][k] = cr[0][k] / det;
                gr[2][k] = cr[1][k] / det;
                gr[3][k] = cr[2][k] / det;
                gr[0][k] = -(gr[1][k] + gr[2][k] + gr[3][k]);
            }
            vol = fabs(det) / 6.0;
        }
        double Dm[9];
        const double *Ds = A.D + (A.per_elem_D ? (int64_t)e * dim * dim : 0);
        const double ks = A.kscale ? A.kscale[e] : 1.0;
        for (int k = 0; k < dim * dim; k++) Dm[k] = ks * Ds[k];
        int la = 0;
        for (int a = 0; a < nv; a++)
            if (vid[a] == node) la = a;
        Frow += vol * A.f[e] / (double)nv;
        const double mdiag = vol * 2.0 / (double)(nv * (nv + 1));
        const double moff = vol / (double)(nv * (nv + 1));
        for (int b = 0; b < nv; b++) {
            const int j = A.dof[vid[b]];
            if (j < 0) {
                // Dirichlet neighbour: its prescribed value moves to the load
                if (A.dval) Frow -= vol * stiff_entry(dim, Dm, gr[la], gr[b]) * A.dval[vid[b]];
                continue;
            }
            int slot = s0;
            while (slot < s1 && A.col[slot] != j) slot++;
            if (slot >= s1) continue;   // cannot happen: the pattern holds every element pair
            const double kab = vol * stiff_entry(dim, Dm, gr[la], gr[b]);
            A.val[slot] += kab;
            if (A.mval) A.mval[slot] += (b == la) ? mdiag : moff;
        }
    }
    A.F[row] = Frow;
}

// ---------------------------------------------------------------- host side
void sell_offsets(const int64_t *rowptr, int64_t n, std::vector<int64_t> &off, int &wmax)
{
    const int64_t ns = (n + kSlice - 1) / kSlice;
    off.assign(ns + 1, 0);
    wmax = 0;
    for (int64_t s = 0; s < ns; s++) {
        int w = 0;
        for (int64_t i = s * kSlice; i < std::min<int64_t>(n, (s + 1) * kSlice); i++)
            w = std::max<int>(w, (int)(rowptr[i + 1] - rowptr[i]));
        off[s + 1] = off[s] + (int64_t)w * kSlice;
        wmax = std::max(wmax, w);
    }
}

nn_status sell_build(nn_ctx *ctx, nn_matrix *A, const int64_t *rowptr_host, const double *csr_val,
                     const double *csr_mval)
{
    std::vector<int64_t> off;
    int wmax = 0;
    sell_offsets(rowptr_host, A->n, off, wmax);
    const int64_t ns = (int64_t)off.size() - 1;
    const int64_t nsell = off.back();
    if (nsell >= ((int64_t)1 << 31)) return fail(ctx, NN_EINVAL, "sliced-ELL size exceeds 32-bit offsets");
    A->nslices = ns;
    A->nsell = nsell;
    A->wmax = wmax;
    std::vector<int> off32(off.begin(), off.end());
    const size_t ne = (size_t)std::max<int64_t>(nsell, 1);
    hipError_t e = dev_malloc(A->al, &A->sl_off, sizeof(int) * (ns + 1));
    if (e == hipSuccess) e = dev_malloc(A->al, &A->sl_col, sizeof(int) * ne);
    if (e == hipSuccess) e = dev_malloc(A->al, &A->val, sizeof(double) * ne);
    if (e == hipSuccess && csr_mval) e = dev_malloc(A->al, &A->mval, sizeof(double) * ne);
    if (e != hipSuccess) return fail(ctx, NN_EOOM, "sliced-ELL allocation failed");
    NN_HIP_TRY(ctx, hipMemcpyAsync(A->sl_off, off32.data(), sizeof(int) * (ns + 1),
                                   hipMemcpyHostToDevice, ctx->stream));
    if (A->n > 0) launch_csr_to_sell(ctx, A, csr_val, csr_mval);
    NN_HIP_TRY(ctx, hipGetLastError());
    NN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return NN_OK;
}

nn_status finish_matrix(nn_ctx *ctx, nn_matrix *A)
{
    if (A->n > 0) {
        // int16 column offsets for the float32-value passes, kept only when
        // every |col - row| fits
        short *sd = nullptr;
        if (dev_malloc(A->al, &sd, sizeof(short) * std::max<int64_t>(A->nsell, 1)) != hipSuccess)
            return fail(ctx, NN_EOOM, "int16 offset allocation failed");
        launch_sell_d16(ctx, A, sd);
        static const int kMaxOp[1] = {OP_MAX};
        double span = 0.0;
        nn_status rc = host_reduce(ctx, A->n, 1, kMaxOp, &span);
        if (rc != NN_OK) {
            dev_free(A->al, sd);
            return rc;
        }
        if (span <= 32767.0) A->sl_d16 = sd;
        else dev_free(A->al, sd);
        if (dev_malloc(A->al, &A->diag, sizeof(double) * A->n) != hipSuccess)
            return fail(ctx, NN_EOOM, "diagonal allocation failed");
        launch_diag(ctx, A, A->val, A->diag);
        std::vector<double> d(A->n);
        NN_HIP_TRY(ctx, hipMemcpyAsync(d.data(), A->diag, sizeof(double) * A->n,
                                       hipMemcpyDeviceToHost, ctx->stream));
        NN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        for (int64_t i = 0; i < A->n; i++) {
            if (!std::isfinite(d[i])) return fail(ctx, NN_ENONFINITE, "non-finite diagonal entry");
            if (!(d[i] > 0.0))
                return fail(ctx, NN_ENOTSPD, "non-positive diagonal entry at row " + std::to_string(i));
        }
    }
    return NN_OK;
}

nn_status assemble_impl(nn_ctx *ctx, const nn_mesh *mesh, const double *D, int64_t nD,
                        const double *kscale, const double *f_elem, const uint8_t *dirichlet,
                        const double *dvals, int with_mass, nn_matrix **K_out, double *F_dev,
                        int64_t *dof_of_node)
{
    if (!mesh || !K_out || !D || !f_elem || !dirichlet)
        return fail(ctx, NN_EINVAL, "null argument to nn_assemble");
    const int dim = mesh->dim;
    if (dim != 2 && dim != 3) return fail(ctx, NN_EINVAL, "mesh dim must be 2 or 3");
    const int64_t nn = mesh->n_nodes, ne = mesh->n_elems;
    if (nn < 0 || ne < 0 || (nn > 0 && !mesh->coords) || (ne > 0 && !mesh->elems))
        return fail(ctx, NN_EINVAL, "bad mesh sizes or arrays");
    if (nn >= (int64_t)1 << 31 || ne >= (int64_t)1 << 31)
        return fail(ctx, NN_EINVAL, "mesh too large for 32-bit indices");
    if (nD != 1 && nD != ne) return fail(ctx, NN_EINVAL, "nD must be 1 or n_elems");
    const int nv = dim + 1;

    // ---- validation
    for (int64_t t = 0; t < ne * nv; t++) {
        const int v = mesh->elems[t];
        if (v < 0 || v >= nn) return fail(ctx, NN_EINVAL, "element node id out of range");
    }
    for (int64_t t = 0; t < nn * dim; t++)
        if (!std::isfinite(mesh->coords[t])) return fail(ctx, NN_ENONFINITE, "non-finite coordinate");
    for (int64_t t = 0; t < nD * dim * dim; t++)
        if (!std::isfinite(D[t])) return fail(ctx, NN_ENONFINITE, "non-finite diffusivity");
    for (int64_t e = 0; e < ne; e++) {
        if (!std::isfinite(f_elem[e])) return fail(ctx, NN_ENONFINITE, "non-finite source");
        if (kscale && !(std::isfinite(kscale[e]) && kscale[e] > 0.0))
            return fail(ctx, NN_ENONFINITE, "kscale must be finite and positive");
    }
    if (dvals)
        for (int64_t v = 0; v < nn; v++)
            if (dirichlet[v] && !std::isfinite(dvals[v]))
                return fail(ctx, NN_ENONFINITE, "non-finite Dirichlet value");

    // ---- free-DOF numbering
    std::vector<int> dof(nn);
    std::vector<int> free_node;
    free_node.reserve(nn);
    for (int64_t v = 0; v < nn; v++) {
        if (dirichlet[v]) {
            dof[v] = -1;
        } else {
            dof[v] = (int)free_node.size();
            free_node.push_back((int)v);
        }
    }
    const int64_t n = (int64_t)free_node.size();
    if (dof_of_node)
        for (int64_t v = 0; v < nn; v++) dof_of_node[v] = dof[v];

    // ---- node -> element incidence (elements ascending per node)
    std::vector<int64_t> inc_ptr(nn + 1, 0);
    for (int64_t t = 0; t < ne * nv; t++) inc_ptr[mesh->elems[t] + 1]++;
    for (int64_t v = 0; v < nn; v++) inc_ptr[v + 1] += inc_ptr[v];
    std::vector<int> inc_elem(std::max<int64_t>(inc_ptr[nn], 1));
    {
        std::vector<int64_t> pos(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t e = 0; e < ne; e++)
            for (int a = 0; a < nv; a++) inc_elem[pos[mesh->elems[e * nv + a]]++] = (int)e;
    }

    // ---- CSR pattern of the free rows
    std::vector<int> rowlen(n);
    auto row_cols = [&](int node, std::vector<int> &buf) {
        buf.clear();
        for (int64_t t = inc_ptr[node]; t < inc_ptr[node + 1]; t++) {
            const int e = inc_elem[t];
            for (int b = 0; b < nv; b++) {
                const int j = dof[mesh->elems[(int64_t)e * nv + b]];
                if (j >= 0) buf.push_back(j);
            }
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    parallel_for(n, [&](int64_t a, int64_t b, int) {
        std::vector<int> buf;
        for (int64_t r = a; r < b; r++) {
            row_cols(free_node[r], buf);
            rowlen[r] = (int)buf.size();
        }
    });
    std::vector<int64_t> rp64(n + 1, 0);
    for (int64_t r = 0; r < n; r++) rp64[r + 1] = rp64[r] + rowlen[r];
    const int64_t nnz = rp64[n];
    if (nnz >= ((int64_t)1 << 31)) return fail(ctx, NN_EINVAL, "nnz exceeds 32-bit row pointers");
    std::vector<int> rowptr(n + 1), col(std::max<int64_t>(nnz, 1));
    for (int64_t r = 0; r <= n; r++) rowptr[r] = (int)rp64[r];
    parallel_for(n, [&](int64_t a, int64_t b, int) {
        std::vector<int> buf;
        for (int64_t r = a; r < b; r++) {
            row_cols(free_node[r], buf);
            std::copy(buf.begin(), buf.end(), col.begin() + rowptr[r]);
        }
    });

    // ---- device numeric phase
    nn_matrix *M = new (std::nothrow) nn_matrix();
    if (!M) return fail(ctx, NN_EOOM, "host allocation");
    M->al = ctx->al;
    M->n = n;
    M->nnz = nnz;
    auto cleanup = [&](nn_status st) {
        nn_matrix_free(ctx, M);
        return st;
    };
    const DevAlloc &ta = ctx->al;   // scratch of this call
    DevBuf d_free(ta), d_incp(ta), d_ince(ta), d_elems(ta), d_coords(ta), d_D(ta), d_ks(ta),
        d_f(ta), d_dv(ta), d_dof(ta), d_F(ta), d_val(ta), d_mval(ta);
    auto up = [&](DevBuf &b, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = dev_malloc(ta, &b.p, bytes > 0 ? bytes : 8);
        if (e != hipSuccess) return e;
        if (src && bytes > 0) e = hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, ctx->stream);
        return e;
    };
#define NN_UP(buf, src, bytes)                                                              \
    do {                                                                                    \
        hipError_t e_ = up(buf, src, bytes);                                                \
        if (e_ != hipSuccess) {                                                             \
            fail(ctx, e_ == hipErrorOutOfMemory ? NN_EOOM : NN_EHIP,                        \
                 std::string("assembly upload: ") + hipGetErrorString(e_));                 \
            return cleanup(e_ == hipErrorOutOfMemory ? NN_EOOM : NN_EHIP);                  \
        }                                                                                   \
    } while (0)
    NN_UP(d_free, free_node.data(), sizeof(int) * n);
    NN_UP(d_incp, inc_ptr.data(), sizeof(int64_t) * (nn + 1));
    NN_UP(d_ince, inc_elem.data(), sizeof(int) * inc_elem.size());
    NN_UP(d_elems, mesh->elems, sizeof(int) * ne * nv);
    NN_UP(d_coords, mesh->coords, sizeof(double) * nn * dim);
    NN_UP(d_D, D, sizeof(double) * nD * dim * dim);
    if (kscale) NN_UP(d_ks, kscale, sizeof(double) * ne);
    NN_UP(d_f, f_elem, sizeof(double) * ne);
    if (dvals) NN_UP(d_dv, dvals, sizeof(double) * nn);
    NN_UP(d_dof, dof.data(), sizeof(int) * nn);
    {
        hipError_t e = dev_malloc(M->al, &M->rowptr, sizeof(int) * (n + 1));
        if (e == hipSuccess) e = dev_malloc(M->al, &M->col, sizeof(int) * std::max<int64_t>(nnz, 1));
        if (e == hipSuccess) e = dev_malloc(ta, &d_val.p, sizeof(double) * std::max<int64_t>(nnz, 1));
        if (e == hipSuccess && with_mass)
            e = dev_malloc(ta, &d_mval.p, sizeof(double) * std::max<int64_t>(nnz, 1));
        if (e == hipSuccess && !F_dev) e = dev_malloc(ta, &d_F.p, sizeof(double) * std::max<int64_t>(n, 1));
        if (e != hipSuccess) {
            fail(ctx, NN_EOOM, std::string("matrix allocation: ") + hipGetErrorString(e));
            return cleanup(NN_EOOM);
        }
    }
    NN_HIP_TRY(ctx, hipMemcpyAsync(M->rowptr, rowptr.data(), sizeof(int) * (n + 1),
                                   hipMemcpyHostToDevice, ctx->stream));
    if (nnz > 0) {
        NN_HIP_TRY(ctx, hipMemcpyAsync(M->col, col.data(), sizeof(int) * nnz, hipMemcpyHostToDevice,
                                       ctx->stream));
        NN_HIP_TRY(ctx, hipMemsetAsync(d_val.p, 0, sizeof(double) * nnz, ctx->stream));
        if (d_mval.p) NN_HIP_TRY(ctx, hipMemsetAsync(d_mval.p, 0, sizeof(double) * nnz, ctx->stream));
    }
    AsmArgs args;
    args.dim = dim;
    args.nfree = (int)n;
    args.free_node = (const int *)d_free.p;
    args.inc_ptr = (const int64_t *)d_incp.p;
    args.inc_elem = (const int *)d_ince.p;
    args.elems = (const int *)d_elems.p;
    args.coords = (const double *)d_coords.p;
    args.D = (const double *)d_D.p;
    args.per_elem_D = nD == 1 ? 0 : 1;
    args.kscale = (const double *)d_ks.p;
    args.f = (const double *)d_f.p;
    args.dval = (const double *)d_dv.p;
    args.dof = (const int *)d_dof.p;
    args.rowptr = M->rowptr;
    args.col = M->col;
    args.val = (double *)d_val.p;
    args.mval = (double *)d_mval.p;
    args.F = F_dev ? F_dev : (double *)d_F.p;
    if (n > 0) {
        const int64_t nb = (n + kBlock - 1) / kBlock;
        k_assemble<<<(unsigned)nb, kBlock, 0, ctx->stream>>>(args);
        NN_HIP_TRY(ctx, hipGetLastError());
    }
    NN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    nn_status st = sell_build(ctx, M, rp64.data(), (const double *)d_val.p, (const double *)d_mval.p);
    if (st == NN_OK) st = finish_matrix(ctx, M);
    if (st != NN_OK) return cleanup(st);
    int mr = 0;
    for (int64_t r = 0; r < n; r++) mr = std::max(mr, rowlen[r]);
    M->max_row = mr;
    *K_out = M;
    return NN_OK;
#undef NN_UP
}

}  // namespace nnqp
