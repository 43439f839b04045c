// Host side of the two-level combination preconditioner (Eq.(2)):
// pr_set_coarse forms R0 = P0^T and A0 = R0 A P0 on the device and factors
// A0 (explicit inverse, or block LU over the band); coarse_add applies
// z += P0 A0^{-1} R0 r inside the preconditioner application.
#include "pr_internal.h"

#include <algorithm>
#include <chrono>

namespace {

double wall_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

bool dev_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

constexpr int64_t kDenseMax = 4096;   // n0 up to which A0 is inverted whole
constexpr int kBandMax = 4096;        // largest block of the banded solve (its vector sits in LDS)
constexpr double kDrop = 1e-13;

int64_t round32(int64_t v) { return (v + 31) / 32 * 32; }

}  // namespace

int coarse_add(pr_handle h, const double* r, double* z, const int32_t* stop) {
    if (h->n0 <= 0) return PR_OK;
    hipStream_t s = h->stream;
    launch_csr_rows_wave(h->n0, h->r0_rp, h->r0_ci, h->r0_v, r, h->c_r0, stop, s);
    if (h->c_dense)
        launch_dense_gemv(h->c_np, h->c_X, h->c_r0, h->c_x, stop, s);
    else
        launch_band_solve(h->c_s, h->c_nb, h->c_X, h->c_G, h->c_H, h->c_r0, h->c_u, h->c_w, h->c_x, stop, s);
    launch_csr_rows_add(h->n, h->p0_rp, h->p0_ci, h->p0_v, h->c_x, z, stop, s);
    return PR_OK;
}

int pr_set_coarse(pr_handle h, const pr_interp* P) {
    if (!h || !P) return pr_fail(h, PR_ERR_INVALID_ARG, "null argument");
    if (h->n0 > 0) return pr_fail(h, PR_ERR_INVALID_ARG, "the handle already has a coarse space");
    if (h->nsys > 0) return pr_fail(h, PR_ERR_INVALID_ARG, "no coarse space for a batch of systems");
    if (P->n_fine != h->n || P->n_coarse < 1 || P->n_coarse > INT32_MAX - 1 || P->nnz < 0)
        return pr_fail(h, PR_ERR_INVALID_ARG, "P0 must have n rows and 1 <= n_coarse < 2^31 columns");
    if (!dev_ptr(P->row_ptr) || (P->nnz > 0 && (!dev_ptr(P->col) || !dev_ptr(P->val))))
        return pr_fail(h, P->row_ptr ? PR_ERR_HOST_POINTER : PR_ERR_INVALID_ARG, "P0 arrays must be device memory");
    const double t0 = wall_s();
    hipStream_t s = h->stream;
    const int64_t n = h->n, n0 = P->n_coarse, nnz = P->nnz;

    // copy and check P0
    int64_t* p0_rp = nullptr;
    int32_t* p0_ci = nullptr;
    double* p0_v = nullptr;
    int32_t* flags = nullptr;
    PR_TRY(dalloc(h, &p0_rp, n + 1));
    PR_TRY(dalloc(h, &p0_ci, nnz));
    PR_TRY(dalloc(h, &p0_v, nnz));
    PR_TRY(dalloc(h, &flags, 4));
    PR_HIP(h, hipMemcpyAsync(p0_rp, P->row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (nnz > 0) {
        PR_HIP(h, hipMemcpyAsync(p0_ci, P->col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        PR_HIP(h, hipMemcpyAsync(p0_v, P->val, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    PR_HIP(h, hipMemsetAsync(flags, 0, 4 * sizeof(int32_t), s));
    launch_interp_check(n, n0, nnz, p0_rp, p0_ci, p0_v, flags, s);
    int32_t fl[4];
    PR_HIP(h, hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    if (fl[0]) return pr_fail(h, PR_ERR_INVALID_ARG, "P0.row_ptr is not monotone from 0 to nnz");
    if (fl[1]) return pr_fail(h, PR_ERR_INVALID_ARG, "a P0 column lies outside [0, n_coarse)");
    if (fl[2]) return pr_fail(h, PR_ERR_NONFINITE, "non-finite P0 value");

    // R0 = P0^T
    int64_t *r0_rp = nullptr, *cnt = nullptr, *fill = nullptr, *scr = nullptr;
    int32_t* r0_ci = nullptr;
    double* r0_v = nullptr;
    const int64_t big = std::max(n, n0) + 1;
    PR_TRY(dalloc(h, &r0_rp, n0 + 1));
    PR_TRY(dalloc(h, &r0_ci, nnz));
    PR_TRY(dalloc(h, &r0_v, nnz));
    PR_TRY(dalloc(h, &cnt, big));
    PR_TRY(dalloc(h, &fill, big));
    PR_TRY(dalloc(h, &scr, scan_scratch_elems(big) + 2));
    {
        int32_t* uc = nullptr;
        double* uv = nullptr;
        PR_TRY(dalloc(h, &uc, nnz));
        PR_TRY(dalloc(h, &uv, nnz));
        if (launch_csr_transpose(n, n0, p0_rp, p0_ci, p0_v, r0_rp, r0_ci, r0_v, cnt, fill, uc, uv, scr, s) != 0)
            return pr_fail(h, PR_ERR_HIP, "transpose of P0");
        PR_HIP(h, hipStreamSynchronize(s));
        dfree(h, uc);
        dfree(h, uv);
    }

    // A0 = R0 (A P0): B = A P0 one fine row per wavefront into padded rows,
    // then one coarse row per wavefront into padded rows, then CSR.  When a
    // row of B reaches more coarse columns than its padding holds, the
    // triple product runs in one kernel instead (R0, A and P0 walked per
    // coarse row).
    const int slots = coarse_gal_slots();
    int32_t *ocnt = nullptr, *ocol = nullptr, *over = nullptr;
    double* oval = nullptr;
    PR_TRY(dalloc(h, &ocnt, n0));
    PR_TRY(dalloc(h, &ocol, (size_t)n0 * slots));
    PR_TRY(dalloc(h, &oval, (size_t)n0 * slots));
    PR_TRY(dalloc(h, &over, 1));
    {
        const int bs = coarse_ap_slots();
        int32_t *bcnt = nullptr, *bcol = nullptr;
        double* bval = nullptr;
        PR_TRY(dalloc(h, &bcnt, n));
        PR_TRY(dalloc(h, &bcol, (size_t)n * bs));
        PR_TRY(dalloc(h, &bval, (size_t)n * bs));
        PR_HIP(h, hipMemsetAsync(over, 0, sizeof(int32_t), s));
        launch_ap(n, h->rowptr, h->col, h->val, p0_rp, p0_ci, p0_v, bcnt, bcol, bval, over, s);
        int32_t ap_over = 0;
        PR_HIP(h, hipMemcpyAsync(&ap_over, over, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        if (!ap_over) {
            launch_rb(n0, r0_rp, r0_ci, r0_v, bcnt, bcol, bval, kDrop, ocnt, ocol, oval, over, s);
        } else {
            PR_HIP(h, hipMemsetAsync(over, 0, sizeof(int32_t), s));
            launch_galerkin(n0, r0_rp, r0_ci, r0_v, h->rowptr, h->col, h->val, p0_rp, p0_ci, p0_v, kDrop, ocnt,
                            ocol, oval, over, s);
        }
        PR_HIP(h, hipStreamSynchronize(s));
        dfree(h, bcnt);
        dfree(h, bcol);
        dfree(h, bval);
    }
    int64_t* a0_rp = nullptr;
    PR_TRY(dalloc(h, &a0_rp, n0 + 1));
    launch_rows_finish(n0, ocnt, cnt, a0_rp, scr, s);
    int64_t a0_nnz = 0;
    int32_t ov = 0;
    PR_HIP(h, hipMemcpyAsync(&a0_nnz, a0_rp + n0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipMemcpyAsync(&ov, over, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    if (ov) return pr_fail(h, PR_ERR_UNSUPPORTED, "a coarse row couples to more than 256 coarse unknowns");
    int32_t* a0_ci = nullptr;
    double* a0_v = nullptr;
    PR_TRY(dalloc(h, &a0_ci, a0_nnz));
    PR_TRY(dalloc(h, &a0_v, a0_nnz));
    launch_rows_compact(n0, a0_rp, ocol, oval, a0_ci, a0_v, s);
    PR_HIP(h, hipStreamSynchronize(s));
    dfree(h, ocol);
    dfree(h, oval);

    // bandwidth and the transpose of A0 (its columns, for the Schur updates)
    int32_t* dbw = nullptr;
    PR_TRY(dalloc(h, &dbw, 1));
    PR_HIP(h, hipMemsetAsync(dbw, 0, sizeof(int32_t), s));
    launch_bandwidth(n0, a0_rp, a0_ci, dbw, s);
    int32_t bw = 0;
    PR_HIP(h, hipMemcpyAsync(&bw, dbw, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));

    int32_t* info = nullptr;
    double *pinv = nullptr, *cbuf = nullptr;
    PR_TRY(dalloc(h, &info, 1));
    PR_HIP(h, hipMemsetAsync(info, 0, sizeof(int32_t), s));
    PR_TRY(dalloc(h, &pinv, 1024));
    int dense = n0 <= kDenseMax ? 1 : 0;
    int64_t np = 0, len = 0;
    int sb = 0, nbk = 0;
    double *X = nullptr, *G = nullptr, *H = nullptr;
    int64_t *a0t_rp = nullptr;
    int32_t* a0t_ci = nullptr;
    double* a0t_v = nullptr;
    if (!dense) {
        sb = (int)round32(std::max<int64_t>(bw, 1));
        if (sb > kBandMax)
            return pr_fail(h, PR_ERR_UNSUPPORTED, "coarse bandwidth " + std::to_string(bw) + " beyond 4096");
        nbk = (int)((n0 + sb - 1) / sb);
        if (nbk == 1) dense = 1;
    }
    if (dense) {
        np = round32(n0);
        len = np;
        PR_TRY(dalloc(h, &X, (size_t)np * np));
        PR_TRY(dalloc(h, &cbuf, (size_t)np * 32));
        launch_dense_from_csr(n0, np, a0_rp, a0_ci, a0_v, X, s);
        launch_gj_inverse(X, (int)np, pinv, cbuf, info, s);
    } else {
        len = (int64_t)nbk * sb;
        PR_TRY(dalloc(h, &a0t_rp, n0 + 1));
        PR_TRY(dalloc(h, &a0t_ci, a0_nnz));
        PR_TRY(dalloc(h, &a0t_v, a0_nnz));
        int32_t* uc = nullptr;
        double* uv = nullptr;
        PR_TRY(dalloc(h, &uc, a0_nnz));
        PR_TRY(dalloc(h, &uv, a0_nnz));
        if (launch_csr_transpose(n0, n0, a0_rp, a0_ci, a0_v, a0t_rp, a0t_ci, a0t_v, cnt, fill, uc, uv, scr, s) != 0)
            return pr_fail(h, PR_ERR_HIP, "transpose of A0");
        PR_HIP(h, hipStreamSynchronize(s));
        dfree(h, uc);
        dfree(h, uv);
        const size_t blk = (size_t)sb * sb;
        PR_TRY(dalloc(h, &X, blk * nbk));
        PR_TRY(dalloc(h, &G, blk * nbk));
        PR_TRY(dalloc(h, &H, blk * nbk));
        PR_TRY(dalloc(h, &cbuf, (size_t)sb * 32));
        // S_i = D_i - L_i H_{i-1}, inverted in place; G_i = S_i^{-1} L_i,
        // H_i = S_i^{-1} U_i
        for (int i = 0; i < nbk; ++i) {
            double* Si = X + blk * i;
            launch_block_schur_h(n0, sb, i, a0_rp, a0_ci, a0_v, i > 0 ? H + blk * (i - 1) : nullptr, Si, s);
            launch_gj_inverse(Si, sb, pinv, cbuf, info, s);
            if (i > 0) launch_block_coupling(n0, sb, i, i - 1, a0t_rp, a0t_ci, a0t_v, Si, G + blk * i, s);
            if (i < nbk - 1) launch_block_coupling(n0, sb, i, i + 1, a0t_rp, a0t_ci, a0t_v, Si, H + blk * i, s);
        }
        PR_HIP(h, hipStreamSynchronize(s));
    }
    int32_t bad = 0;
    PR_HIP(h, hipMemcpyAsync(&bad, info, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    PR_HIP(h, hipGetLastError());
    if (bad) return pr_fail(h, PR_ERR_SINGULAR_PATCH, "zero pivot in the coarse factorisation");
    dfree(h, cbuf);

    double *cr0 = nullptr, *cu = nullptr, *cw = nullptr, *cx = nullptr;
    PR_TRY(dalloc(h, &cr0, len));
    PR_TRY(dalloc(h, &cu, len));
    PR_TRY(dalloc(h, &cw, len));
    PR_TRY(dalloc(h, &cx, len));
    // the padding of the coarse vectors stays zero (kernels write rows < n0
    // of cr0 only; the solves write every row of cw and cx)
    PR_HIP(h, hipMemsetAsync(cr0, 0, len * sizeof(double), s));
    PR_HIP(h, hipMemsetAsync(cx, 0, len * sizeof(double), s));
    PR_HIP(h, hipStreamSynchronize(s));

    if (h->gexec) {                   // a captured cycle has no coarse term
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
        h->graph_m = -1;
    }
    h->n0 = n0;
    h->a0_nnz = a0_nnz;
    h->p0_rp = p0_rp; h->p0_ci = p0_ci; h->p0_v = p0_v;
    h->r0_rp = r0_rp; h->r0_ci = r0_ci; h->r0_v = r0_v;
    h->a0_rp = a0_rp; h->a0_ci = a0_ci; h->a0_v = a0_v;
    h->a0t_rp = a0t_rp; h->a0t_ci = a0t_ci; h->a0t_v = a0t_v;
    h->c_dense = dense;
    h->c_np = np;
    h->c_s = sb;
    h->c_nb = dense ? 1 : nbk;
    h->c_X = X;
    h->c_G = G;
    h->c_H = H;
    h->c_r0 = cr0;
    h->c_u = cu;
    h->c_w = cw;
    h->c_x = cx;
    h->stats.n_coarse = n0;
    h->stats.coarse_nnz = a0_nnz;
    h->stats.coarse_bandwidth = bw;
    h->stats.coarse_block = dense ? 0 : sb;
    h->stats.coarse_blocks = dense ? 1 : nbk;
    h->stats.t_coarse = wall_s() - t0;
    return PR_OK;
}

int pr_get_coarse_matrix(pr_handle h, int64_t* n0, int64_t* nnz, int64_t* row_ptr, int32_t* col, double* val) {
    if (!h || h->n0 <= 0) return pr_fail(h, PR_ERR_INVALID_ARG, "no coarse space in this handle");
    if (n0) *n0 = h->n0;
    if (nnz) *nnz = h->a0_nnz;
    if (row_ptr || col || val) {
        PR_HIP(h, hipStreamSynchronize(h->stream));
        if (row_ptr) PR_HIP(h, hipMemcpy(row_ptr, h->a0_rp, (h->n0 + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
        if (col) PR_HIP(h, hipMemcpy(col, h->a0_ci, h->a0_nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (val) PR_HIP(h, hipMemcpy(val, h->a0_v, h->a0_nnz * sizeof(double), hipMemcpyDeviceToHost));
    }
    return PR_OK;
}
