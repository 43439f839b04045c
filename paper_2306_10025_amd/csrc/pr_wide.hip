// Host side of the patches above 32 dofs (kernels in k_wide.hip): Algorithm 1
// in rounds of one entry each.
#include <algorithm>
#include <cstring>

#include "pr_internal.h"

// Algorithm 1 (Section 3.1) for handles with a patch above 32 dofs.  Round
// m: the lowest open patch opens entry m (no earlier entry matched it, and
// every entry so far was opened by a lower patch), then every other open
// patch of its size is compared with entry m; the matched ones are mapped to
// it and close.  A patch therefore meets the entries in creation order and
// closes at the first within eps, the sequential algorithm's result and
// comparison count (evaluations plus pruned pairs).  The spectral criterion
// needs the entry's inverse during its round; the entrywise ones invert all
// entries in one batch at the end.
int run_alg1_wide(pr_handle h) {
    hipStream_t s = h->stream;
    const int64_t n_p = h->n_p;
    const int crit = h->prm.criterion;
    const bool spectral = crit == PR_CRIT_SPECTRAL;
    const int pm = h->max_ps;
    const int64_t stride = (int64_t)pm * pm;
    const int ups = h->uniform ? pm : 0;
    const int64_t* toff = h->uniform ? nullptr : h->toff;
    int32_t *U = nullptr, *Un = nullptr, *info = nullptr;
    int64_t *keep = nullptr, *excl = nullptr, *scr = nullptr;
    unsigned long long* counters = nullptr;
    PR_TRY(dalloc(h, &U, n_p));
    PR_TRY(dalloc(h, &Un, n_p));
    PR_TRY(dalloc(h, &keep, n_p + 1));
    PR_TRY(dalloc(h, &excl, n_p + 1));
    PR_TRY(dalloc(h, &scr, scan_scratch_elems(n_p + 1) + 2));
    PR_TRY(dalloc(h, &counters, 4));
    PR_TRY(dalloc(h, &info, n_p));
    PR_TRY(dalloc(h, &h->phi, n_p));
    PR_HIP(h, hipMemsetAsync(counters, 0, 4 * sizeof(unsigned long long), s));
    PR_HIP(h, hipMemsetAsync(info, 0, n_p * sizeof(int32_t), s));
    launch_iota(U, n_p, s);
    double* dbcap = nullptr;          // spectral: inverses of the entries so far
    int64_t cap = 0;
    double* scratch = nullptr;
    int64_t grid = 1;
    if (spectral) {
        cap = std::min<int64_t>(n_p, 64);
        PR_TRY(dalloc(h, &dbcap, (size_t)cap * stride));
        grid = a1w_spectral_grid(n_p - 1);
        PR_TRY(dalloc(h, &scratch, (size_t)grid * 2 * stride));
    }
    std::vector<int32_t> reps;
    int64_t nU = n_p;
    int32_t first = 0;
    while (nU > 0) {
        const int32_t m = (int32_t)reps.size();
        reps.push_back(first);
        const double* Xm = nullptr;
        if (spectral) {
            if (m >= cap) {
                const int64_t ncap = std::min<int64_t>(n_p, 2 * cap);
                double* nb = nullptr;
                PR_TRY(dalloc(h, &nb, (size_t)ncap * stride));
                PR_HIP(h, hipMemcpyAsync(nb, dbcap, (size_t)m * stride * sizeof(double), hipMemcpyDeviceToDevice, s));
                PR_HIP(h, hipStreamSynchronize(s));
                dfree(h, dbcap);
                dbcap = nb;
                cap = ncap;
            }
            launch_gj_wide(1, U, h->pptr, h->tiles, toff, ups, pm, dbcap + (int64_t)m * stride, nullptr, info + m, s);
            Xm = dbcap + (int64_t)m * stride;
        }
        const int64_t nu = nU - 1;
        launch_a1w_round(nu, U, m, crit, h->prm.eps, h->pptr, h->tiles, toff, ups, h->fnorm, h->l1norm, Xm,
                         scratch, spectral ? std::min<int64_t>(grid, a1w_spectral_grid(nu)) : 0, pm, h->phi,
                         keep, counters, s);
        int64_t nn = 0;
        if (nu > 0) {
            launch_exclusive_scan_i64(keep, excl, nu + 1, scr, s);
            launch_a1w_compact(nu, U + 1, keep, excl, Un, s);
            PR_HIP(h, hipMemcpyAsync(&nn, excl + nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            PR_HIP(h, hipMemcpyAsync(&first, Un, sizeof(int32_t), hipMemcpyDeviceToHost, s));  // used when nn > 0
            PR_HIP(h, hipStreamSynchronize(s));
        }
        std::swap(U, Un);
        nU = nn;
    }
    PR_HIP(h, hipGetLastError());
    const int64_t m_p = (int64_t)reps.size();
    h->m_p = m_p;
    h->reps_host = reps;
    PR_TRY(dalloc(h, &h->reps, m_p));
    PR_HIP(h, hipMemcpyAsync(h->reps, reps.data(), m_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    std::vector<int64_t> pptr_host(n_p + 1);
    PR_HIP(h, hipMemcpyAsync(pptr_host.data(), h->pptr, (n_p + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    h->dbps_host.resize(m_p);
    h->dboff_host.resize(m_p + 1);
    for (int64_t j = 0; j < m_p; ++j) {
        h->dbps_host[j] = (int32_t)(pptr_host[reps[j] + 1] - pptr_host[reps[j]]);
        h->dboff_host[j] = j * stride;
    }
    h->dboff_host[m_p] = m_p * stride;
    if (spectral) {
        h->db = dbcap;                    // entries at j * stride (capacity beyond m_p unused)
    } else {
        int64_t* xoff = nullptr;
        PR_TRY(dalloc(h, &h->db, (size_t)m_p * stride));
        PR_TRY(dalloc(h, &xoff, m_p + 1));
        PR_HIP(h, hipMemcpyAsync(xoff, h->dboff_host.data(), (m_p + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        launch_gj_wide(m_p, h->reps, h->pptr, h->tiles, toff, ups, pm, h->db, xoff, info, s);
    }
    std::vector<int32_t> info_h(m_p);
    unsigned long long c4[4];
    PR_HIP(h, hipMemcpyAsync(info_h.data(), info, m_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipMemcpyAsync(c4, counters, sizeof(c4), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    PR_HIP(h, hipGetLastError());
    for (int64_t j = 0; j < m_p; ++j)
        if (info_h[j] != 0)
            return pr_fail(h, PR_ERR_SINGULAR_PATCH, "zero pivot in database patch " + std::to_string(reps[j]));
    h->stats.crit_evals = (int64_t)c4[0];
    h->stats.crit_pruned = (int64_t)c4[1];
    h->stats.crit_refined = (int64_t)c4[2];
    h->stats.crit_exact = (int64_t)c4[3];
    h->stats.alg1_rounds = m_p;
    return PR_OK;
}
