// C ABI of libpatchrelax.so: handle lifecycle, setup orchestration
// (Section 2 objects, database construction of Section 3, factorisation,
// grouping), the preconditioner apply of Eq.(3) and the right-preconditioned
// GMRES solve used in Section 4.
#include "pr_internal.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <unordered_map>

namespace {

std::mutex g_mu;
std::string g_last_error;

// database handed from pr_setup_reuse to the setup it runs (this thread only)
struct ReuseSeed {
    std::vector<int32_t> phi, reps;
};
thread_local const ReuseSeed* g_reuse_pending = nullptr;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}


bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

int check_dev(pr_handle h, const void* p, const char* what) {
    if (!p) return pr_fail(h, PR_ERR_INVALID_ARG, std::string(what) + " is null");
    if (!is_device_ptr(p)) return pr_fail(h, PR_ERR_HOST_POINTER, std::string(what) + " is not device memory");
    return PR_OK;
}


// ---- Algorithm 1 ------------------------------------------------------------
int run_alg1(pr_handle h) {
    hipStream_t s = h->stream;
    const int64_t n_p = h->n_p;
    const int64_t stride = (int64_t)h->max_ps * h->max_ps;
    A1Run R;
    PR_TRY(alg1_core(h, nullptr, n_p, R));
    h->m_p = R.m;
    // entries numbered by ascending patch id
    PR_TRY(dalloc(h, &h->phi, n_p));
    PR_TRY(dalloc(h, &h->reps, n_p));
    PR_TRY(dalloc(h, &h->db, (size_t)h->m_p * stride));
    launch_a1_finish(n_p, R.repof, R.flag, R.excl, R.scr, h->phi, h->reps, s);
    launch_a1_copy_db(h->m_p, h->reps, R.slot_of_patch, h->pptr, R.dbt, h->db, stride, s);
    h->reps_host.resize(h->m_p);
    PR_HIP(h, hipMemcpyAsync(h->reps_host.data(), h->reps, h->m_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    // sizes of the entries' patches
    std::vector<int32_t> rsz(h->m_p, h->max_ps);
    int32_t* dsz = nullptr;
    PR_TRY(dalloc(h, &dsz, h->m_p));
    if (!h->uniform) {
        launch_rep_sizes(h->reps, h->pptr, h->m_p, dsz, s);
        PR_HIP(h, hipMemcpyAsync(rsz.data(), dsz, h->m_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    PR_HIP(h, hipStreamSynchronize(s));
    h->stats.crit_evals = (int64_t)R.cnt[0];
    h->stats.crit_exact = (int64_t)R.cnt[1];
    h->stats.crit_refined = (int64_t)R.cnt[3];
    h->stats.alg1_rounds = R.rounds;
    // pairs the sequential algorithm compares: patch i against the entries of
    // its size up to its own (excluded for an entry's patch); the rest were
    // skipped by the certified bound.  The per-patch sum runs on the device.
    {
        std::vector<int32_t> before(h->m_p);       // earlier entries of the same size
        std::vector<int32_t> seen(33, 0);
        for (int64_t j = 0; j < h->m_p; ++j) before[j] = seen[rsz[j]]++;
        int32_t* dbefore = nullptr;
        unsigned long long* dnaive = nullptr;
        PR_TRY(dalloc(h, &dbefore, h->m_p));
        PR_TRY(dalloc(h, &dnaive, 1));
        PR_HIP(h, hipMemcpyAsync(dbefore, before.data(), h->m_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PR_HIP(h, hipMemsetAsync(dnaive, 0, sizeof(unsigned long long), s));
        launch_naive_pairs(h->phi, h->reps, dbefore, n_p, h->m_p, dnaive, s);
        unsigned long long naive = 0;
        PR_HIP(h, hipMemcpyAsync(&naive, dnaive, sizeof(naive), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        h->stats.crit_pruned = (int64_t)naive - h->stats.crit_evals;
    }
    if (h->prm.alg1_match == 1) {
        // closest matching over the same database; R.excl holds, for every
        // patch, the number of entries with a lower patch id
        const int crit = h->prm.criterion;
        const double* keynorm = (crit == PR_CRIT_L1) ? h->l1norm : h->fnorm;
        const int64_t grid = std::min<int64_t>(n_p, 2048);
        double* ekey = nullptr;
        int32_t* esz = nullptr;
        double* lbscr = nullptr;
        int32_t* phi0 = nullptr;
        unsigned long long* cc = nullptr;
        PR_TRY(dalloc(h, &ekey, h->m_p));
        PR_TRY(dalloc(h, &esz, h->m_p));
        PR_TRY(dalloc(h, &lbscr, (size_t)grid * h->m_p));
        PR_TRY(dalloc(h, &phi0, n_p));
        PR_TRY(dalloc(h, &cc, 5));
        PR_HIP(h, hipMemsetAsync(cc, 0, 5 * sizeof(unsigned long long), s));
        PR_HIP(h, hipMemcpyAsync(phi0, h->phi, n_p * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        launch_a1_closest(n_p, h->pptr, h->tiles, h->uniform ? nullptr : h->toff, h->uniform ? h->max_ps : 0,
                          h->reps, h->m_p, R.excl, keynorm, ekey, esz, h->db, stride, crit, h->prm.eps,
                          h->prm.tie_rel, h->phi, lbscr, grid, cc, s);
        launch_count_eq(n_p, h->phi, 1, phi0, cc + 4, s);
        unsigned long long c5[5];
        PR_HIP(h, hipMemcpyAsync(c5, cc, sizeof(c5), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        h->stats.closest_evals = (int64_t)c5[0];
        h->stats.crit_exact += (int64_t)c5[1];
        h->stats.crit_refined += (int64_t)c5[3];
        h->stats.closest_moved = n_p - (int64_t)c5[4];
    }
    h->dbps_host.resize(h->m_p);
    h->dboff_host.resize(h->m_p + 1);
    for (int64_t j = 0; j < h->m_p; ++j) {
        h->dbps_host[j] = rsz[j];
        h->dboff_host[j] = j * stride;
    }
    h->dboff_host[h->m_p] = h->m_p * stride;
    return PR_OK;
}

// ---- FULL path: every patch is its own entry -------------------------------
int run_full(pr_handle h) {
    hipStream_t s = h->stream;
    const int64_t n_p = h->n_p;
    PR_TRY(dalloc(h, &h->phi, n_p));
    PR_TRY(dalloc(h, &h->reps, n_p));
    PR_TRY(dalloc(h, &h->db, h->total_tile));
    launch_iota(h->phi, n_p, s);
    launch_iota(h->reps, n_p, s);
    int32_t* info = nullptr;
    PR_TRY(dalloc(h, &info, n_p));
    if (h->wide)
        launch_gj_wide(n_p, nullptr, h->pptr, h->tiles, h->uniform ? nullptr : h->toff, h->uniform ? h->max_ps : 0,
                       h->max_ps, h->db, h->uniform ? nullptr : h->toff, info, s);
    else
        launch_batch_inverse(h->max_ps, n_p, h->tiles, h->uniform ? nullptr : h->toff, nullptr,
                             h->uniform ? nullptr : h->pptr, h->db, h->uniform ? nullptr : h->toff, info, s);
    std::vector<int32_t> info_h(n_p);
    PR_HIP(h, hipMemcpyAsync(info_h.data(), info, n_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    for (int64_t k = 0; k < n_p; ++k)
        if (info_h[k] != 0)
            return pr_fail(h, PR_ERR_SINGULAR_PATCH, "zero pivot in patch " + std::to_string(k));
    h->m_p = n_p;
    h->reps_host.resize(n_p);
    for (int64_t k = 0; k < n_p; ++k) h->reps_host[k] = (int32_t)k;
    std::vector<int64_t> pptr_host(n_p + 1);
    PR_HIP(h, hipMemcpy(pptr_host.data(), h->pptr, (n_p + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    h->dbps_host.resize(n_p);
    h->dboff_host.resize(n_p + 1);
    int64_t off = 0;
    for (int64_t k = 0; k < n_p; ++k) {
        const int p = (int)(pptr_host[k + 1] - pptr_host[k]);
        h->dbps_host[k] = p;
        h->dboff_host[k] = off;
        off += (int64_t)p * p;
    }
    h->dboff_host[n_p] = off;
    h->stats.crit_evals = 0;
    return PR_OK;
}

// ---- Algorithm 2 and its variants (Section 3.2) ----------------------------

// SplitMix64 (Steele, Lea and Flood, 2014): the state advances by the golden
// gamma, the output is two xor-shift-multiply rounds and a final xor-shift.
uint64_t splitmix64_next(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Clusters per group in proportion to the group sizes: floor shares, the
// remaining seats to the largest remainders (lower group on ties), then every
// empty group takes one seat from the fullest group (lower group on ties).
bool apportion_clusters(const std::vector<int64_t>& sizes, int64_t m_total, std::vector<int64_t>& out) {
    const int64_t N = std::accumulate(sizes.begin(), sizes.end(), (int64_t)0);
    const int64_t G = (int64_t)sizes.size();
    if (m_total < G || m_total > N) return false;
    out.assign(G, 0);
    std::vector<int64_t> rem(G);
    int64_t used = 0;
    for (int64_t g = 0; g < G; ++g) {
        const __int128 prod = (__int128)m_total * sizes[g];
        out[g] = (int64_t)(prod / N);
        rem[g] = (int64_t)(prod % N);
        used += out[g];
    }
    std::vector<int64_t> ord(G);
    std::iota(ord.begin(), ord.end(), (int64_t)0);
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return rem[a] > rem[b]; });
    for (int64_t t = 0; t < m_total - used; ++t) out[ord[t]] += 1;
    for (;;) {
        int64_t g0 = -1;
        for (int64_t g = 0; g < G && g0 < 0; ++g)
            if (out[g] == 0) g0 = g;
        if (g0 < 0) break;
        int64_t donor = 0;
        for (int64_t g = 1; g < G; ++g)
            if (out[g] > out[donor]) donor = g;
        out[donor] -= 1;
        out[g0] += 1;
    }
    return true;
}

int run_kmeans(pr_handle h) {
    hipStream_t s = h->stream;
    const int64_t n_p = h->n_p;
    const int algo = h->prm.algo;
    const bool boot = algo == PR_ALGO_BOOTSTRAP;
    const int64_t stride = (int64_t)h->max_ps * h->max_ps;
    const int crit = (algo == PR_ALGO_KMEANS_ENTRYWISE) ? PR_CRIT_L1 : PR_CRIT_SPECTRAL;
    const int medoid = (algo == PR_ALGO_VARMIN || boot) ? 1 : 0;
    const double tie = h->prm.tie_rel;
    const int max_iter = h->prm.kmeans_max_iter;
    const int ups = h->uniform ? h->max_ps : 0;
    const int64_t* toff = h->uniform ? nullptr : h->toff;

    std::vector<int32_t> boot_reps, boot_ps;
    int64_t boot_evals = 0, boot_exact = 0, boot_pruned = 0, boot_refined = 0;
    if (boot) {
        // initial database from Algorithm 1
        PR_TRY(run_alg1(h));
        boot_reps = h->reps_host;
        boot_ps = h->dbps_host;
        boot_evals = h->stats.crit_evals;
        boot_exact = h->stats.crit_exact;
        boot_refined = h->stats.crit_refined;
        boot_pruned = h->stats.crit_pruned;
    }

    // 1. groups: (size, boundary key), or size alone; members in ascending id
    const int partition = (!boot && h->prm.partition_bc) ? 1 : 0;
    const int64_t N = next_pow2(n_p);
    uint64_t *keys = nullptr, *kscr = nullptr;
    int32_t *vals = nullptr, *vscr = nullptr, *pg = nullptr, *gp = nullptr;
    int64_t *flag = nullptr, *excl = nullptr, *scr = nullptr, *gstart = nullptr;
    PR_TRY(dalloc(h, &keys, n_p));
    PR_TRY(dalloc(h, &kscr, N));
    PR_TRY(dalloc(h, &vals, n_p));
    PR_TRY(dalloc(h, &vscr, N));
    PR_TRY(dalloc(h, &flag, n_p + 1));
    PR_TRY(dalloc(h, &excl, n_p + 1));
    PR_TRY(dalloc(h, &scr, scan_scratch_elems(n_p + 1) + 2));
    PR_TRY(dalloc(h, &pg, n_p));
    PR_TRY(dalloc(h, &gstart, n_p + 1));
    PR_TRY(dalloc(h, &gp, n_p));
    launch_km_key1(n_p, h->pptr, h->keys, partition, keys, vals, s);
    launch_sort_pairs(keys, vals, n_p, kscr, vscr, s);
    launch_km_flags(n_p, keys, flag, s);
    launch_exclusive_scan_i64(flag, excl, n_p + 1, scr, s);
    launch_km_gid(n_p, keys, vals, flag, excl, pg, gstart, gp, s);
    int64_t G = 0;
    PR_HIP(h, hipMemcpyAsync(&G, excl + n_p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    std::vector<int64_t> gstart_h(G + 1);
    std::vector<int32_t> gp_h(G);
    PR_HIP(h, hipMemcpyAsync(gstart_h.data(), gstart, (G + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipMemcpyAsync(gp_h.data(), gp, G * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    launch_km_key2(n_p, pg, keys, vals, s);
    launch_sort_pairs(keys, vals, n_p, kscr, vscr, s);   // vals: members by (group, id)
    PR_HIP(h, hipStreamSynchronize(s));

    // 2. initial centres
    std::vector<int64_t> m_per(G, 0);
    std::vector<int32_t> rep0_h;          // boot: patch ids; else sorted positions (gathered below)
    std::vector<int64_t> pos_h;
    if (boot) {
        for (int64_t g = 0; g < G; ++g)
            for (size_t j = 0; j < boot_reps.size(); ++j)
                if (boot_ps[j] == gp_h[g]) {
                    rep0_h.push_back(boot_reps[j]);
                    m_per[g] += 1;
                }
    } else {
        std::vector<int64_t> sizes(G);
        for (int64_t g = 0; g < G; ++g) sizes[g] = gstart_h[g + 1] - gstart_h[g];
        if (!apportion_clusters(sizes, h->prm.m_target, m_per))
            return pr_fail(h, PR_ERR_INVALID_ARG,
                           "m_target must lie between the number of groups (" + std::to_string(G) +
                               ") and the number of patches");
        if (h->has_reuse && (int64_t)h->reuse_reps.size() != h->prm.m_target)
            return pr_fail(h, PR_ERR_INVALID_ARG, "the blob's database size differs from m_target");
        // partial Fisher-Yates draw per group, groups in order, one stream:
        // position i swaps with i + (u mod (L - i))
        uint64_t st = h->prm.seed;
        for (int64_t g = 0; g < G && !h->has_reuse; ++g) {
            const int64_t L = sizes[g];
            std::unordered_map<int64_t, int64_t> moved;
            auto at = [&](int64_t x) {
                auto it = moved.find(x);
                return it == moved.end() ? x : it->second;
            };
            for (int64_t i = 0; i < m_per[g]; ++i) {
                const uint64_t u = splitmix64_next(st);
                const int64_t j = i + (int64_t)(u % (uint64_t)(L - i));
                const int64_t vi = at(i), vj = at(j);
                moved[i] = vj;
                moved[j] = vi;
                pos_h.push_back(gstart_h[g] + vj);
            }
        }
    }
    const int64_t m_p = std::accumulate(m_per.begin(), m_per.end(), (int64_t)0);
    if (m_p <= 0) return pr_fail(h, PR_ERR_INVALID_ARG, "empty database");
    std::vector<int32_t> cgroup_h(m_p), cps_h(m_p), gc0_h(G), gc1_h(G);
    int64_t lbld = 0;
    {
        int64_t j = 0;
        for (int64_t g = 0; g < G; ++g) {
            gc0_h[g] = (int32_t)j;
            for (int64_t t = 0; t < m_per[g]; ++t, ++j) {
                cgroup_h[j] = (int32_t)g;
                cps_h[j] = gp_h[g];
            }
            gc1_h[g] = (int32_t)j;
            lbld = std::max(lbld, m_per[g]);
        }
    }
    int32_t *rep = nullptr, *cgroup = nullptr, *cps = nullptr, *gc0 = nullptr, *gc1 = nullptr;
    int32_t *gactive = nullptr, *gupd = nullptr, *gchanged = nullptr, *info = nullptr, *phi = nullptr;
    int32_t* mem = nullptr;
    int64_t *cptr = nullptr, *coff = nullptr, *csz = nullptr;
    unsigned long long *counters = nullptr, *ccount = nullptr;
    double *B = nullptr, *X = nullptr, *lbscr = nullptr;
    PR_TRY(dalloc(h, &rep, m_p));
    PR_TRY(dalloc(h, &cgroup, m_p));
    PR_TRY(dalloc(h, &cps, m_p));
    PR_TRY(dalloc(h, &gc0, G));
    PR_TRY(dalloc(h, &gc1, G));
    PR_TRY(dalloc(h, &gactive, G));
    PR_TRY(dalloc(h, &gupd, G));
    PR_TRY(dalloc(h, &gchanged, G));
    PR_TRY(dalloc(h, &info, m_p));
    PR_TRY(dalloc(h, &phi, n_p));
    PR_TRY(dalloc(h, &mem, n_p));
    PR_TRY(dalloc(h, &cptr, m_p + 1));
    PR_TRY(dalloc(h, &ccount, m_p + 1));
    PR_TRY(dalloc(h, &counters, 4));
    PR_TRY(dalloc(h, &B, (size_t)m_p * stride));
    PR_TRY(dalloc(h, &X, (size_t)m_p * stride));
    std::vector<int32_t> warm_rep;
    if (h->has_reuse) {
        // warm start: every previous centre j lies in group cgroup[j]; its
        // lowest member seeds B_j until the update below replaces it
        std::vector<int32_t> pg_h(n_p);
        PR_HIP(h, hipMemcpy(pg_h.data(), pg, n_p * sizeof(int32_t), hipMemcpyDeviceToHost));
        warm_rep.assign(m_p, -1);
        for (int64_t i = 0; i < n_p; ++i) {
            const int32_t j = h->reuse_phi[i];
            if (cgroup_h[j] != pg_h[i])
                return pr_fail(h, PR_ERR_INVALID_ARG, "the blob's assignment leaves a patch's group");
            if (warm_rep[j] < 0) warm_rep[j] = (int32_t)i;
        }
        for (int64_t j = 0; j < m_p; ++j)
            if (warm_rep[j] < 0)
                return pr_fail(h, PR_ERR_INVALID_ARG, "the blob leaves a centre without members");
    }
    if (boot) {
        PR_HIP(h, hipMemcpyAsync(rep, rep0_h.data(), m_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    } else if (h->has_reuse) {
        PR_HIP(h, hipMemcpyAsync(rep, warm_rep.data(), m_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    } else {
        int64_t* pos = nullptr;
        PR_TRY(dalloc(h, &pos, m_p));
        PR_HIP(h, hipMemcpyAsync(pos, pos_h.data(), m_p * sizeof(int64_t), hipMemcpyHostToDevice, s));
        launch_gather_i32(m_p, vals, pos, rep, s);
    }
    PR_HIP(h, hipMemcpyAsync(cgroup, cgroup_h.data(), m_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PR_HIP(h, hipMemcpyAsync(cps, cps_h.data(), m_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PR_HIP(h, hipMemcpyAsync(gc0, gc0_h.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PR_HIP(h, hipMemcpyAsync(gc1, gc1_h.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!h->uniform) {
        // centre j: size cps[j], stored at j * stride
        std::vector<int64_t> csz_h(m_p + 1), coff_h(m_p + 1);
        csz_h[0] = 0;
        for (int64_t j = 0; j < m_p; ++j) {
            csz_h[j + 1] = csz_h[j] + cps_h[j];
            coff_h[j] = j * stride;
        }
        coff_h[m_p] = m_p * stride;
        PR_TRY(dalloc(h, &csz, m_p + 1));
        PR_TRY(dalloc(h, &coff, m_p + 1));
        PR_HIP(h, hipMemcpyAsync(csz, csz_h.data(), (m_p + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        PR_HIP(h, hipMemcpyAsync(coff, coff_h.data(), (m_p + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    }
    launch_km_init(m_p, rep, h->pptr, h->tiles, toff, ups, B, stride, s);
    launch_fill_i32(phi, n_p, -1, s);
    if (h->has_reuse) {
        // centres start as the update of the previous assignment
        PR_HIP(h, hipMemcpyAsync(phi, h->reuse_phi.data(), n_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
        std::vector<int32_t> all(G, 1);
        PR_HIP(h, hipMemcpyAsync(gupd, all.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PR_HIP(h, hipMemsetAsync(ccount, 0, (m_p + 1) * sizeof(unsigned long long), s));
        launch_km_keys(n_p, phi, pg, gupd, keys, mem, ccount, s);
        launch_sort_pairs(keys, mem, n_p, kscr, vscr, s);
        launch_exclusive_scan_i64((const int64_t*)ccount, cptr, m_p + 1, scr, s);
        launch_km_update(m_p, cgroup, gupd, cptr, mem, cps, medoid, h->tiles, toff, ups, B, stride, rep, tie,
                         counters, s);
        PR_HIP(h, hipStreamSynchronize(s));
    }
    PR_HIP(h, hipMemsetAsync(counters, 0, 4 * sizeof(unsigned long long), s));
    const int64_t grid = km_assign_grid(n_p, lbld);
    PR_TRY(dalloc(h, &lbscr, (size_t)grid * lbld));

    auto invert = [&](double* dst) -> int {
        launch_batch_inverse(h->max_ps, m_p, B, coff, nullptr, csz, dst, coff, info, s);
        std::vector<int32_t> info_h(m_p);
        PR_HIP(h, hipMemcpyAsync(info_h.data(), info, m_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        for (int64_t j = 0; j < m_p; ++j)
            if (info_h[j] != 0)
                return pr_fail(h, PR_ERR_SINGULAR_PATCH, "singular cluster centre " + std::to_string(j));
        return PR_OK;
    };

    // 3. assignment / update passes, each group until no assignment changes
    std::vector<int32_t> act(G, 1), upd(G, 0), changed(G, 0);
    std::vector<int64_t> its(G, 0);
    for (;;) {
        for (int64_t g = 0; g < G; ++g)
            if (act[g]) its[g] += 1;
        if (crit == PR_CRIT_SPECTRAL) PR_TRY(invert(X));
        PR_HIP(h, hipMemcpyAsync(gactive, act.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PR_HIP(h, hipMemsetAsync(gchanged, 0, G * sizeof(int32_t), s));
        launch_km_assign(grid, n_p, h->pptr, h->tiles, toff, ups, pg, gc0, gc1, gactive, crit, h->l1norm,
                         crit == PR_CRIT_SPECTRAL ? X : B, stride, tie, phi, gchanged, lbscr, lbld, counters, s);
        PR_HIP(h, hipMemcpyAsync(changed.data(), gchanged, G * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        PR_HIP(h, hipGetLastError());
        bool any = false;
        for (int64_t g = 0; g < G; ++g) {
            upd[g] = 0;
            if (!act[g]) continue;
            if (changed[g] == 0 || its[g] >= max_iter) continue;   // converged, or out of passes
            upd[g] = 1;
            any = true;
        }
        if (!any) break;
        PR_HIP(h, hipMemcpyAsync(gupd, upd.data(), G * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PR_HIP(h, hipMemsetAsync(ccount, 0, (m_p + 1) * sizeof(unsigned long long), s));
        launch_km_keys(n_p, phi, pg, gupd, keys, mem, ccount, s);
        launch_sort_pairs(keys, mem, n_p, kscr, vscr, s);
        launch_exclusive_scan_i64((const int64_t*)ccount, cptr, m_p + 1, scr, s);
        launch_km_update(m_p, cgroup, gupd, cptr, mem, cps, medoid, h->tiles, toff, ups, B, stride, rep, tie,
                         counters, s);
        act = upd;
    }

    // 4. the database: inverses of the final centres
    PR_TRY(dalloc(h, &h->db, (size_t)m_p * stride));
    PR_TRY(invert(h->db));
    unsigned long long cnt[4];
    PR_HIP(h, hipMemcpyAsync(cnt, counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
    h->m_p = m_p;
    h->phi = phi;
    h->reps = rep;
    h->db_mat = B;
    h->reps_host.resize(m_p);
    PR_HIP(h, hipMemcpyAsync(h->reps_host.data(), rep, m_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    h->stats.crit_evals = (int64_t)cnt[0] + boot_evals;
    h->stats.crit_exact = (int64_t)cnt[1] + boot_exact;
    h->stats.crit_refined = (int64_t)cnt[3] + boot_refined;
    h->stats.crit_pruned = boot_pruned;
    h->stats.empty_events = (int64_t)cnt[2];
    h->stats.kmeans_iters = (int32_t)*std::max_element(its.begin(), its.end());
    h->dbps_host = cps_h;
    h->dboff_host.resize(m_p + 1);
    for (int64_t j = 0; j <= m_p; ++j) h->dboff_host[j] = j * stride;
    return PR_OK;
}

// ---- grouping and precision conversion -------------------------------------
int run_group(pr_handle h) {
    hipStream_t s = h->stream;
    const int64_t n_p = h->n_p, m_p = h->m_p;
    // order = patches sorted by (entry, id)
    uint64_t* keys = nullptr;
    uint64_t* kscr = nullptr;
    int32_t* vscr = nullptr;
    const int64_t N = next_pow2(n_p);
    PR_TRY(dalloc(h, &keys, n_p));
    PR_TRY(dalloc(h, &kscr, N));
    PR_TRY(dalloc(h, &vscr, N));
    PR_TRY(dalloc(h, &h->order, n_p));
    int32_t* gbad = nullptr;
    int32_t* estart = nullptr;
    PR_TRY(dalloc(h, &gbad, 1));
    PR_TRY(dalloc(h, &estart, m_p + 1));
    PR_HIP(h, hipMemsetAsync(gbad, 0, sizeof(int32_t), s));
    launch_group_keys(h->phi, n_p, m_p, keys, h->order, gbad, s);
    launch_sort_pairs(keys, h->order, n_p, kscr, vscr, s);
    // grouped copy of the dof lists and the entry of each grouped position
    PR_TRY(dalloc(h, &h->gdofs, h->total_dofs));
    PR_TRY(dalloc(h, &h->gphi, n_p));
    if (!h->uniform) {
        int64_t* sizes = nullptr;
        int64_t* scr = nullptr;
        PR_TRY(dalloc(h, &sizes, n_p + 1));
        PR_TRY(dalloc(h, &scr, scan_scratch_elems(n_p + 1) + 2));
        PR_TRY(dalloc(h, &h->goff, n_p + 1));
        launch_group_sizes(h->order, n_p, h->pptr, sizes, s);
        launch_exclusive_scan_i64(sizes, h->goff, n_p + 1, scr, s);
    }
    launch_group_gather(h->order, n_p, h->pptr, h->pdofs, h->goff, h->uniform ? h->max_ps : 0, h->gdofs,
                        h->gphi, h->phi, s);
    // entry sizes for the work items: first grouped position of each entry
    std::vector<int64_t> count(m_p, 0);
    {
        PR_HIP(h, hipMemsetAsync(estart, 0xFF, (m_p + 1) * sizeof(int32_t), s));   // -1: no patch
        launch_entry_starts(h->gphi, n_p, m_p, estart, s);
        std::vector<int32_t> st(m_p + 1);
        int32_t bad = 0;
        PR_HIP(h, hipMemcpyAsync(st.data(), estart, m_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipMemcpyAsync(&bad, gbad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        if (bad) return pr_fail(h, PR_ERR_INVALID_ARG, "internal: patch map out of range");
        st[m_p] = (int32_t)n_p;
        for (int64_t j = m_p - 1; j >= 0; --j)
            if (st[j] < 0) st[j] = st[j + 1];
        for (int64_t j = 0; j < m_p; ++j) count[j] = st[j + 1] - st[j];
    }
    if (h->prm.deterministic) {
        // dof -> grouped slots, ascending (fixed summation order)
        int64_t* cnt64 = nullptr;
        int64_t* scr = nullptr;
        int32_t* fill = nullptr;
        PR_TRY(dalloc(h, &cnt64, h->n + 1));
        PR_TRY(dalloc(h, &scr, scan_scratch_elems(h->n + 1) + 2));
        PR_TRY(dalloc(h, &fill, h->n));
        PR_TRY(dalloc(h, &h->dof_ptr, h->n + 1));
        PR_TRY(dalloc(h, &h->dof_slots, h->total_dofs));
        launch_i32_to_i64(h->cnt, cnt64, h->n, s);
        launch_exclusive_scan_i64(cnt64, h->dof_ptr, h->n + 1, scr, s);
        PR_HIP(h, hipMemsetAsync(fill, 0, h->n * sizeof(int32_t), s));
        // slots in tiles of 16 grouped patches, row-plane by row-plane (the
        // rows of neighbouring patches are contiguous)
        launch_transpose_fill(h->gdofs, h->goff, h->uniform ? h->max_ps : 0, n_p, h->max_ps, h->dof_ptr, fill,
                              h->dof_slots, s);
        launch_transpose_sort(h->n, h->dof_ptr, h->dof_slots, s);
        if (h->prm.apply_form != PR_FORM_GENERAL) {
            // padded table when no dof lies in more than 8 patches
            int32_t* cmax = nullptr;
            PR_TRY(dalloc(h, &cmax, 1));
            PR_HIP(h, hipMemsetAsync(cmax, 0, sizeof(int32_t), s));
            launch_max_i32(h->cnt, h->n, cmax, s);
            int32_t c = 0;
            PR_HIP(h, hipMemcpyAsync(&c, cmax, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            PR_HIP(h, hipStreamSynchronize(s));
            // the table is the faster form even where it is mostly padding
            // (high-order cells, most dofs in one patch and a few in eight:
            // Q5 12.8 against 19.3 us, Q2 8.0 against 9.4 us for the lists,
            // whose loads depend on each other)
            if (c >= 1 && c <= 8) {
                const int C = c <= 1 ? 1 : c <= 2 ? 2 : c <= 4 ? 4 : 8;
                PR_TRY(dalloc(h, &h->dof_ell, (size_t)h->n * C));
                launch_build_ell(h->n, h->dof_ptr, h->dof_slots, C, h->dof_ell, s);
                h->ell_c = C;
            }
        }
        const size_t ybytes = h->prm.apply_precision == PR_FP64 ? 8 : 4;
        char* yb = nullptr;
        PR_TRY(dalloc(h, &yb, (size_t)((n_p + 15) / 16) * 16 * h->max_ps * ybytes));
        h->Ybuf = yb;
    }
    // work items of <= 16 (p <= 16) or <= 32 members of one entry
    std::vector<int32_t> items;
    int64_t start = 0;
    for (int64_t j = 0; j < m_p; ++j) {
        const int p = h->dbps_host[j];
        // MFMA tile: 16x16x16 or 32x32x8; 16 members per item for every
        // entry of a handle with patches above 32 dofs (16 x 16 x 4 FP64)
        const int nb = (p <= 16 || h->wide) ? 16 : 32;
        for (int64_t t = 0; t < count[j]; t += nb) {
            items.push_back((int32_t)j);
            items.push_back((int32_t)(start + t));
            items.push_back((int32_t)std::min<int64_t>(nb, count[j] - t));
            items.push_back(p);
        }
        start += count[j];
    }
    h->n_items = (int64_t)items.size() / 4;
    // Every patch of one size: the MFMA apply can run over fixed tiles of 16
    // or 32 grouped patches instead of items. A tile straddles the entries
    // its members use, and each further entry costs it one more dependent
    // operand load. Measured (Nedelec 64^3, Q2 32^3 at four tolerances,
    // Taylor-Hood 64^2): 16-patch tiles won where the groups were long (1.02
    // items per tile: 23.3 against 31.1 us); 32-patch tiles lost to items at
    // every mix (1.04 to 8.8 items per tile), so the automatic choice takes
    // tiles for 16-patch tiles of long groups only.
    {
        const int64_t tile_nb = h->max_ps <= 16 ? 16 : 32;
        const int64_t n_tiles = (n_p + tile_nb - 1) / tile_nb;
        const bool can_tile = h->uniform && h->max_ps <= 32;
        const bool tiles = can_tile && (h->prm.apply_form == PR_FORM_TILES ||
                                        (h->prm.apply_form == PR_FORM_AUTO && h->max_ps <= 16 &&
                                         4 * h->n_items <= 5 * n_tiles));
        h->tile_p = tiles ? h->max_ps : 0;
    }
    PR_TRY(dalloc(h, &h->items, items.size()));
    PR_HIP(h, hipMemcpyAsync(h->items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    // database offsets / sizes on the device
    int32_t* dbps = nullptr;
    PR_TRY(dalloc(h, &dbps, m_p));
    PR_HIP(h, hipMemcpyAsync(dbps, h->dbps_host.data(), m_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PR_TRY(dalloc(h, &h->dboff, m_p + 1));
    PR_HIP(h, hipMemcpyAsync(h->dboff, h->dboff_host.data(), (m_p + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    const int64_t dbsize = h->dboff_host[m_p];
    const int prec = h->prm.apply_precision;
    h->apply_prec = prec;
    if (prec == PR_FP32) PR_TRY(dalloc(h, &h->db_f32, dbsize));
    int64_t lp_elems = 0;
    if (prec == PR_BF16 || prec == PR_FP16 || prec == PR_BF16X3) {
        const int64_t mult = prec == PR_BF16X3 ? 2 : 1;   // high and low parts
        std::vector<int64_t> off(m_p + 1);
        for (int64_t j = 0; j < m_p; ++j) {
            off[j] = lp_elems;
            lp_elems += mult * (h->dbps_host[j] <= 16 ? 256 : 1024);
        }
        off[m_p] = lp_elems;
        uint16_t* lp = nullptr;
        PR_TRY(dalloc(h, &lp, lp_elems));
        h->db_lp = lp;
        PR_TRY(dalloc(h, &h->dblp_off, m_p + 1));
        PR_HIP(h, hipMemcpyAsync(h->dblp_off, off.data(), (m_p + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        PR_TRY(dalloc(h, &h->db_exp, m_p));
    }
    if (h->wide) {
        // column-major copies for the wide apply; grouped matrix-core items
        // unless (almost) every patch is its own entry
        if (prec == PR_FP64) PR_TRY(dalloc(h, &h->db_t, dbsize));
        launch_transpose_db(m_p, h->db, h->dboff, dbps, h->db_t, h->db_f32, s);
        h->wide_form = (2 * m_p > n_p) ? 2 : 1;
    } else {
        launch_convert_db(prec, m_p, h->db, h->dboff, dbps, 0, (uint16_t*)h->db_lp, h->dblp_off, h->db_exp,
                          h->db_f32, s);
    }
    PR_HIP(h, hipStreamSynchronize(s));
    PR_HIP(h, hipGetLastError());
    h->stats.n_items = h->n_items;
    // the FP64 and FP32 applies run per row whatever the form
    h->stats.apply_tile_p = (prec == PR_BF16 || prec == PR_FP16 || prec == PR_BF16X3) ? h->tile_p : 0;
    h->stats.bytes_db = dbsize * 8;
    h->stats.bytes_db_lowp = prec == PR_FP32 ? dbsize * 4 : lp_elems * 2;
    h->stats.bytes_index = n_p * 4;
    return PR_OK;
}

// z = omega M~^{-1} r, or z += omega M~^{-1} r when accumulate (tmp: n doubles,
// used by the deterministic scatter, which overwrites its output)
int apply_op(pr_handle h, const double* r, double* z, bool accumulate, double* tmp,
             const int32_t* stop = nullptr) {
    hipStream_t s = h->stream;
    const bool two = h->prm.deterministic != 0;
    ApplyLaunch a{};
    a.stop = stop;
    a.n = h->n;
    a.n_p = h->n_p;
    a.gdofs = h->gdofs;
    a.goff = h->goff;
    a.pst = h->uniform ? h->max_ps : 0;
    a.gphi = h->gphi;
    a.maxp = h->max_ps;
    a.db = h->db;
    a.db_f32 = h->db_f32;
    a.dboff = h->dboff;
    a.dbst = 0;
    a.db_lp = (const uint16_t*)h->db_lp;
    a.dblp_off = h->dblp_off;
    a.db_exp = h->db_exp;
    a.items = h->items;
    a.n_items = h->n_items;
    a.W = h->W;
    a.omega = h->prm.omega;
    a.r = r;
    a.Y = h->Ybuf;
    a.dof_ptr = h->dof_ptr;
    a.dof_slots = h->dof_slots;
    a.ell = h->dof_ell;
    a.ell_c = h->ell_c;
    a.tile_p = h->tile_p;
    a.threads = h->tune_threads;
    a.grid_cap = h->tune_cap;
    a.tiles_per_wave = h->tune_tpw;
    a.xcd_remap = h->tune_remap;
    a.slot_threads = h->tune_slot;
    a.wide = h->wide ? h->wide_form : 0;
    a.db_t = h->db_t;
    if (two) {
        a.z = accumulate ? tmp : z;
        launch_apply(h->apply_prec, true, a, s);
        if (accumulate) launch_axpy_dev(z, tmp, 1.0, h->n, s);
    } else {
        if (!accumulate) launch_zero(z, h->n, s, stop);
        a.z = z;
        launch_apply(h->apply_prec, false, a, s);
    }
    return PR_OK;
}

// e = `sweeps` damped smoothing steps from 0 applied to v (t3: 2n doubles
// scratch), plus the coarse term P0 A0^{-1} R0 v of the two-level combination
// when the handle has a coarse space and `coarse` is set
int precond(pr_handle h, const double* v, double* e, double* t3, const int32_t* stop = nullptr,
            bool coarse = true) {
    hipStream_t s = h->stream;
    PR_TRY(apply_op(h, v, e, false, nullptr, stop));
    for (int sw = 1; sw < h->prm.sweeps; ++sw) {
        launch_spmv_sell(h->sell(), h->n, e, v, t3, s, stop);
        PR_TRY(apply_op(h, t3, e, true, t3 + h->n, stop));
    }
    if (coarse) PR_TRY(coarse_add(h, v, e, stop));
    return PR_OK;
}

int ensure_workspace(pr_handle h, int m) {
    if (h->ws_restart >= m) return PR_OK;
    const int64_t n = h->n;
    h->ldv = (n + 63) / 64 * 64;   // 512-byte aligned basis columns
    PR_TRY(dalloc(h, &h->V, (size_t)(m + 1) * h->ldv));
    // defined contents: rows of a masked system may be read before written
    PR_HIP(h, hipMemsetAsync(h->V, 0, (size_t)(m + 1) * h->ldv * sizeof(double), h->stream));
    PR_TRY(dalloc(h, &h->w, n));
    PR_TRY(dalloc(h, &h->t1, n));
    PR_TRY(dalloc(h, &h->t2, 3 * n));   // preconditioned vector, sweep residual, scratch
    PR_TRY(dalloc(h, &h->red, (size_t)gs_blocks(n) * 72 + 64));   // up to 33 + 33 partials per block
    PR_TRY(dalloc(h, &h->gm, 16384));
    PR_TRY(dalloc(h, &h->gctl, 4));
    PR_TRY(dalloc(h, &h->hd, 256));
    if (!h->hh) PR_HIP(h, pool_host_alloc(256 * sizeof(double), (void**)&h->hh, &h->hh_got));
    h->ws_restart = m;
    return PR_OK;
}

// Times launch shapes of the apply on this handle's data and keeps the
// fastest: threads per block and block cap of the patch kernel, then the
// threads per block of the slot sum.  Every shape computes the same result
// (deterministic mode: bit for bit; atomic mode: up to summation order).
//
// The choice depends only on the shape of the grouped apply, so it is kept
// per process, keyed on that shape, and a later setup of the same shape on
// the same device reuses it without timing.
using TuneKey = std::array<int64_t, 11>;

// tiles per wave of the default shape (0 when the fixed-tile kernel does not run)
inline int tpw_choice_default(pr_handle h) {
    return (h->tile_p > 0 && h->tile_p <= 16 && h->apply_prec != PR_FP64 && h->apply_prec != PR_FP32) ? 1 : 0;
}
std::mutex g_tune_mu;
std::map<TuneKey, std::array<int64_t, 5>> g_tune_cache;

int autotune_apply(pr_handle h) {
    const double t0 = now_s();
    const TuneKey key = {h->device,   h->n,      h->n_p,           h->total_dofs, h->m_p,
                         h->n_items,  h->max_ps, h->min_ps,        h->apply_prec,
                         h->prm.deterministic,   h->uniform ? 1 : 0};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            h->tune_threads = h->stats.tune_threads = (int)it->second[0];
            h->tune_cap = h->stats.tune_cap = it->second[1];
            h->tune_slot = h->stats.tune_slot = (int)it->second[2];
            h->tune_tpw = (int)it->second[3];
            h->stats.tune_tiles_per_wave = it->second[3];
            h->tune_remap = h->stats.tune_xcd_remap = (int)it->second[4];
            h->stats.t_autotune = now_s() - t0;
            return PR_OK;
        }
    }
    hipStream_t s = h->stream;
    const int64_t n = h->n;
    // three vectors (argument, result, scratch) that live only while timing
    struct Scratch {
        hipStream_t s;
        int device;
        double* buf = nullptr;
        size_t got = 0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Scratch() {
            (void)hipStreamSynchronize(s);
            if (buf) pool_release(device, buf, got);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } sc{s, h->device};
    {
        hipError_t e = pool_alloc(h->device, (size_t)3 * (n > 0 ? n : 1) * sizeof(double), (void**)&sc.buf, &sc.got);
        if (e != hipSuccess) {
            sc.buf = nullptr;
            (void)hipGetLastError();
            return pr_fail(h, PR_ERR_OOM, std::string("hipMalloc of the autotune vectors failed: ") +
                                              hipGetErrorString(e));
        }
    }
    double *r = sc.buf, *z = sc.buf + n, *tmp = sc.buf + 2 * n;
    launch_copy(r, h->W, n, s);               // any vector will do
    // a 512 MB write between timed applications evicts the caches: inside a
    // solve the apply follows a product and an orthogonalisation that stream
    // more than the last-level cache holds, so its data arrives cold
    struct Flush {
        int device;
        double* buf = nullptr;
        size_t got = 0;
        ~Flush() {
            if (buf) pool_release(device, buf, got);
        }
    } fl{h->device};
    const int64_t nflush = (int64_t)64 << 20;
    if (pool_alloc(h->device, (size_t)nflush * sizeof(double), (void**)&fl.buf, &fl.got) != hipSuccess) {
        fl.buf = nullptr;
        (void)hipGetLastError();
    }
    PR_HIP(h, hipEventCreate(&sc.e0));
    PR_HIP(h, hipEventCreate(&sc.e1));
    hipEvent_t e0 = sc.e0, e1 = sc.e1;
    auto time_shape = [&](int T, int64_t cap, int T2, int tpw, int rm, float& ms) -> int {
        h->tune_threads = T;
        h->tune_cap = cap;
        h->tune_slot = T2;
        h->tune_tpw = tpw;
        h->tune_remap = rm;
        for (int k = 0; k < 2; ++k) PR_TRY(apply_op(h, r, z, false, tmp));
        ms = 0.0f;
        for (int k = 0; k < 5; ++k) {
            if (fl.buf) launch_zero(fl.buf, nflush, s);
            PR_HIP(h, hipEventRecord(e0, s));
            PR_TRY(apply_op(h, r, z, false, tmp));
            PR_HIP(h, hipEventRecord(e1, s));
            PR_HIP(h, hipEventSynchronize(e1));
            float one = 0.0f;
            PR_HIP(h, hipEventElapsedTime(&one, e0, e1));
            ms += one;
        }
        return PR_OK;
    };
    int bt = 256, bs = 256, bu = 0, br = 1;
    int64_t bc = 0;
    // the default shape is timed first and a later one replaces the best
    // only when it is more than 3 % faster, so that timing noise does not
    // flip the choice between near-equal shapes from run to run
    constexpr float kGain = 0.97f;
    float best = 1e30f;
    {
        float ms = 0.0f;
        PR_TRY(time_shape(256, 0, 256, tpw_choice_default(h), 1, ms));
        best = ms;
        bu = tpw_choice_default(h);
    }
    // tiles per wave is a choice of the fixed-tile kernel for 16-member tiles
    // of p % 4 == 0 only
    const bool tpw_choice = h->tile_p > 0 && h->tile_p <= 16 && (h->tile_p & 3) == 0 &&
                            h->apply_prec != PR_FP64 && h->apply_prec != PR_FP32;
    // XCD-contiguous block order: a choice of the fixed-tile kernel and the padded slot sum
    const bool remap_choice = h->tile_p > 0 || h->ell_c > 0;
    for (int rm : {1, 0}) {
        if (rm == 0 && !remap_choice) break;
        for (int u : {1, 2, 4}) {
            if (u >= 2 && !tpw_choice) break;
            for (int T : {64, 128, 256})
                for (int64_t cap : {(int64_t)0, (int64_t)1024, (int64_t)2048, (int64_t)4096, (int64_t)8192}) {
                    float ms = 0.0f;
                    PR_TRY(time_shape(T, cap, 256, tpw_choice ? u : 0, rm, ms));
                    if (ms < kGain * best) {
                        best = ms;
                        bt = T;
                        bc = cap;
                        bu = tpw_choice ? u : 0;
                        br = rm;
                    }
                }
        }
    }
    if (h->prm.deterministic) {
        best = 1e30f;
        for (int T2 : {256, 128, 64}) {
            float ms = 0.0f;
            PR_TRY(time_shape(bt, bc, T2, bu, br, ms));
            if (ms < (T2 == 256 ? 1.0f : kGain) * best) {
                best = ms;
                bs = T2;
            }
        }
    }
    h->tune_threads = bt;
    h->tune_cap = bc;
    h->tune_slot = bs;
    h->tune_tpw = bu;
    h->stats.tune_tiles_per_wave = bu;
    h->tune_remap = br;
    h->stats.tune_xcd_remap = br;
    h->stats.tune_threads = bt;
    h->stats.tune_slot = bs;
    h->stats.tune_cap = bc;
    h->stats.t_autotune = now_s() - t0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {bt, bc, bs, bu, br};
    return PR_OK;
}

}  // namespace

int pr_precond_internal(pr_handle h, const double* v, double* e, double* t3, const int32_t* stop) {
    return precond(h, v, e, t3, stop);
}

int pr_workspace_internal(pr_handle h, int m) { return ensure_workspace(h, m); }

// Algorithm 1 on subset[0..ns) (all patches when subset is null).
int alg1_core(pr_handle h, const int32_t* subset, int64_t ns, A1Run& R) {
    hipStream_t s = h->stream;
    const int64_t n_p = h->n_p;
    const int64_t stride = (int64_t)h->max_ps * h->max_ps;
    const int crit = h->prm.criterion;
    const double* keynorm = (crit == PR_CRIT_L1) ? h->l1norm : h->fnorm;
    const int64_t N = next_pow2(ns);
    uint64_t *keys = nullptr, *kscr = nullptr;
    int32_t *sidx = nullptr, *vscr = nullptr;
    PR_TRY(dalloc(h, &keys, ns));
    PR_TRY(dalloc(h, &kscr, N));
    PR_TRY(dalloc(h, &sidx, ns));
    PR_TRY(dalloc(h, &vscr, N));
    PR_TRY(dalloc(h, &R.flag, ns + 1));
    PR_TRY(dalloc(h, &R.excl, ns + 1));
    PR_TRY(dalloc(h, &R.scr, scan_scratch_elems(ns + 1) + 2));
    // 1. sort by (size, key); 2. components where no match can cross a gap
    launch_a1_keys(ns, subset, h->pptr, keynorm, keys, sidx, s);
    launch_sort_pairs(keys, sidx, ns, kscr, vscr, s);
    launch_a1_comp_flags(ns, sidx, h->pptr, keynorm, crit, h->prm.eps, h->prm.alg1_prune, R.flag, s);
    launch_exclusive_scan_i64(R.flag, R.excl, ns + 1, R.scr, s);
    int64_t n_comp = 0;
    PR_HIP(h, hipMemcpyAsync(&n_comp, R.excl + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    // 3. members of each component in ascending patch id
    A1Dev d{};
    d.n_p = ns;
    d.n_comp = n_comp;
    d.ptr = h->pptr;
    d.tiles = h->tiles;
    d.toff = h->uniform ? nullptr : h->toff;
    d.uniform_ps = h->uniform ? h->max_ps : 0;
    d.stride = stride;
    int32_t *mem = nullptr, *pos_comp = nullptr, *cstart = nullptr, *next = nullptr, *status = nullptr;
    int32_t *rep_slot = nullptr, *rep_patch = nullptr;
    int32_t *active = nullptr, *cand = nullptr, *ctl = nullptr;
    unsigned long long* counters = nullptr;
    PR_TRY(dalloc(h, &mem, ns));
    PR_TRY(dalloc(h, &pos_comp, ns));
    PR_TRY(dalloc(h, &cstart, n_comp + 1));
    PR_TRY(dalloc(h, &next, n_comp));
    PR_TRY(dalloc(h, &status, ns));
    PR_TRY(dalloc(h, &rep_slot, n_comp));
    PR_TRY(dalloc(h, &rep_patch, ns));
    PR_TRY(dalloc(h, &R.slot_of_patch, n_p));
    PR_TRY(dalloc(h, &R.repof, n_p));
    PR_TRY(dalloc(h, &active, n_comp));
    PR_TRY(dalloc(h, &cand, ns));
    int4* cinfo = nullptr;
    PR_TRY(dalloc(h, &cinfo, ns));
    PR_TRY(dalloc(h, &ctl, 8));
    PR_TRY(dalloc(h, &counters, 4));
    PR_TRY(dalloc(h, &R.dbt, (size_t)ns * stride));
    launch_a1_key2(ns, R.flag, R.excl, sidx, keys, mem, s);
    launch_sort_pairs(keys, mem, ns, kscr, vscr, s);
    launch_a1_cstart(ns, n_comp, keys, pos_comp, cstart, next, s);
    PR_HIP(h, hipMemsetAsync(status, 0, ns * sizeof(int32_t), s));
    PR_HIP(h, hipMemsetAsync(ctl, 0, 8 * sizeof(int32_t), s));
    PR_HIP(h, hipMemsetAsync(counters, 0, 4 * sizeof(unsigned long long), s));
    d.ctl = ctl;
    d.counters = counters;
    d.cstart = cstart;
    d.next = next;
    d.mem = mem;
    d.pos_comp = pos_comp;
    d.status = status;
    d.rep_slot = rep_slot;
    d.rep_patch = rep_patch;
    d.slot_of_patch = R.slot_of_patch;
    d.repof = R.repof;
    d.active = active;
    d.cand = cand;
    d.cinfo = cinfo;
    d.dbt = R.dbt;
    d.inv = nullptr;
    d.inv_info = nullptr;
    d.spec = d.spec_n = d.pairm = d.ent = d.ent_n = d.ent_slot = nullptr;
    // 4. rounds, all components at once, until no component opens an entry.
    // Once they run long (about one entry per round in a large component),
    // the unresolved patches are inverted in one batch and later rounds open
    // up to kA1Spec entries per component, with the inverses taken from the
    // batch (skipped when that much memory is not free).
    int batch = 2;
    int64_t started = 0;
    int32_t c8[8];
    for (;;) {
        if (d.inv) launch_a1_spec_rounds(batch, d, crit, h->prm.eps, h->max_ps, s);
        else launch_a1_rounds(batch, d, crit, h->prm.eps, h->max_ps, s);
        started += batch;
        PR_HIP(h, hipMemcpyAsync(c8, ctl, sizeof(c8), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        if (c8[2]) break;
        if (!d.inv && started >= kA1BatchInvertAfter) {
            const size_t need = (size_t)ns * stride * sizeof(double);
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b / 2 > need) {
                PR_TRY(dalloc(h, &d.inv, (size_t)ns * stride));
                PR_TRY(dalloc(h, &d.inv_info, ns));
                const size_t nk = (size_t)n_comp * kA1Spec;
                PR_TRY(dalloc(h, &d.spec, nk));
                PR_TRY(dalloc(h, &d.spec_n, n_comp));
                PR_TRY(dalloc(h, &d.pairm, nk));
                PR_TRY(dalloc(h, &d.ent, nk));
                PR_TRY(dalloc(h, &d.ent_n, n_comp));
                PR_TRY(dalloc(h, &d.ent_slot, nk));
                launch_a1_preinvert(d, h->max_ps, s);
                h->stats.alg1_batch_inverted = 1;
            } else {
                (void)hipGetLastError();
            }
        }
        if (batch < 64) batch *= 2;
    }
    PR_HIP(h, hipGetLastError());
    if (d.inv) {
        dfree(h, d.inv);       // the stream was synchronised above
        dfree(h, d.inv_info);
        for (int32_t* q : {d.spec, d.spec_n, d.pairm, d.ent, d.ent_n, d.ent_slot}) dfree(h, q);
    }
    if (c8[5] != 0)
        return pr_fail(h, PR_ERR_SINGULAR_PATCH, "zero pivot in database patch " + std::to_string(c8[5] - 1));
    R.m = c8[0];
    R.rounds = c8[4];
    PR_HIP(h, hipMemcpyAsync(R.cnt, counters, sizeof(R.cnt), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    return PR_OK;
}


void pr_set_global_error(const std::string& s) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_last_error = s;
}

int pr_fail(pr_handle h, int code, const std::string& msg) {
    if (h) h->last_error = msg;
    pr_set_global_error(msg);
    return code;
}

extern "C" {

void pr_params_default(pr_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->algo = PR_ALGO_FULL;
    p->criterion = PR_CRIT_SPECTRAL;
    p->eps = 1e-8;
    p->m_target = 0;
    p->partition_bc = 1;
    p->kmeans_max_iter = 100;
    p->seed = 5;
    p->tie_rel = 1e-9;
    p->apply_precision = PR_FP64;
    p->omega = 1.0;
    p->sweeps = 1;
    p->gmres_restart = 30;
    p->max_iters = 10000;
    p->deterministic = 0;
    p->stream = nullptr;
    p->mlp = 0;
    p->mlp_topk = 4;
    p->mlp_train_frac = 0.1;
    p->mlp_epochs = 60;
    p->mlp_hidden = 64;
    p->mlp_seed = 6;
    p->mlp_lr = 3e-3;
    p->mlp_batch = 256;
    p->mlp_precision = PR_FP16;
    p->graph = 0;
    p->autotune = 0;
    p->apply_form = PR_FORM_AUTO;
    p->alg1_prune = 1;
    p->alg1_match = 0;
    p->flexible = 0;
    p->orth = 0;
}

const char* pr_status_string(int st) {
    switch (st) {
        case PR_OK: return "ok";
        case PR_NOT_CONVERGED: return "not converged";
        case PR_ERR_INVALID_ARG: return "invalid argument";
        case PR_ERR_HOST_POINTER: return "host pointer where device memory is required";
        case PR_ERR_DOF_OUT_OF_RANGE: return "patch dof out of range";
        case PR_ERR_DUP_DOF_IN_PATCH: return "duplicate dof in a patch";
        case PR_ERR_UNCOVERED_DOF: return "dof in no patch";
        case PR_ERR_SINGULAR_PATCH: return "singular patch matrix";
        case PR_ERR_NONFINITE: return "non-finite value";
        case PR_ERR_OOM: return "out of device memory";
        case PR_ERR_HIP: return "HIP runtime error";
        case PR_ERR_UNSUPPORTED: return "unsupported input";
        case PR_ERR_BAD_CSR: return "malformed CSR matrix";
        case PR_ERR_BAD_PATCH_PTR: return "malformed patch pointer array";
        default: return "unknown status";
    }
}

const char* pr_last_error(pr_handle h) {
    if (h) return h->last_error.c_str();
    std::lock_guard<std::mutex> lk(g_mu);
    return g_last_error.c_str();
}

void pr_destroy(pr_handle h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (auto e : h->evpool) (void)hipEventDestroy(e);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->bgexec) (void)hipGraphExecDestroy(h->bgexec);
    if (h->gstream) {
        (void)hipStreamSynchronize(h->gstream);
        (void)hipStreamDestroy(h->gstream);
    }
    for (auto& b : h->owned) pool_release(h->device, b.p, b.bytes);
    if (h->hh) pool_host_release(h->hh, h->hh_got);
    delete h;
}

int pr_set_stream(pr_handle h, void* st) {
    if (!h) return PR_ERR_INVALID_ARG;
    // work queued on the old stream finishes first: pr_destroy waits for the
    // current stream only before the handle's blocks go back to the cache
    if ((hipStream_t)st != h->stream) PR_HIP(h, hipStreamSynchronize(h->stream));
    h->stream = (hipStream_t)st;
    h->prm.stream = st;
    return PR_OK;
}

int pr_validate_host(const pr_csr* A, const pr_patches* P) {
    if (!A || !P) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "null argument");
    if (A->n <= 0 || A->nnz < 0 || P->n_p <= 0 || !A->row_ptr || !P->ptr || (A->nnz > 0 && (!A->col || !A->val)))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "bad sizes or null arrays");
    const int64_t n = A->n;
    if (A->row_ptr[0] != 0 || A->row_ptr[n] != A->nnz) return pr_fail(nullptr, PR_ERR_BAD_CSR, "row_ptr ends");
    for (int64_t i = 0; i < n; ++i) {
        if (A->row_ptr[i + 1] < A->row_ptr[i]) return pr_fail(nullptr, PR_ERR_BAD_CSR, "row_ptr not monotone");
        int32_t prev = -1;
        for (int64_t q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q) {
            const int32_t c = A->col[q];
            if (c < 0 || c >= n || c <= prev) return pr_fail(nullptr, PR_ERR_BAD_CSR, "column out of range or unsorted");
            prev = c;
        }
    }
    const int64_t total = P->ptr[P->n_p];
    if (P->ptr[0] != 0 || total < 0 || (total > 0 && !P->dofs)) return pr_fail(nullptr, PR_ERR_BAD_PATCH_PTR, "ptr ends");
    std::vector<int32_t> cnt(n, 0);
    int rc_unsup = 0;
    for (int64_t k = 0; k < P->n_p; ++k) {
        const int64_t s = P->ptr[k], e = P->ptr[k + 1];
        if (e <= s || e > total) return pr_fail(nullptr, PR_ERR_BAD_PATCH_PTR, "empty patch or ptr not monotone");
        if (e - s > kWideMaxPs) rc_unsup = 1;
        for (int64_t q = s; q < e; ++q) {
            const int32_t g = P->dofs[q];
            if (g < 0 || g >= n) return pr_fail(nullptr, PR_ERR_DOF_OUT_OF_RANGE, "dof out of range in patch " + std::to_string(k));
            for (int64_t q2 = s; q2 < q; ++q2)
                if (P->dofs[q2] == g) return pr_fail(nullptr, PR_ERR_DUP_DOF_IN_PATCH, "duplicate dof in patch " + std::to_string(k));
            cnt[g]++;
        }
    }
    if (rc_unsup) return pr_fail(nullptr, PR_ERR_UNSUPPORTED, "patch with more than " + std::to_string(kWideMaxPs) + " dofs");
    for (int64_t i = 0; i < n; ++i)
        if (cnt[i] == 0) return pr_fail(nullptr, PR_ERR_UNCOVERED_DOF, "dof " + std::to_string(i) + " in no patch");
    for (int64_t q = 0; q < A->nnz; ++q)
        if (!std::isfinite(A->val[q])) return pr_fail(nullptr, PR_ERR_NONFINITE, "non-finite matrix value");
    return PR_OK;
}

namespace {
constexpr char kDbMagic[8] = {'P', 'R', 'D', 'B', '0', '0', '0', '1'};
constexpr int64_t kDbHeader = 40;
}  // namespace

int pr_export_database(pr_handle h, void* buf, int64_t* bytes) {
    if (!h || !bytes) return pr_fail(h, PR_ERR_INVALID_ARG, "null argument");
    const int64_t need = kDbHeader + 4 * (h->n_p + h->m_p);
    if (!buf) {
        *bytes = need;
        return PR_OK;
    }
    if (*bytes < need) return pr_fail(h, PR_ERR_INVALID_ARG, "buffer smaller than " + std::to_string(need) + " bytes");
    char* b = (char*)buf;
    std::memcpy(b, kDbMagic, 8);
    std::memcpy(b + 8, &h->n_p, 8);
    std::memcpy(b + 16, &h->m_p, 8);
    std::memcpy(b + 24, &h->prm.algo, 4);
    std::memcpy(b + 28, &h->prm.criterion, 4);
    std::memcpy(b + 32, &h->prm.eps, 8);
    PR_HIP(h, hipStreamSynchronize(h->stream));
    PR_HIP(h, hipMemcpy(b + kDbHeader, h->phi, h->n_p * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::memcpy(b + kDbHeader + 4 * h->n_p, h->reps_host.data(), h->m_p * sizeof(int32_t));
    *bytes = need;
    return PR_OK;
}

int pr_setup_reuse(const pr_csr* A, const pr_patches* P, const pr_params* prm, const void* db, int64_t bytes,
                   pr_handle* out) {
    if (!A || !P || !prm || !db || !out) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "null argument");
    if (prm->algo == PR_ALGO_FULL || prm->algo == PR_ALGO_BOOTSTRAP || prm->mlp || prm->alg1_match)
        return pr_fail(nullptr, PR_ERR_INVALID_ARG,
                       "reuse serves Algorithm 1 (first match, no predictor) and the k-means variants");
    const char* b = (const char*)db;
    int64_t n_p = 0, m_p = 0;
    if (bytes < kDbHeader || std::memcmp(b, kDbMagic, 8) != 0)
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "not a database blob");
    std::memcpy(&n_p, b + 8, 8);
    std::memcpy(&m_p, b + 16, 8);
    if (n_p != P->n_p || m_p < 1 || m_p > n_p || bytes < kDbHeader + 4 * (n_p + m_p))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "blob does not fit these patches");
    ReuseSeed seed;
    seed.phi.resize(n_p);
    seed.reps.resize(m_p);
    std::memcpy(seed.phi.data(), b + kDbHeader, 4 * n_p);
    std::memcpy(seed.reps.data(), b + kDbHeader + 4 * n_p, 4 * m_p);
    for (int64_t i = 0; i < n_p; ++i)
        if (seed.phi[i] < 0 || seed.phi[i] >= m_p)
            return pr_fail(nullptr, PR_ERR_INVALID_ARG, "blob maps a patch outside the database");
    if (prm->algo == PR_ALGO_TOLERANCE) {
        for (int64_t j = 0; j < m_p; ++j) {
            const int32_t r = seed.reps[j];
            if (r < 0 || r >= n_p || seed.phi[r] != j || (j > 0 && r <= seed.reps[j - 1]))
                return pr_fail(nullptr, PR_ERR_INVALID_ARG,
                               "blob entries must be ascending patch ids mapped to themselves");
        }
    }
    g_reuse_pending = &seed;
    const int rc = pr_setup(A, P, prm, out);
    g_reuse_pending = nullptr;
    return rc;
}

int pr_setup(const pr_csr* A, const pr_patches* P, const pr_params* prm, pr_handle* out) {
    if (!A || !P || !out) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    pr_params defaults;
    pr_params_default(&defaults);
    const pr_params& pm = prm ? *prm : defaults;
    if (A->n <= 0 || A->nnz < 0 || P->n_p <= 0) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "bad sizes");
    if (A->n > INT_MAX - 1 || P->n_p > INT_MAX - 1) return pr_fail(nullptr, PR_ERR_UNSUPPORTED, "more than 2^31 dofs or patches");
    if (pm.algo < PR_ALGO_FULL || pm.algo > PR_ALGO_BOOTSTRAP || pm.criterion < 0 || pm.criterion > 2 ||
        pm.apply_precision < 0 || pm.apply_precision > 4 || pm.sweeps < 1 || pm.gmres_restart < 1 ||
        pm.gmres_restart > 64 || !(pm.eps >= 0.0) || !(pm.omega > 0.0) ||
        (pm.apply_form != PR_FORM_AUTO && pm.apply_form != PR_FORM_GENERAL && pm.apply_form != PR_FORM_TILES) ||
        (pm.alg1_prune != 0 && pm.alg1_prune != 1) || (pm.alg1_match != 0 && pm.alg1_match != 1) ||
        (pm.flexible != 0 && pm.flexible != 1) || (pm.orth != 0 && pm.orth != 1))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "bad parameter value");
    if (pm.alg1_match == 1 && (pm.algo != PR_ALGO_TOLERANCE || pm.mlp != 0 || !(pm.tie_rel >= 0.0)))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "closest matching needs PR_ALGO_TOLERANCE without mlp");
    if (pm.algo != PR_ALGO_FULL && pm.algo != PR_ALGO_TOLERANCE &&
        (pm.kmeans_max_iter < 1 || !(pm.tie_rel >= 0.0)))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "bad clustering parameter");
    if (pm.mlp && (pm.algo != PR_ALGO_TOLERANCE || pm.mlp_topk < 1 || pm.mlp_topk > 8 ||
                   !(pm.mlp_train_frac > 0.0 && pm.mlp_train_frac <= 1.0) || pm.mlp_epochs < 0 ||
                   pm.mlp_hidden < 1 || pm.mlp_hidden > 1024 || pm.mlp_batch < 1 || !(pm.mlp_lr > 0.0) ||
                   (pm.mlp_precision != PR_FP16 && pm.mlp_precision != PR_FP32)))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "bad predictor parameter");
    {
        int rc;
        if ((rc = check_dev(nullptr, A->row_ptr, "A.row_ptr")) < 0) return rc;
        if (A->nnz > 0 && (rc = check_dev(nullptr, A->col, "A.col")) < 0) return rc;
        if (A->nnz > 0 && (rc = check_dev(nullptr, A->val, "A.val")) < 0) return rc;
        if ((rc = check_dev(nullptr, P->ptr, "P.ptr")) < 0) return rc;
        if ((rc = check_dev(nullptr, P->dofs, "P.dofs")) < 0) return rc;
    }
    pr_handle h = new pr_handle_s();
    h->prm = pm;
    h->stream = (hipStream_t)pm.stream;
    hipStream_t s = h->stream;
    (void)hipGetDevice(&h->device);
    if (g_reuse_pending) {
        h->has_reuse = true;
        h->reuse_phi = g_reuse_pending->phi;
        h->reuse_reps = g_reuse_pending->reps;
    }
    const double t0 = now_s();
    h->n = A->n;
    h->nnz = A->nnz;
    h->n_p = P->n_p;
    auto fail = [&](int rc) {
        pr_set_global_error(h->last_error);
        pr_destroy(h);
        return rc;
    };
#define SETUP_TRY(expr)               \
    do {                              \
        int _s = (expr);              \
        if (_s < 0) return fail(_s);  \
    } while (0)
#define SETUP_HIP(expr)                                                                      \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess) {                                                              \
            pr_fail(h, _e == hipErrorOutOfMemory ? PR_ERR_OOM : PR_ERR_HIP,                  \
                    std::string(#expr) + ": " + hipGetErrorString(_e));                      \
            return fail(_e == hipErrorOutOfMemory ? PR_ERR_OOM : PR_ERR_HIP);                \
        }                                                                                    \
    } while (0)

    int64_t total = 0;
    SETUP_HIP(hipMemcpyAsync(&total, P->ptr + P->n_p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipStreamSynchronize(s));
    if (total <= 0 || total > INT_MAX) {
        pr_fail(h, PR_ERR_BAD_PATCH_PTR, "patch ptr[n_p] out of range");
        return fail(PR_ERR_BAD_PATCH_PTR);
    }
    h->total_dofs = total;
    SETUP_TRY(dalloc(h, &h->rowptr, h->n + 1));
    SETUP_TRY(dalloc(h, &h->col, h->nnz + kCsrPad));     // padded: the SpMV reads entries in pairs
    SETUP_TRY(dalloc(h, &h->val, h->nnz + kCsrPad));
    SETUP_TRY(dalloc(h, &h->pptr, h->n_p + 1));
    SETUP_TRY(dalloc(h, &h->pdofs, total));
    SETUP_HIP(hipMemcpyAsync(h->rowptr, A->row_ptr, (h->n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (h->nnz > 0) {
        SETUP_HIP(hipMemcpyAsync(h->col, A->col, h->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        SETUP_HIP(hipMemcpyAsync(h->val, A->val, h->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    SETUP_HIP(hipMemsetAsync(h->col + h->nnz, 0, kCsrPad * sizeof(int32_t), s));
    SETUP_HIP(hipMemsetAsync(h->val + h->nnz, 0, kCsrPad * sizeof(double), s));
    SETUP_HIP(hipMemcpyAsync(h->pptr, P->ptr, (h->n_p + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    SETUP_HIP(hipMemcpyAsync(h->pdofs, P->dofs, total * sizeof(int32_t), hipMemcpyDeviceToDevice, s));

    // ---- validation -------------------------------------------------------
    int32_t* flags = nullptr;
    int32_t* minmax = nullptr;
    SETUP_TRY(dalloc(h, &flags, 8));
    SETUP_TRY(dalloc(h, &minmax, 2));
    const int32_t f0[8] = {0, 0, INT_MAX, INT_MAX, INT_MAX, INT_MAX, 0, 0};
    const int32_t mm0[2] = {INT_MAX, 0};
    SETUP_HIP(hipMemcpyAsync(flags, f0, sizeof(f0), hipMemcpyHostToDevice, s));
    SETUP_HIP(hipMemcpyAsync(minmax, mm0, sizeof(mm0), hipMemcpyHostToDevice, s));
    launch_validate_csr(h->rowptr, h->col, h->n, h->nnz, flags, s);
    launch_validate_patches(h->pptr, h->pdofs, h->n_p, h->n, total, flags, minmax, s);
    int32_t fl[8], mm[2];
    SETUP_HIP(hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipMemcpyAsync(mm, minmax, sizeof(mm), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipStreamSynchronize(s));
    SETUP_HIP(hipGetLastError());
    if (fl[0]) { pr_fail(h, PR_ERR_BAD_CSR, "malformed CSR (row_ptr, column range or order)"); return fail(PR_ERR_BAD_CSR); }
    if (fl[1]) { pr_fail(h, PR_ERR_BAD_PATCH_PTR, "malformed patch ptr or empty patch"); return fail(PR_ERR_BAD_PATCH_PTR); }
    if (fl[6]) {
        // a patch above 32 dofs: the block-per-patch kernels (k_wide.hip)
        if (mm[1] > kWideMaxPs) {
            pr_fail(h, PR_ERR_UNSUPPORTED, "patch with more than " + std::to_string(kWideMaxPs) + " dofs");
            return fail(PR_ERR_UNSUPPORTED);
        }
        const char* why = nullptr;
        if (pm.algo != PR_ALGO_FULL && pm.algo != PR_ALGO_TOLERANCE) why = "Algorithm 2";
        else if (pm.mlp) why = "the learned predictor";
        else if (pm.alg1_match != 0) why = "closest matching";
        else if (h->has_reuse) why = "database reuse";
        else if (pm.apply_precision != PR_FP64 && pm.apply_precision != PR_FP32) why = "a 16-bit apply";
        if (why) {
            pr_fail(h, PR_ERR_UNSUPPORTED, std::string("patches above 32 dofs do not support ") + why);
            return fail(PR_ERR_UNSUPPORTED);
        }
        h->wide = true;
        launch_validate_wide(h->pptr, h->pdofs, h->n_p, h->n, flags, s);
        SETUP_HIP(hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, s));
        SETUP_HIP(hipStreamSynchronize(s));
        SETUP_HIP(hipGetLastError());
    }
    if (fl[2] != INT_MAX) { pr_fail(h, PR_ERR_DOF_OUT_OF_RANGE, "dof out of range in patch " + std::to_string(fl[2])); return fail(PR_ERR_DOF_OUT_OF_RANGE); }
    if (fl[3] != INT_MAX) { pr_fail(h, PR_ERR_DUP_DOF_IN_PATCH, "duplicate dof in patch " + std::to_string(fl[3])); return fail(PR_ERR_DUP_DOF_IN_PATCH); }
    h->min_ps = mm[0];
    h->max_ps = mm[1];
    h->uniform = (h->min_ps == h->max_ps);

    // ---- W (Section 2) ------------------------------------------------------
    SETUP_TRY(dalloc(h, &h->cnt, h->n));
    SETUP_TRY(dalloc(h, &h->W, h->n));
    SETUP_HIP(hipMemsetAsync(h->cnt, 0, h->n * sizeof(int32_t), s));
    launch_cover(h->pdofs, total, h->cnt, s);
    launch_weights(h->cnt, h->n, h->W, flags, s);
    const double t1 = now_s();

    // ---- tiles (Section 2) --------------------------------------------------
    SETUP_TRY(dalloc(h, &h->toff, h->n_p + 1));
    int64_t* scan_scr = nullptr;
    SETUP_TRY(dalloc(h, &scan_scr, h->n_p + 2 + scan_scratch_elems(h->n_p + 1)));
    launch_tile_offsets(h->pptr, h->n_p, h->toff, scan_scr, s);
    SETUP_HIP(hipMemcpyAsync(&h->total_tile, h->toff + h->n_p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipStreamSynchronize(s));
    if (fl[4] != INT_MAX) { pr_fail(h, PR_ERR_UNCOVERED_DOF, "dof " + std::to_string(fl[4]) + " lies in no patch"); return fail(PR_ERR_UNCOVERED_DOF); }
    SETUP_TRY(dalloc(h, &h->tiles, h->total_tile));
    SETUP_TRY(dalloc(h, &h->keys, h->n_p));
    SETUP_TRY(dalloc(h, &h->fnorm, h->n_p));
    SETUP_TRY(dalloc(h, &h->l1norm, h->n_p));
    if (h->wide)
        launch_extract_wide(h->rowptr, h->col, h->val, h->pptr, h->pdofs, h->n_p, h->uniform ? nullptr : h->toff,
                            h->uniform ? h->max_ps : 0, h->tiles, h->keys, h->fnorm, h->l1norm, flags, s);
    else
        launch_extract(h->rowptr, h->col, h->val, h->pptr, h->pdofs, h->n_p, h->uniform ? nullptr : h->toff,
                       h->uniform ? h->max_ps : 0, h->max_ps, h->tiles, h->keys, h->fnorm, h->l1norm, flags, s);
    SETUP_HIP(hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipStreamSynchronize(s));
    SETUP_HIP(hipGetLastError());
    if (fl[5] != INT_MAX) { pr_fail(h, PR_ERR_NONFINITE, "non-finite entry in patch " + std::to_string(fl[5])); return fail(PR_ERR_NONFINITE); }
    const double t2 = now_s();

    // ---- database (Section 3) ----------------------------------------------
    if (pm.algo == PR_ALGO_FULL) SETUP_TRY(run_full(h));
    else if (pm.algo == PR_ALGO_TOLERANCE && h->has_reuse) SETUP_TRY(run_alg1_reuse(h));
    else if (pm.algo == PR_ALGO_TOLERANCE && h->wide) SETUP_TRY(run_alg1_wide(h));
    else if (pm.algo == PR_ALGO_TOLERANCE && pm.mlp) SETUP_TRY(run_alg1_mlp(h));
    else if (pm.algo == PR_ALGO_TOLERANCE) SETUP_TRY(run_alg1(h));
    else SETUP_TRY(run_kmeans(h));
    SETUP_HIP(hipStreamSynchronize(s));
    SETUP_HIP(hipGetLastError());
    const double t3 = now_s();
    // hybrid sliced-ELL copy of A for the solve (64-row slices, diagonal or
    // column form per slice)
    {
        const int64_t ns = (h->n + 63) / 64;
        int64_t* slen = nullptr;
        int64_t* sscr = nullptr;
        int32_t* dtmp = nullptr;
        unsigned long long* sacc = nullptr;
        SETUP_TRY(dalloc(h, &slen, ns + 1));
        SETUP_TRY(dalloc(h, &sscr, scan_scratch_elems(ns + 1) + 2));
        SETUP_TRY(dalloc(h, &h->soff, ns + 1));
        SETUP_TRY(dalloc(h, &h->sfmt, ns));
        SETUP_TRY(dalloc(h, &dtmp, (size_t)ns * (kSellMaxDiag + 1)));
        SETUP_TRY(dalloc(h, &sacc, 5));
        SETUP_HIP(hipMemsetAsync(sacc, 0, 5 * sizeof(unsigned long long), s));
        launch_sell_plan(h->rowptr, h->col, h->n, slen, h->sfmt, dtmp, sacc, s);
        launch_exclusive_scan_i64(slen, h->soff, ns + 1, sscr, s);
        int64_t stot = 0;
        unsigned long long sa[5];
        SETUP_HIP(hipMemcpyAsync(&stot, h->soff + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SETUP_HIP(hipMemcpyAsync(sa, sacc, sizeof(sa), hipMemcpyDeviceToHost, s));
        SETUP_HIP(hipStreamSynchronize(s));
        SETUP_TRY(dalloc(h, &h->sval, stot));
        SETUP_TRY(dalloc(h, &h->scol, sa[2] > 0 ? stot : 1));   // column-form slices only
        SETUP_TRY(dalloc(h, &h->sdoff, stot / 64 + kSellOffsetPad));
        launch_sell_fill(h->rowptr, h->col, h->val, h->n, h->soff, h->sfmt, dtmp, h->sval, h->scol, h->sdoff, s);
        h->stats.sell_slots = stot;
        h->stats.sell_diag_slices = (int64_t)sa[0];
        h->stats.sell_diag_offsets = (int64_t)sa[1];
        h->stats.sell_col_entries = (int64_t)sa[2];
        h->stats.sell_csr_slices = (int64_t)sa[3];
        h->stats.sell_csr_entries = (int64_t)sa[4];
    }
    SETUP_TRY(run_group(h));
    h->stats.tune_xcd_remap = (h->tile_p > 0 || h->ell_c > 0) ? h->tune_remap : 0;
    if (pm.autotune && !h->wide) SETUP_TRY(autotune_apply(h));   // the wide kernels have one shape

    // boundary groups (distinct keys) for the stats
    {
        int64_t T = 1024;
        while (T < 2 * h->n_p) T <<= 1;
        uint32_t* table = nullptr;
        unsigned* dcount = nullptr;
        SETUP_TRY(dalloc(h, &table, T));
        SETUP_TRY(dalloc(h, &dcount, 2));
        launch_count_distinct_u32(h->keys, h->n_p, table, T, dcount, s);
        unsigned c2[2];
        SETUP_HIP(hipMemcpyAsync(c2, dcount, sizeof(c2), hipMemcpyDeviceToHost, s));
        SETUP_HIP(hipStreamSynchronize(s));
        SETUP_HIP(hipGetLastError());
        h->stats.n_groups = (int32_t)(c2[0] + c2[1]);
    }
    const double t4 = now_s();
    h->stats.n = h->n;
    h->stats.nnz = h->nnz;
    h->stats.n_p = h->n_p;
    h->stats.m_p = h->m_p;
    h->stats.max_ps = h->max_ps;
    h->stats.min_ps = h->min_ps;
    h->stats.algo = pm.algo;
    h->stats.bytes_tiles = h->total_tile * 8;
    h->stats.t_validate = t1 - t0;
    h->stats.t_extract = t2 - t1;
    h->stats.t_database = t3 - t2;
    h->stats.t_factor = 0.0;
    h->stats.t_group = t4 - t3;
    h->stats.t_total = t4 - t0;
    h->stats.apply_precision = pm.apply_precision;
#undef SETUP_TRY
#undef SETUP_HIP
    *out = h;
    return PR_OK;
}

int pr_apply(pr_handle h, const double* r, double* z) {
    if (!h) return PR_ERR_INVALID_ARG;
    PR_TRY(check_dev(h, r, "r"));
    PR_TRY(check_dev(h, z, "z"));
    if (r == z) return pr_fail(h, PR_ERR_INVALID_ARG, "r and z must be distinct");
    PR_TRY(apply_op(h, r, z, false, nullptr));
    PR_TRY(coarse_add(h, r, z, nullptr));
    PR_HIP(h, hipGetLastError());
    return PR_OK;
}

int pr_solve(pr_handle h, const double* b, double* x, double tol) {
    if (!h) return PR_ERR_INVALID_ARG;
    PR_TRY(check_dev(h, b, "b"));
    PR_TRY(check_dev(h, x, "x"));
    if (!(tol > 0.0)) return pr_fail(h, PR_ERR_INVALID_ARG, "tol must be positive");
    if (h->nsys > 0) return solve_batch(h, b, x, tol);
    const double tstart = now_s();
    // optional per-class device timing: 0 apply, 1 spmv, 2 orthogonalisation
    const bool timing = h->prm.timing != 0;
    // timing = k > 1: only every k-th Arnoldi step is bracketed (the events
    // themselves add a gap between kernels)
    const int tstride = h->prm.timing > 1 ? h->prm.timing : 1;
    bool tsel = timing;
    // graph replay of whole restart cycles (not with per-kernel timing)
    const bool use_graph = h->prm.graph != 0 && !timing;
    // a span records the cycle and Arnoldi step it belongs to (-1: cycle end),
    // so that the steps a stopped cycle skipped are not counted
    struct Span { int cls; hipEvent_t a, b; int64_t cyc; int j; };
    std::vector<Span> spans;
    std::vector<int64_t> done_cols;   // Arnoldi steps that ran, per cycle
    int64_t tcyc = -1;
    int tj = -1;
    size_t evnext = 0;
    auto grab = [&]() -> hipEvent_t {
        if (evnext >= h->evpool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            h->evpool.push_back(e);
        }
        return h->evpool[evnext++];
    };
    hipStream_t s = h->stream;
    hipEvent_t tb = nullptr;
    auto tbeg = [&]() {
        if (tsel) {
            tb = grab();
            if (tb) (void)hipEventRecord(tb, s);
        }
    };
    auto tend = [&](int cls) {
        if (tsel && tb) {
            hipEvent_t te = grab();
            if (te) {
                (void)hipEventRecord(te, s);
                spans.push_back({cls, tb, te, tcyc, tj});
            }
        }
    };
    const int m = h->prm.gmres_restart;
    const int64_t n = h->n;
    PR_TRY(ensure_workspace(h, m));
    const bool flex = h->prm.flexible != 0;
    if (flex && h->zb_restart < m) {
        PR_TRY(dalloc(h, &h->Zb, (size_t)m * h->ldv));
        h->zb_restart = m;
        if (h->gexec) {                     // a captured cycle holds the old basis
            (void)hipGraphExecDestroy(h->gexec);
            h->gexec = nullptr;
            h->graph_m = -1;
        }
    }
    if (use_graph) {
        // a capture needs a stream of its own; b and x live in handle memory
        // so that one captured cycle serves every later solve
        if (!h->gstream) PR_HIP(h, hipStreamCreate(&h->gstream));
        if (!h->gb) {
            PR_TRY(dalloc(h, &h->gb, n));
            PR_TRY(dalloc(h, &h->gx, n));
        }
        PR_HIP(h, hipStreamSynchronize(h->stream));
        s = h->gstream;
    }
    struct StreamSwap {
        pr_handle h;
        hipStream_t keep;
        ~StreamSwap() { h->stream = keep; }
    } swap{h, h->stream};
    h->stream = s;
    double* V = h->V;
    double* w = h->w;
    double* r = h->t1;
    double* zt = h->t2;
    double* t3 = h->t2 + n;
    double* hd = h->hd;
    double* hh = h->hh;
    const int64_t ldv = h->ldv;
    double* red = h->red;
    // device GMRES state: R ((m+1) x m), rotations, residual vector g, y,
    // estimate, absolute tolerance and iteration base
    double* R = h->gm;
    double* cs = R + (int64_t)(m + 1) * m;
    double* sn = cs + m;
    double* g = sn + m;
    double* y = g + m + 1;
    double* est_d = y + m;
    double* tol_d = est_d + 1;
    int64_t* itb_d = reinterpret_cast<int64_t*>(tol_d + 1);
    // delayed reorthogonalisation: the unrotated Hessenberg matrix, T and
    // the update coefficients
    double* Hu = reinterpret_cast<double*>(itb_d + 1);
    double* Tm = Hu + (int64_t)(m + 1) * m;
    double* coef = Tm + (int64_t)m * m;
    const bool delayed = h->prm.orth == 0 && m <= 31;
    double* red_dot = red;                                    // dot-pass partials, output-major
    double* red_upd = red + (int64_t)gs_blocks(n) * 33;       // update-pass partials, output-major
    int32_t* gctl = h->gctl;
    int32_t* gctl_h = reinterpret_cast<int32_t*>(hh + 240);   // pinned mirror of gctl
    int64_t* itb_h = reinterpret_cast<int64_t*>(hh + 236);

    const double* bw = use_graph ? h->gb : b;
    double* xw = use_graph ? h->gx : x;
    if (use_graph) launch_copy(h->gb, b, n, s);
    auto sync_read = [&](int count) -> int {
        PR_HIP(h, hipMemcpyAsync(hh, hd, count * sizeof(double), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        return PR_OK;
    };
    // ||b||
    launch_gs(0, bw, n, 1, const_cast<double*>(bw), n, nullptr, red, hd, s);
    PR_TRY(sync_read(1));
    const double bnorm = std::sqrt(hh[0]);
    launch_zero(xw, n, s);
    h->sinfo = pr_solve_info{};
    if (!std::isfinite(bnorm)) return pr_fail(h, PR_ERR_NONFINITE, "non-finite right-hand side");
    if (bnorm == 0.0) {
        if (use_graph) launch_copy(x, xw, n, s);
        h->sinfo.status = PR_OK;
        PR_HIP(h, hipStreamSynchronize(s));
        return PR_OK;
    }
    hh[235] = tol * bnorm;
    PR_HIP(h, hipMemcpyAsync(tol_d, hh + 235, sizeof(double), hipMemcpyHostToDevice, s));
    launch_copy(r, bw, n, s);
    launch_gs(0, r, n, 1, r, n, nullptr, red, hd, s);     // ||r||^2 -> hd[0]

    // One restart cycle, all on the device: V_0 = r / ||r||, m Arnoldi steps
    // (each ends in the device-side Givens update and stopping test; later
    // kernels of a stopped cycle return at once), then x += M(V y),
    // r = b - A x and ||r||^2 -> hd[0] for the next cycle.
    auto enqueue_cycle = [&]() -> int {
        ++tcyc;
        launch_cycle_init(g, m, hd, gctl, s);
        launch_scale(r, V, hd, n, s);
        for (int j = 0; j < m; ++j) {
            tsel = timing && (tcyc * m + j) % tstride == 0;
            tj = j;
            double* vj = V + (int64_t)j * ldv;
            double* zj = flex ? h->Zb + (int64_t)j * ldv : zt;   // flexible: keep z_j = M v_j
            tbeg();
            PR_TRY(precond(h, vj, zj, t3, gctl, false));
            tend(0);
            if (h->n0 > 0) {
                tbeg();
                PR_TRY(coarse_add(h, vj, zj, gctl));
                tend(3);
            }
            tbeg();
            launch_spmv_sell(h->sell(), n, zj, nullptr, w, s, gctl);
            tend(1);
            // classical Gram-Schmidt with selective reorthogonalisation:
            // pass 1: h1 = V^T w, ||w||^2 ; pass 2: w -= V h1, h2 = V^T w, ||w||^2 ;
            // pass 3 (only when pass 2 lost more than a factor sqrt(2)):
            // w -= V h2, ||w||^2 ; then v_{j+1} = w / ||w||.  Beyond 31 basis
            // vectors every step takes all three passes.
            if (delayed) {
                // delayed reorthogonalisation: the dot pass [Q, u_raw]^T w, the
                // coefficient step (column j-1 made final with its Givens
                // rotation and stopping test, the provisional column j), the
                // update pass (v_j over u_raw, the next unnormalised vector in
                // column j+1 and its dots with [Q, v_j])
                tbeg();
                launch_gs_partials(V, ldv, j + 1, w, n, red_dot, s, gctl);
                launch_dcgs_coef(j, m, false, red_dot, red_upd, n, Hu, R, cs, sn, g, est_d, Tm, coef, gctl, tol_d,
                                 itb_d, h->prm.max_iters, s);
                launch_gs_upd(V, ldv, j, vj, w, V + (int64_t)(j + 1) * ldv, n, coef, red_upd, s, gctl);
                tend(2);
                continue;
            }
            const bool sel = j + 1 < 32;
            tbeg();
            launch_gs(0, V, ldv, j + 1, w, n, nullptr, red, hd, s, gctl, sel);
            launch_gs(1, V, ldv, j + 1, w, n, hd, red, hd + 64, s, gctl, sel);
            launch_gs(2, V, ldv, j + 1, w, n, hd + 64, red, nullptr, s, gctl, false, sel ? hd : nullptr);
            // ||w||, v_{j+1} = w / ||w||, Givens update and stopping test
            launch_step_end(red, sel ? hd : nullptr, w, V + (int64_t)(j + 1) * ldv, n, j, m, hd, R, cs, sn, g,
                            est_d, gctl, tol_d, itb_d, h->prm.max_iters, s);
            tend(2);
        }
        if (delayed) {
            // the last column made final from the last update pass's dots
            tsel = timing && tstride == 1;
            tj = m - 1;
            tbeg();
            launch_dcgs_coef(m, m, true, red_dot, red_upd, n, Hu, R, cs, sn, g, est_d, Tm, coef, gctl, tol_d,
                             itb_d, h->prm.max_iters, s);
            tend(2);
        }
        tsel = timing && tstride == 1;
        tj = -1;
        launch_trisolve(m, R, g, y, gctl, s);
        if (flex) {
            // x += Z y (delayed form: Z holds M u_j, so x += Z T^{-1} y)
            if (delayed) launch_trisolve_T(m, Tm, y, gctl, s);
            launch_gemv_small(h->Zb, ldv, gctl + 1, y, n, zt, s);
        } else {
            // x += M (V y)
            launch_gemv_small(V, ldv, gctl + 1, y, n, r, s);
            tbeg();
            PR_TRY(precond(h, r, zt, t3));
            tend(0);
        }
        launch_axpy_dev(xw, zt, 1.0, n, s);
        tbeg();
        launch_spmv_sell(h->sell(), n, xw, bw, r, s);
        tend(1);
        launch_gs(0, r, n, 1, r, n, nullptr, red, hd, s);
        return PR_OK;
    };
    if (use_graph && (!h->gexec || h->graph_m != m)) {
        if (h->gexec) {
            (void)hipGraphExecDestroy(h->gexec);
            h->gexec = nullptr;
        }
        hipGraph_t gr = nullptr;
        PR_HIP(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_cycle();
        const hipError_t ec = hipStreamEndCapture(s, &gr);
        if (rc < 0) return rc;
        if (ec != hipSuccess) return pr_fail(h, PR_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&h->gexec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ei != hipSuccess) return pr_fail(h, PR_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
        h->graph_m = m;
    }

    PR_TRY(sync_read(1));
    int64_t iters = 0, cycles = 0, reorth = 0;
    double relres = std::sqrt(hh[0]) / bnorm, est = relres;
    const int64_t maxit = h->prm.max_iters;
    for (;;) {
        if (!std::isfinite(relres)) return pr_fail(h, PR_ERR_NONFINITE, "non-finite residual");
        if (relres <= tol || iters >= maxit) break;
        ++cycles;
        *itb_h = iters;
        PR_HIP(h, hipMemcpyAsync(itb_d, itb_h, sizeof(int64_t), hipMemcpyHostToDevice, s));
        if (use_graph) PR_HIP(h, hipGraphLaunch(h->gexec, s));
        else PR_TRY(enqueue_cycle());
        // one host wait per restart cycle
        PR_HIP(h, hipMemcpyAsync(gctl_h, gctl, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipMemcpyAsync(hh + 239, est_d, sizeof(double), hipMemcpyDeviceToHost, s));
        PR_TRY(sync_read(1));
        iters += gctl_h[1];
        reorth += gctl_h[2];
        done_cols.push_back(gctl_h[1]);
        est = hh[239] / bnorm;
        relres = std::sqrt(hh[0]) / bnorm;
    }
    if (use_graph) launch_copy(x, xw, n, s);
    PR_HIP(h, hipStreamSynchronize(s));
    PR_HIP(h, hipGetLastError());
    h->sinfo.iters = iters;
    h->sinfo.cycles = cycles;
    h->sinfo.reorth = (int32_t)reorth;
    h->sinfo.relres = relres;
    h->sinfo.relres_est = est;
    h->sinfo.status = relres <= tol ? PR_OK : PR_NOT_CONVERGED;
    h->sinfo.seconds = now_s() - tstart;
    // the delayed form's end-of-cycle pass is recorded under the cycle's last
    // step: its time adds to that step's orthogonalisation, one launch
    int64_t orth_cyc = -1;
    int orth_j = -1;
    for (const Span& sp : spans) {
        float ms = 0.0f;
        if (sp.j >= 0 && (sp.cyc >= (int64_t)done_cols.size() || sp.j >= done_cols[sp.cyc])) continue;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) != hipSuccess) continue;
        if (sp.cls == 0) { h->sinfo.apply_ms += ms; h->sinfo.n_apply++; }
        if (sp.cls == 1) { h->sinfo.spmv_ms += ms; h->sinfo.n_spmv++; }
        if (sp.cls == 2) {
            h->sinfo.orth_ms += ms;
            if (sp.j < 0 || sp.cyc != orth_cyc || sp.j != orth_j) h->sinfo.n_orth++;
            orth_cyc = sp.cyc;
            orth_j = sp.j;
        }
        if (sp.cls == 3) { h->sinfo.coarse_ms += ms; h->sinfo.n_coarse++; }
    }
    return h->sinfo.status;
}

int pr_get_solve_info(pr_handle h, pr_solve_info* info) {
    if (!h || !info) return PR_ERR_INVALID_ARG;
    *info = h->sinfo;
    return PR_OK;
}

int pr_get_stats(pr_handle h, pr_stats* st) {
    if (!h || !st) return PR_ERR_INVALID_ARG;
    *st = h->stats;
    return PR_OK;
}

int pr_get_assignment(pr_handle h, int32_t* phi, int32_t* reps, int64_t* m_p) {
    if (!h) return PR_ERR_INVALID_ARG;
    PR_HIP(h, hipStreamSynchronize(h->stream));
    if (phi) PR_HIP(h, hipMemcpy(phi, h->phi, h->n_p * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (reps) std::memcpy(reps, h->reps_host.data(), h->m_p * sizeof(int32_t));
    if (m_p) *m_p = h->m_p;
    return PR_OK;
}

int pr_get_patch_tile(pr_handle h, int64_t k, double* tile) {
    if (!h || !tile || k < 0 || k >= h->n_p) return PR_ERR_INVALID_ARG;
    int64_t pp[2];
    PR_HIP(h, hipStreamSynchronize(h->stream));
    PR_HIP(h, hipMemcpy(pp, h->pptr + k, 2 * sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t p = pp[1] - pp[0];
    int64_t off = 0;
    if (h->uniform) off = k * p * p;
    else PR_HIP(h, hipMemcpy(&off, h->toff + k, sizeof(int64_t), hipMemcpyDeviceToHost));
    PR_HIP(h, hipMemcpy(tile, h->tiles + off, p * p * sizeof(double), hipMemcpyDeviceToHost));
    return PR_OK;
}

int pr_get_weights(pr_handle h, double* W) {
    if (!h || !W) return PR_ERR_INVALID_ARG;
    PR_HIP(h, hipStreamSynchronize(h->stream));
    PR_HIP(h, hipMemcpy(W, h->W, h->n * sizeof(double), hipMemcpyDeviceToHost));
    return PR_OK;
}

int pr_get_boundary_keys(pr_handle h, uint32_t* keys) {
    if (!h || !keys) return PR_ERR_INVALID_ARG;
    PR_HIP(h, hipStreamSynchronize(h->stream));
    PR_HIP(h, hipMemcpy(keys, h->keys, h->n_p * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return PR_OK;
}

int pr_get_rep_inverse(pr_handle h, int64_t j, double* X) {
    if (!h || !X || j < 0 || j >= h->m_p) return PR_ERR_INVALID_ARG;
    PR_HIP(h, hipStreamSynchronize(h->stream));
    const int64_t p = h->dbps_host[j];
    PR_HIP(h, hipMemcpy(X, h->db + h->dboff_host[j], p * p * sizeof(double), hipMemcpyDeviceToHost));
    return PR_OK;
}

int pr_get_entry_matrix(pr_handle h, int64_t j, double* B) {
    if (!h || !B || j < 0 || j >= h->m_p) return PR_ERR_INVALID_ARG;
    if (!h->db_mat) return pr_get_patch_tile(h, h->reps_host[j], B);
    PR_HIP(h, hipStreamSynchronize(h->stream));
    const int64_t p = h->dbps_host[j];
    PR_HIP(h, hipMemcpy(B, h->db_mat + h->dboff_host[j], p * p * sizeof(double), hipMemcpyDeviceToHost));
    return PR_OK;
}

int pr_batch_inverse(int32_t p, int64_t count, const double* A, double* X, int32_t* info, void* stream) {
    if (p < 1 || p > kWideMaxPs || count < 0)
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "p must be in [1, " + std::to_string(kWideMaxPs) + "]");
    if (count == 0) return PR_OK;
    int rc;
    if ((rc = check_dev(nullptr, A, "A")) < 0) return rc;
    if ((rc = check_dev(nullptr, X, "X")) < 0) return rc;
    if ((rc = check_dev(nullptr, info, "info")) < 0) return rc;
    if (p > 32) launch_gj_wide(count, nullptr, nullptr, A, nullptr, p, p, X, nullptr, info, (hipStream_t)stream);
    else launch_batch_inverse(p, count, A, nullptr, nullptr, nullptr, X, nullptr, info, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return pr_fail(nullptr, PR_ERR_HIP, hipGetErrorString(e));
    return PR_OK;
}

int pr_batch_criterion(int32_t p, int64_t count, int32_t crit, const double* A, const double* B,
                       const double* X, double* d, void* stream) {
    if (p < 1 || p > 32 || count < 0 || crit < 0 || crit > 2)
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "bad p, count or criterion");
    if (count == 0) return PR_OK;
    int rc;
    if ((rc = check_dev(nullptr, A, "A")) < 0) return rc;
    if ((rc = check_dev(nullptr, d, "d")) < 0) return rc;
    if (crit == PR_CRIT_SPECTRAL) {
        if ((rc = check_dev(nullptr, X, "X")) < 0) return rc;
    } else {
        if ((rc = check_dev(nullptr, B, "B")) < 0) return rc;
    }
    launch_batch_criterion(p, count, crit, A, B, X, d, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return pr_fail(nullptr, PR_ERR_HIP, hipGetErrorString(e));
    return PR_OK;
}

}  // extern "C"
