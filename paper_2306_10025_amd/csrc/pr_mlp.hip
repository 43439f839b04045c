// Algorithm 1 with the learned entry predictor, and the standalone MLP entry
// points of the C ABI.
//
// Setup with the predictor (params.mlp = 1, algo = PR_ALGO_TOLERANCE):
//  1. a seeded sample of the patches (partial Fisher-Yates, SplitMix64) is
//     the training set; Algorithm 1 runs on it alone and its entries are the
//     classes;
//  2. the network (features -> 2 hidden ReLU layers -> class logits) is
//     trained on the GPU on the training patches' entries, Adam on
//     minibatches, with the GEMMs in FP16 MFMA (FP32 accumulation and master
//     weights) or FP32;
//  3. every other patch takes the first of its top-k predicted entries with
//     d < eps (the exact criterion decides), else the first entry in append
//     order with d < eps, else Algorithm 1 runs on the patches left and
//     appends their entries after the training entries.
// The result is, patch for patch, the sequential procedure "Algorithm 1 on
// the training set, then each other patch in ascending id: predicted
// candidates, then the current database in append order, else append".
#include "pr_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

namespace {

struct MlpDims {
    int F = 0, H = 0, C = 0;
    int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0, n = 0;
    MlpDims(int F_, int H_, int C_) : F(F_), H(H_), C(C_) {
        oW1 = 0;
        ob1 = oW1 + (int64_t)F * H;
        oW2 = ob1 + H;
        ob2 = oW2 + (int64_t)H * H;
        oW3 = ob2 + H;
        ob3 = oW3 + (int64_t)H * C;
        n = ob3 + C;
    }
};

struct MlpWork {
    float *H1 = nullptr, *H2 = nullptr, *L = nullptr, *G3 = nullptr, *G2 = nullptr, *G1 = nullptr;
    double* loss_rows = nullptr;
};

// activations for B rows: H1, H2 (B x H), logits L (B x C)
void mlp_forward(int prec, const MlpDims& d, const float* P, const float* X, int B, MlpWork& w, hipStream_t s) {
    launch_gemm(prec, false, false, B, d.H, d.F, X, d.F, P + d.oW1, d.H, w.H1, d.H, 1.0f, P + d.ob1, 1, nullptr, 0,
                s);
    launch_gemm(prec, false, false, B, d.H, d.H, w.H1, d.H, P + d.oW2, d.H, w.H2, d.H, 1.0f, P + d.ob2, 1, nullptr,
                0, s);
    launch_gemm(prec, false, false, B, d.C, d.H, w.H2, d.H, P + d.oW3, d.C, w.L, d.C, 1.0f, P + d.ob3, 0, nullptr,
                0, s);
}

// Backpropagated signals are carried times kGradScale (a power of two, so
// the scaling is exact) and the weight gradients are scaled back at the end:
// the FP16 operands then stay clear of the subnormal range (loss scaling).
constexpr float kGradScale = 1024.0f;

// mean cross-entropy gradient for every parameter (after mlp_forward)
void mlp_backward(int prec, const MlpDims& d, const float* P, const float* X, const int32_t* y,
                  const int32_t* rkey, const int32_t* ckey, int B, MlpWork& w, float* G, hipStream_t s) {
    const float un = 1.0f / kGradScale;
    launch_softmax_ce(B, d.C, w.L, d.C, y, rkey, ckey, w.G3, d.C, w.loss_rows, kGradScale / (float)B, s);
    launch_gemm(prec, true, false, d.H, d.C, B, w.H2, d.H, w.G3, d.C, G + d.oW3, d.C, un, nullptr, 0, nullptr, 0, s);
    launch_colsum(B, d.C, w.G3, d.C, un, G + d.ob3, s);
    launch_gemm(prec, false, true, B, d.H, d.C, w.G3, d.C, P + d.oW3, d.C, w.G2, d.H, 1.0f, nullptr, 0, w.H2, d.H, s);
    launch_gemm(prec, true, false, d.H, d.H, B, w.H1, d.H, w.G2, d.H, G + d.oW2, d.H, un, nullptr, 0, nullptr, 0, s);
    launch_colsum(B, d.H, w.G2, d.H, un, G + d.ob2, s);
    launch_gemm(prec, false, true, B, d.H, d.H, w.G2, d.H, P + d.oW2, d.H, w.G1, d.H, 1.0f, nullptr, 0, w.H1, d.H, s);
    launch_gemm(prec, true, false, d.F, d.H, B, X, d.F, w.G1, d.H, G + d.oW1, d.H, un, nullptr, 0, nullptr, 0, s);
    launch_colsum(B, d.H, w.G1, d.H, un, G + d.ob1, s);
}

uint64_t sm64(uint64_t& st) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// first m of a partial Fisher-Yates shuffle of 0..L-1: position i swaps with
// i + (u mod (L - i))
std::vector<int32_t> fisher_yates_prefix(int64_t L, int64_t m, uint64_t& st) {
    std::unordered_map<int64_t, int64_t> moved;
    auto at = [&](int64_t x) {
        auto it = moved.find(x);
        return it == moved.end() ? x : it->second;
    };
    std::vector<int32_t> out(m);
    for (int64_t i = 0; i < m; ++i) {
        const uint64_t u = sm64(st);
        const int64_t j = i + (int64_t)(u % (uint64_t)(L - i));
        const int64_t vi = at(i), vj = at(j);
        moved[i] = vj;
        moved[j] = vi;
        out[i] = (int32_t)vj;
    }
    return out;
}

int compact(pr_handle h, int64_t n, const int32_t* ids, const int32_t* keep, int want, int32_t* out,
            int64_t* f, int64_t* pos, int64_t* scr, int64_t& count) {
    hipStream_t s = h->stream;
    launch_compact_flags(n, keep, want, f, s);
    launch_exclusive_scan_i64(f, pos, n + 1, scr, s);
    launch_compact(n, ids, f, pos, out, s);
    PR_HIP(h, hipMemcpyAsync(&count, pos + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    return PR_OK;
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct SeedResult {
    int64_t evals = 0, exact = 0, refined = 0, rounds = 0;
    int64_t accepted = 0, scanned = 0, fallback = 0;   // matched a candidate / the scan / neither
};

// Algorithm 1 seeded with n0 entries (entries[0..n0), patch ids): every
// query patch Q[q] tries its k candidate entries cand[q*k..] in order (none
// when cand is null), then scans the seed entries in append order, and the
// patches still unmatched run Algorithm 1 among themselves, their entries
// appended after the seed.  rank_of_patch and repof hold the seed entries on
// entry (rank_of_patch[e] = j, repof[e] = e for seed entry e).  Sets h->phi,
// h->reps, h->m_p, the FP64 database and the entry sizes and offsets.
int alg1_from_seed(pr_handle h, int32_t* entries, int64_t n0, int32_t* rank_of_patch, int32_t* repof,
                   const int32_t* Q, int64_t nq, const int32_t* cand, int k, SeedResult& out) {
    hipStream_t s = h->stream;
    const pr_params& pm = h->prm;
    const int64_t n_p = h->n_p;
    const int64_t stride = (int64_t)h->max_ps * h->max_ps;
    const int ups = h->uniform ? h->max_ps : 0;
    const int64_t* toff = h->uniform ? nullptr : h->toff;
    const int crit = pm.criterion;
    const double* keynorm = (crit == PR_CRIT_L1) ? h->l1norm : h->fnorm;
    int32_t* csize = nullptr;
    PR_TRY(dalloc(h, &csize, std::max<int64_t>(1, n0)));
    launch_sizes(n0, entries, h->pptr, csize, s);
    int64_t *f = nullptr, *pos = nullptr, *scr = nullptr;
    PR_TRY(dalloc(h, &f, n_p + 1));
    PR_TRY(dalloc(h, &pos, n_p + 1));
    PR_TRY(dalloc(h, &scr, scan_scratch_elems(n_p + 1) + 2));
    double *Bm = nullptr, *X0 = nullptr;
    int32_t* info = nullptr;
    int64_t *csz = nullptr, *coff = nullptr;
    PR_TRY(dalloc(h, &Bm, (size_t)n0 * stride));
    PR_TRY(dalloc(h, &X0, (size_t)n0 * stride));
    PR_TRY(dalloc(h, &info, n_p));
    std::vector<int32_t> csize_h(n0);
    PR_HIP(h, hipMemcpyAsync(csize_h.data(), csize, n0 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    auto invert = [&](int64_t m, const int32_t* ents, const std::vector<int32_t>& sz, double* dst) -> int {
        launch_km_init(m, ents, h->pptr, h->tiles, toff, ups, Bm, stride, s);
        if (!h->uniform) {
            std::vector<int64_t> a(m + 1), o(m + 1);
            a[0] = 0;
            for (int64_t j = 0; j < m; ++j) {
                a[j + 1] = a[j] + sz[j];
                o[j] = j * stride;
            }
            o[m] = m * stride;
            PR_TRY(dalloc(h, &csz, m + 1));
            PR_TRY(dalloc(h, &coff, m + 1));
            PR_HIP(h, hipMemcpyAsync(csz, a.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
            PR_HIP(h, hipMemcpyAsync(coff, o.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        }
        launch_batch_inverse(h->max_ps, m, Bm, h->uniform ? nullptr : coff, nullptr, h->uniform ? nullptr : csz,
                             dst, h->uniform ? nullptr : coff, info, s);
        std::vector<int32_t> info_h(m);
        PR_HIP(h, hipMemcpyAsync(info_h.data(), info, m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        for (int64_t j = 0; j < m; ++j)
            if (info_h[j] != 0)
                return pr_fail(h, PR_ERR_SINGULAR_PATCH, "zero pivot in database entry " + std::to_string(j));
        return PR_OK;
    };
    PR_TRY(invert(n0, entries, csize_h, X0));
    int32_t *res1 = nullptr, *U = nullptr, *res2 = nullptr, *V = nullptr;
    unsigned long long* cnt = nullptr;
    PR_TRY(dalloc(h, &res1, std::max<int64_t>(1, nq)));
    PR_TRY(dalloc(h, &U, std::max<int64_t>(1, nq)));
    PR_TRY(dalloc(h, &res2, std::max<int64_t>(1, nq)));
    PR_TRY(dalloc(h, &V, std::max<int64_t>(1, nq)));
    PR_TRY(dalloc(h, &cnt, 4));
    PR_HIP(h, hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), s));
    int64_t nu = 0, nv = 0;
    if (cand && k > 0) {
        launch_mlp_match(0, nq, Q, cand, k, h->pptr, h->tiles, toff, ups, entries, n0, X0, stride, crit, pm.eps,
                         keynorm, repof, res1, cnt, s);
        PR_TRY(compact(h, nq, Q, res1, 0, U, f, pos, scr, nu));
    } else {
        nu = nq;
        if (nq > 0) PR_HIP(h, hipMemcpyAsync(U, Q, nq * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    launch_mlp_match(1, nu, U, nullptr, 0, h->pptr, h->tiles, toff, ups, entries, n0, X0, stride, crit, pm.eps,
                     keynorm, repof, res2, cnt, s);
    PR_TRY(compact(h, nu, U, res2, 0, V, f, pos, scr, nv));
    int64_t n1 = 0;
    A1Run R1;
    if (nv > 0) {
        PR_TRY(alg1_core(h, V, nv, R1));
        n1 = R1.m;
        launch_a1_subset_entries(nv, V, R1.repof, R1.flag, R1.excl, R1.scr, (int32_t)n0, entries + n0,
                                 rank_of_patch, s);
        launch_copy_at(nv, V, R1.repof, repof, s);
    }

    // 6. phi, the database and the statistics
    const int64_t m_p = n0 + n1;
    PR_TRY(dalloc(h, &h->phi, n_p));
    launch_map_at(n_p, nullptr, repof, rank_of_patch, h->phi, s);
    h->m_p = m_p;
    h->reps = entries;
    h->reps_host.resize(m_p);
    PR_HIP(h, hipMemcpyAsync(h->reps_host.data(), entries, m_p * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    std::vector<int64_t> pptr_h(n_p + 1);
    PR_HIP(h, hipMemcpyAsync(pptr_h.data(), h->pptr, (n_p + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    unsigned long long c4[4];
    PR_HIP(h, hipMemcpyAsync(c4, cnt, sizeof(c4), hipMemcpyDeviceToHost, s));
    PR_HIP(h, hipStreamSynchronize(s));
    h->dbps_host.resize(m_p);
    h->dboff_host.resize(m_p + 1);
    for (int64_t j = 0; j < m_p; ++j) {
        const int32_t r = h->reps_host[j];
        h->dbps_host[j] = (int32_t)(pptr_h[r + 1] - pptr_h[r]);
        h->dboff_host[j] = j * stride;
    }
    h->dboff_host[m_p] = m_p * stride;
    PR_TRY(dalloc(h, &Bm, (size_t)m_p * stride));     // room for every entry
    PR_TRY(dalloc(h, &h->db, (size_t)m_p * stride));
    PR_TRY(invert(m_p, entries, h->dbps_host, h->db));

    out.evals = (int64_t)(c4[0] + R1.cnt[0]);
    out.exact = (int64_t)(c4[1] + R1.cnt[1]);
    out.refined = (int64_t)(c4[3] + R1.cnt[3]);
    out.rounds = R1.rounds;
    out.accepted = nq - nu;
    out.scanned = nu - nv;
    out.fallback = nv;
    return PR_OK;
}

int run_alg1_mlp(pr_handle h) {
    hipStream_t s = h->stream;
    const pr_params& pm = h->prm;
    const int64_t n_p = h->n_p;
    const int64_t stride = (int64_t)h->max_ps * h->max_ps;
    const int ups = h->uniform ? h->max_ps : 0;
    const int64_t* toff = h->uniform ? nullptr : h->toff;
    const int crit = pm.criterion;
    const double* keynorm = (crit == PR_CRIT_L1) ? h->l1norm : h->fnorm;
    const int prec = pm.mlp_precision;
    const int k = pm.mlp_topk;

    // 1. training sample and Algorithm 1 on it
    int64_t ns = (int64_t)std::llround(pm.mlp_train_frac * (double)n_p);
    ns = std::max<int64_t>(1, std::min<int64_t>(ns, n_p));
    uint64_t st = pm.mlp_seed;
    std::vector<int32_t> train_h = fisher_yates_prefix(n_p, ns, st);
    std::sort(train_h.begin(), train_h.end());
    int32_t* train = nullptr;
    PR_TRY(dalloc(h, &train, ns));
    PR_HIP(h, hipMemcpyAsync(train, train_h.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
    A1Run R0;
    PR_TRY(alg1_core(h, train, ns, R0));
    const int64_t n0 = R0.m;
    int32_t *entries = nullptr, *rank_of_patch = nullptr, *repof = nullptr, *ytr = nullptr, *psize = nullptr;
    int32_t* csize = nullptr;
    PR_TRY(dalloc(h, &entries, n_p));
    PR_TRY(dalloc(h, &rank_of_patch, n_p));
    PR_TRY(dalloc(h, &repof, n_p));
    PR_TRY(dalloc(h, &ytr, ns));
    PR_TRY(dalloc(h, &psize, n_p));
    PR_TRY(dalloc(h, &csize, n0));
    launch_fill_i32(rank_of_patch, n_p, -1, s);
    launch_fill_i32(repof, n_p, -1, s);
    launch_a1_subset_entries(ns, train, R0.repof, R0.flag, R0.excl, R0.scr, 0, entries, rank_of_patch, s);
    launch_copy_at(ns, train, R0.repof, repof, s);
    launch_map_at(ns, train, R0.repof, rank_of_patch, ytr, s);
    launch_sizes(n_p, nullptr, h->pptr, psize, s);
    launch_sizes(n0, entries, h->pptr, csize, s);
    const int32_t* rkey_all = h->uniform ? nullptr : psize;
    const int32_t* ckey = h->uniform ? nullptr : csize;

    // 2. features, standardised on the training rows
    const double t_train0 = now_s();
    const int pmax = h->max_ps;
    const int F = 3 * pmax + 1, H = pm.mlp_hidden;
    const int C = (int)n0;
    MlpDims dm(F, H, C);
    float *Xall = nullptr, *mu = nullptr, *sd = nullptr, *Xtr = nullptr;
    int32_t* ktr = nullptr;
    PR_TRY(dalloc(h, &Xall, (size_t)n_p * F));
    PR_TRY(dalloc(h, &mu, F));
    PR_TRY(dalloc(h, &sd, F));
    PR_TRY(dalloc(h, &Xtr, (size_t)ns * F));
    PR_TRY(dalloc(h, &ktr, ns));
    launch_mlp_features(n_p, h->pptr, h->tiles, toff, ups, h->keys, pmax, Xall, s);
    launch_mlp_moments(ns, train, Xall, F, mu, sd, s);
    launch_mlp_gather(ns, train, Xall, F, mu, sd, Xtr, nullptr, nullptr, psize, ktr, s);

    // parameters: He-uniform weights from the SplitMix64 stream, zero biases
    float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vv = nullptr;
    PR_TRY(dalloc(h, &P, dm.n));
    PR_TRY(dalloc(h, &G, dm.n));
    PR_TRY(dalloc(h, &Mo, dm.n));
    PR_TRY(dalloc(h, &Vv, dm.n));
    PR_HIP(h, hipMemsetAsync(P, 0, dm.n * sizeof(float), s));
    PR_HIP(h, hipMemsetAsync(Mo, 0, dm.n * sizeof(float), s));
    PR_HIP(h, hipMemsetAsync(Vv, 0, dm.n * sizeof(float), s));
    launch_init_uniform((int64_t)F * H, P + dm.oW1, (float)std::sqrt(6.0 / F), pm.mlp_seed, 0, s);
    launch_init_uniform((int64_t)H * H, P + dm.oW2, (float)std::sqrt(6.0 / H), pm.mlp_seed, (uint64_t)F * H, s);
    launch_init_uniform((int64_t)H * C, P + dm.oW3, (float)std::sqrt(6.0 / H), pm.mlp_seed,
                        (uint64_t)F * H + (uint64_t)H * H, s);

    // 3. training: Adam on shuffled minibatches
    const int Bt = (int)std::min<int64_t>(pm.mlp_batch, ns);
    const int64_t Bw = std::max<int64_t>(Bt, 8192);        // rows of the work buffers (inference chunks)
    MlpWork w;
    PR_TRY(dalloc(h, &w.H1, (size_t)Bw * H));
    PR_TRY(dalloc(h, &w.H2, (size_t)Bw * H));
    PR_TRY(dalloc(h, &w.L, (size_t)Bw * C));
    PR_TRY(dalloc(h, &w.G3, (size_t)Bt * C));
    PR_TRY(dalloc(h, &w.G2, (size_t)Bt * H));
    PR_TRY(dalloc(h, &w.G1, (size_t)Bt * H));
    PR_TRY(dalloc(h, &w.loss_rows, Bw));
    float* Xb = nullptr;
    int32_t *yb = nullptr, *kb = nullptr, *perm = nullptr;
    PR_TRY(dalloc(h, &Xb, (size_t)Bt * F));
    PR_TRY(dalloc(h, &yb, Bt));
    PR_TRY(dalloc(h, &kb, Bt));
    PR_TRY(dalloc(h, &perm, ns));
    int64_t tstep = 0;
    for (int e = 0; e < pm.mlp_epochs; ++e) {
        std::vector<int32_t> perm_h = fisher_yates_prefix(ns, ns, st);
        PR_HIP(h, hipMemcpyAsync(perm, perm_h.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
        for (int64_t b0 = 0; b0 < ns; b0 += Bt) {
            const int bs = (int)std::min<int64_t>(Bt, ns - b0);
            launch_rows_gather(bs, perm + b0, Xtr, F, Xb, ytr, yb, ktr, rkey_all ? kb : nullptr, s);
            mlp_forward(prec, dm, P, Xb, bs, w, s);
            mlp_backward(prec, dm, P, Xb, yb, rkey_all ? kb : nullptr, ckey, bs, w, G, s);
            ++tstep;
            const float bc1 = (float)(1.0 - std::pow(0.9, (double)tstep));
            const float bc2 = (float)(1.0 - std::pow(0.999, (double)tstep));
            launch_adam(dm.n, P, G, Mo, Vv, (float)pm.mlp_lr, 0.9f, 0.999f, 1e-8f, bc1, bc2, s);
        }
        PR_HIP(h, hipStreamSynchronize(s));     // one epoch in flight at a time
    }
    // loss and top-1 accuracy on the whole training set
    double loss_sum = 0.0;
    unsigned long long* acc_cnt = nullptr;
    int32_t* top1 = nullptr;
    PR_TRY(dalloc(h, &acc_cnt, 1));
    PR_TRY(dalloc(h, &top1, Bw));
    PR_HIP(h, hipMemsetAsync(acc_cnt, 0, sizeof(unsigned long long), s));
    std::vector<double> lr_h(Bw);
    for (int64_t b0 = 0; b0 < ns; b0 += Bw) {
        const int bs = (int)std::min<int64_t>(Bw, ns - b0);
        mlp_forward(prec, dm, P, Xtr + b0 * F, bs, w, s);
        launch_softmax_ce(bs, C, w.L, C, ytr + b0, rkey_all ? ktr + b0 : nullptr, ckey, nullptr, C, w.loss_rows,
                          1.0f, s);
        launch_topk(bs, C, w.L, C, 1, rkey_all ? ktr + b0 : nullptr, ckey, top1, s);
        launch_count_eq(bs, top1, 1, ytr + b0, acc_cnt, s);
        PR_HIP(h, hipMemcpyAsync(lr_h.data(), w.loss_rows, bs * sizeof(double), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        for (int r = 0; r < bs; ++r) loss_sum += lr_h[r];
    }
    unsigned long long acc_h = 0;
    PR_HIP(h, hipMemcpy(&acc_h, acc_cnt, sizeof(acc_h), hipMemcpyDeviceToHost));
    const double t_train1 = now_s();

    // 4. predictions for the other patches
    int32_t *mark = nullptr, *all_ids = nullptr, *Q = nullptr, *cand = nullptr;
    int64_t *f = nullptr, *pos = nullptr, *scr = nullptr;
    PR_TRY(dalloc(h, &mark, n_p));
    PR_TRY(dalloc(h, &all_ids, n_p));
    PR_TRY(dalloc(h, &Q, n_p));
    PR_TRY(dalloc(h, &f, n_p + 1));
    PR_TRY(dalloc(h, &pos, n_p + 1));
    PR_TRY(dalloc(h, &scr, scan_scratch_elems(n_p + 1) + 2));
    launch_fill_i32(mark, n_p, 0, s);
    launch_set_at(ns, train, 1, mark, s);
    launch_iota(all_ids, n_p, s);
    int64_t nq = 0;
    PR_TRY(compact(h, n_p, all_ids, mark, 0, Q, f, pos, scr, nq));
    PR_TRY(dalloc(h, &cand, std::max<int64_t>(1, nq) * k));
    float* Xq = nullptr;
    int32_t* kq = nullptr;
    PR_TRY(dalloc(h, &Xq, (size_t)Bw * F));
    PR_TRY(dalloc(h, &kq, Bw));
    for (int64_t b0 = 0; b0 < nq; b0 += Bw) {
        const int bs = (int)std::min<int64_t>(Bw, nq - b0);
        launch_mlp_gather(bs, Q + b0, Xall, F, mu, sd, Xq, nullptr, nullptr, psize, kq, s);
        mlp_forward(prec, dm, P, Xq, bs, w, s);
        launch_topk(bs, C, w.L, C, k, rkey_all ? kq : nullptr, ckey, cand + b0 * k, s);
    }

    // 5. the exact criterion decides: predicted candidates, then the scan,
    // then Algorithm 1 on the patches no entry matched
    SeedResult sr;
    PR_TRY(alg1_from_seed(h, entries, n0, rank_of_patch, repof, Q, nq, cand, k, sr));

    h->mlp_X = Xall;
    h->mlp_F = F;
    h->mlp_train = train;
    h->mlp_ns = ns;
    h->mlp_q = Q;
    h->mlp_nq = nq;
    h->mlp_cand = cand;
    h->mlp_k = k;
    h->stats.crit_evals = (int64_t)R0.cnt[0] + sr.evals;
    h->stats.crit_exact = (int64_t)R0.cnt[1] + sr.exact;
    h->stats.crit_refined = (int64_t)R0.cnt[3] + sr.refined;
    h->stats.crit_pruned = 0;
    h->stats.alg1_rounds = R0.rounds + sr.rounds;
    h->stats.mlp_train = ns;
    h->stats.mlp_classes = n0;
    h->stats.mlp_accepted = sr.accepted;
    h->stats.mlp_scanned = sr.scanned;
    h->stats.mlp_fallback = sr.fallback;
    h->stats.mlp_loss = loss_sum / (double)ns;
    h->stats.mlp_train_acc = (double)acc_h / (double)ns;
    h->stats.t_mlp_train = t_train1 - t_train0;
    return PR_OK;
}


// Algorithm 1 seeded with the previous system's database (pr_setup_reuse):
// the previous entries come first; every other patch tries its previous
// entry, then the in-order scan, then Algorithm 1 on the patches left.
int run_alg1_reuse(pr_handle h) {
    hipStream_t s = h->stream;
    const int64_t n_p = h->n_p;
    const int64_t n0 = (int64_t)h->reuse_reps.size();
    std::vector<int32_t> rank_h(n_p, -1), repof_h(n_p, -1), q_h, cand_h;
    for (int64_t j = 0; j < n0; ++j) {
        const int32_t r = h->reuse_reps[j];
        rank_h[r] = (int32_t)j;
        repof_h[r] = r;
    }
    q_h.reserve(n_p - n0);
    cand_h.reserve(n_p - n0);
    for (int64_t i = 0; i < n_p; ++i)
        if (repof_h[i] < 0) {
            q_h.push_back((int32_t)i);
            cand_h.push_back(h->reuse_phi[i]);
        }
    const int64_t nq = (int64_t)q_h.size();
    int32_t *entries = nullptr, *rank_of_patch = nullptr, *repof = nullptr, *Q = nullptr, *cand = nullptr;
    PR_TRY(dalloc(h, &entries, n_p));
    PR_TRY(dalloc(h, &rank_of_patch, n_p));
    PR_TRY(dalloc(h, &repof, n_p));
    PR_TRY(dalloc(h, &Q, std::max<int64_t>(1, nq)));
    PR_TRY(dalloc(h, &cand, std::max<int64_t>(1, nq)));
    PR_HIP(h, hipMemcpyAsync(entries, h->reuse_reps.data(), n0 * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PR_HIP(h, hipMemcpyAsync(rank_of_patch, rank_h.data(), n_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PR_HIP(h, hipMemcpyAsync(repof, repof_h.data(), n_p * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (nq > 0) {
        PR_HIP(h, hipMemcpyAsync(Q, q_h.data(), nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PR_HIP(h, hipMemcpyAsync(cand, cand_h.data(), nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    SeedResult sr;
    PR_TRY(alg1_from_seed(h, entries, n0, rank_of_patch, repof, Q, nq, cand, 1, sr));
    h->stats.crit_evals = sr.evals;
    h->stats.crit_exact = sr.exact;
    h->stats.crit_refined = sr.refined;
    h->stats.crit_pruned = 0;
    h->stats.alg1_rounds = sr.rounds;
    h->stats.reuse_kept = sr.accepted;
    h->stats.reuse_rescanned = sr.scanned;
    h->stats.reuse_appended = h->m_p - n0;
    return PR_OK;
}

// ---------------------------------------------------------------------------
// standalone entry points
// ---------------------------------------------------------------------------
namespace {

bool on_device(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

struct RawBufs {
    std::vector<void*> p;
    ~RawBufs() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    bool get(T** out, size_t n) {
        if (n == 0) n = 1;
        if (hipMalloc((void**)out, n * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        p.push_back(*out);
        return true;
    }
};

int check_mlp_args(int32_t precision, int64_t rows, int32_t F, int32_t H, int32_t C) {
    if ((precision != PR_FP32 && precision != PR_FP16) || rows < 1 || rows > (1 << 24) || F < 1 || H < 1 ||
        C < 1 || F > 4096 || H > 4096 || C > (1 << 20))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "bad MLP sizes or precision");
    return PR_OK;
}

}  // namespace

int pr_mlp_loss_grad(int32_t precision, int64_t rows, int32_t F, int32_t H, int32_t C, const float* X,
                     const int32_t* y, const int32_t* row_key, const int32_t* class_key, const float* params,
                     float* grads, double* loss, void* stream) {
    int rc = check_mlp_args(precision, rows, F, H, C);
    if (rc < 0) return rc;
    if (!loss) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "loss is null");
    for (const void* q : {(const void*)X, (const void*)y, (const void*)params, (const void*)grads})
        if (!on_device(q)) return pr_fail(nullptr, q ? PR_ERR_HOST_POINTER : PR_ERR_INVALID_ARG,
                                          "X, y, params and grads must be device memory");
    if ((row_key == nullptr) != (class_key == nullptr) || (row_key && (!on_device(row_key) || !on_device(class_key))))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "row_key and class_key: both device arrays or both null");
    hipStream_t s = (hipStream_t)stream;
    MlpDims d(F, H, C);
    RawBufs rb;
    MlpWork w;
    if (!rb.get(&w.H1, (size_t)rows * H) || !rb.get(&w.H2, (size_t)rows * H) || !rb.get(&w.L, (size_t)rows * C) ||
        !rb.get(&w.G3, (size_t)rows * C) || !rb.get(&w.G2, (size_t)rows * H) || !rb.get(&w.G1, (size_t)rows * H) ||
        !rb.get(&w.loss_rows, rows))
        return pr_fail(nullptr, PR_ERR_OOM, "MLP work buffers");
    mlp_forward(precision, d, params, X, (int)rows, w, s);
    mlp_backward(precision, d, params, X, y, row_key, class_key, (int)rows, w, grads, s);
    std::vector<double> lr((size_t)rows);
    if (hipMemcpyAsync(lr.data(), w.loss_rows, rows * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return pr_fail(nullptr, PR_ERR_HIP, "MLP loss copy");
    double sum = 0.0;
    for (double v : lr) sum += v;
    *loss = sum / (double)rows;
    return PR_OK;
}

int pr_mlp_predict(int32_t precision, int64_t rows, int32_t F, int32_t H, int32_t C, const float* X,
                   const int32_t* row_key, const int32_t* class_key, const float* params, int32_t k,
                   float* logits, int32_t* topk, void* stream) {
    int rc = check_mlp_args(precision, rows, F, H, C);
    if (rc < 0) return rc;
    if (k < 0 || k > 8 || k > C || (k > 0 && !topk)) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "k must lie in [0, min(8, C)]");
    for (const void* q : {(const void*)X, (const void*)params})
        if (!on_device(q)) return pr_fail(nullptr, q ? PR_ERR_HOST_POINTER : PR_ERR_INVALID_ARG,
                                          "X and params must be device memory");
    if ((logits && !on_device(logits)) || (topk && !on_device(topk)))
        return pr_fail(nullptr, PR_ERR_HOST_POINTER, "logits and topk must be device memory");
    if ((row_key == nullptr) != (class_key == nullptr) || (row_key && (!on_device(row_key) || !on_device(class_key))))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "row_key and class_key: both device arrays or both null");
    hipStream_t s = (hipStream_t)stream;
    MlpDims d(F, H, C);
    RawBufs rb;
    MlpWork w;
    if (!rb.get(&w.H1, (size_t)rows * H) || !rb.get(&w.H2, (size_t)rows * H))
        return pr_fail(nullptr, PR_ERR_OOM, "MLP work buffers");
    if (logits) w.L = logits;
    else if (!rb.get(&w.L, (size_t)rows * C)) return pr_fail(nullptr, PR_ERR_OOM, "MLP work buffers");
    mlp_forward(precision, d, params, X, (int)rows, w, s);
    if (k > 0) launch_topk(rows, C, w.L, C, k, row_key, class_key, topk, s);
    if (hipStreamSynchronize(s) != hipSuccess) return pr_fail(nullptr, PR_ERR_HIP, "MLP predict");
    return PR_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free forward pass: the activations live in one fixed device
// array instead of buffers from hipMalloc.  Each device that runs the library
// holds its own copy of the array until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); it looks up the device address once per device and uses that.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kScratchFloats = PR_MLP_NOALLOC_SCRATCH_BYTES / (int64_t)sizeof(float);
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (looked up on first use)
int scratch_for_current_device(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pr_fail(nullptr, PR_ERR_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return pr_fail(nullptr, PR_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return pr_fail(nullptr, PR_ERR_HIP,
                           std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (float*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return PR_OK;
}

int64_t round_up_64(int64_t v) { return (v + 63) / 64 * 64; }

}  // namespace

int pr_mlp_predict_noalloc(int32_t precision, int64_t rows, int32_t F, int32_t H, int32_t C, const float* X,
                           const int32_t* row_key, const int32_t* class_key, const float* params, int32_t k,
                           float* logits, int32_t* topk, void* stream) {
    int rc = check_mlp_args(precision, rows, F, H, C);
    if (rc < 0) return rc;
    if (k < 0 || k > 8 || k > C || (k > 0 && !topk)) return pr_fail(nullptr, PR_ERR_INVALID_ARG, "k must lie in [0, min(8, C)]");
    for (const void* q : {(const void*)X, (const void*)params})
        if (!on_device(q)) return pr_fail(nullptr, q ? PR_ERR_HOST_POINTER : PR_ERR_INVALID_ARG,
                                          "X and params must be device memory");
    if ((logits && !on_device(logits)) || (topk && !on_device(topk)))
        return pr_fail(nullptr, PR_ERR_HOST_POINTER, "logits and topk must be device memory");
    if ((row_key == nullptr) != (class_key == nullptr) || (row_key && (!on_device(row_key) || !on_device(class_key))))
        return pr_fail(nullptr, PR_ERR_INVALID_ARG, "row_key and class_key: both device arrays or both null");
    // workspace: H1 and H2 (rows x H each), then the logits unless the caller gives them
    const int64_t nh = round_up_64(rows * (int64_t)H);
    const int64_t need = 2 * nh + (logits ? 0 : round_up_64(rows * (int64_t)C));
    if (need > kScratchFloats)
        return pr_fail(nullptr, PR_ERR_INVALID_ARG,
                       "rows x (2 H + C without logits) needs " + std::to_string(need * 4) +
                           " bytes of workspace, more than PR_MLP_NOALLOC_SCRATCH_BYTES");
    float* ws = nullptr;
    if ((rc = scratch_for_current_device(&ws)) < 0) return rc;
    hipStream_t s = (hipStream_t)stream;
    MlpDims d(F, H, C);
    MlpWork w;
    w.H1 = ws;
    w.H2 = ws + nh;
    w.L = logits ? logits : ws + 2 * nh;
    mlp_forward(precision, d, params, X, (int)rows, w, s);
    if (k > 0) launch_topk(rows, C, w.L, C, k, row_key, class_key, topk, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return pr_fail(nullptr, PR_ERR_HIP, hipGetErrorString(e));
    return PR_OK;
}

int pr_get_mlp_features(pr_handle h, float* X, int32_t* F) {
    if (!h || !h->mlp_X) return pr_fail(h, PR_ERR_INVALID_ARG, "no predictor in this handle");
    if (F) *F = h->mlp_F;
    if (X) {
        PR_HIP(h, hipStreamSynchronize(h->stream));
        PR_HIP(h, hipMemcpy(X, h->mlp_X, (size_t)h->n_p * h->mlp_F * sizeof(float), hipMemcpyDeviceToHost));
    }
    return PR_OK;
}

int pr_get_mlp_candidates(pr_handle h, int32_t* train, int32_t* cand) {
    if (!h || !h->mlp_cand) return pr_fail(h, PR_ERR_INVALID_ARG, "no predictor in this handle");
    PR_HIP(h, hipStreamSynchronize(h->stream));
    if (train) PR_HIP(h, hipMemcpy(train, h->mlp_train, h->mlp_ns * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (cand) {
        std::vector<int32_t> q(h->mlp_nq), c((size_t)h->mlp_nq * h->mlp_k);
        if (h->mlp_nq > 0) {
            PR_HIP(h, hipMemcpy(q.data(), h->mlp_q, h->mlp_nq * sizeof(int32_t), hipMemcpyDeviceToHost));
            PR_HIP(h, hipMemcpy(c.data(), h->mlp_cand, c.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        }
        for (int64_t i = 0; i < h->n_p * h->mlp_k; ++i) cand[i] = -1;
        for (int64_t t = 0; t < h->mlp_nq; ++t)
            for (int j = 0; j < h->mlp_k; ++j) cand[(int64_t)q[t] * h->mlp_k + j] = c[(size_t)t * h->mlp_k + j];
    }
    return PR_OK;
}
