// Independent systems in one handle (a block-diagonal A, e.g. an uneven
// batch of small problems): pr_set_systems records the row ranges, and
// pr_solve then runs one right-preconditioned GMRES per system, each with
// its own Krylov space, Hessenberg matrix, rotations and stopping test on
// its own right-hand side; converged systems are masked while the others
// continue, and every launch serves all systems at once.
#include "pr_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace {

constexpr int64_t kChunk = 2048;   // rows per reduction chunk (chunks never straddle systems)

// flag[0]: a CSR entry couples two systems; flag[1]: a patch spans two systems
__global__ void k_check_systems(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                int64_t n_p, const int64_t* __restrict__ pptr, const int32_t* __restrict__ dofs,
                                const int64_t* __restrict__ sptr, int nsys, int32_t* __restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    auto sys_of = [&](int64_t i) {
        int lo = 0, hi = nsys - 1;          // last system whose start <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (sptr[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    if (t < n) {
        const int s = sys_of(t);
        for (int64_t q = rowptr[t]; q < rowptr[t + 1]; ++q)
            if (col[q] < sptr[s] || col[q] >= sptr[s + 1]) flag[0] = 1;
    }
    if (t < n_p) {
        const int s = sys_of(dofs[pptr[t]]);
        for (int64_t q = pptr[t]; q < pptr[t + 1]; ++q)
            if (dofs[q] < sptr[s] || dofs[q] >= sptr[s + 1]) flag[1] = 1;
    }
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

int pr_set_systems(pr_handle h, const int64_t* sptr, int64_t nsys) {
    if (!h || !sptr || nsys < 1 || nsys > (1 << 20)) return pr_fail(h, PR_ERR_INVALID_ARG, "bad system list");
    if (sptr[0] != 0 || sptr[nsys] != h->n) return pr_fail(h, PR_ERR_INVALID_ARG, "system_ptr must run from 0 to n");
    if (h->n0 > 0) return pr_fail(h, PR_ERR_INVALID_ARG, "the handle has a coarse space; batches take none");
    if (h->wide) return pr_fail(h, PR_ERR_UNSUPPORTED, "batches of systems take patches of at most 32 dofs");
    for (int64_t s = 0; s < nsys; ++s)
        if (sptr[s + 1] <= sptr[s]) return pr_fail(h, PR_ERR_INVALID_ARG, "empty or unordered system");
    hipStream_t st = h->stream;
    // the matrix must be block diagonal and every patch inside one system
    int64_t* sptr_d = nullptr;
    int32_t* flag = nullptr;
    PR_TRY(dalloc(h, &sptr_d, nsys + 1));
    PR_TRY(dalloc(h, &flag, 2));
    PR_HIP(h, hipMemcpyAsync(sptr_d, sptr, (nsys + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    PR_HIP(h, hipMemsetAsync(flag, 0, 2 * sizeof(int32_t), st));
    const int64_t nt = std::max(h->n, h->n_p);
    k_check_systems<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(h->n, h->rowptr, h->col, h->n_p, h->pptr,
                                                                  h->pdofs, sptr_d, (int)nsys, flag);
    int32_t fl[2] = {0, 0};
    PR_HIP(h, hipMemcpyAsync(fl, flag, sizeof(fl), hipMemcpyDeviceToHost, st));
    PR_HIP(h, hipStreamSynchronize(st));
    PR_HIP(h, hipGetLastError());
    if (fl[0]) return pr_fail(h, PR_ERR_INVALID_ARG, "the matrix couples two systems");
    if (fl[1]) return pr_fail(h, PR_ERR_INVALID_ARG, "a patch spans two systems");
    // reduction chunks
    std::vector<int32_t> ch_sys, ch_len, sys_ch0(nsys), sys_nch(nsys);
    std::vector<int64_t> ch_lo;
    for (int64_t s = 0; s < nsys; ++s) {
        sys_ch0[s] = (int32_t)ch_sys.size();
        for (int64_t lo = sptr[s]; lo < sptr[s + 1]; lo += kChunk) {
            ch_sys.push_back((int32_t)s);
            ch_lo.push_back(lo);
            ch_len.push_back((int32_t)std::min<int64_t>(kChunk, sptr[s + 1] - lo));
        }
        sys_nch[s] = (int32_t)ch_sys.size() - sys_ch0[s];
    }
    const int64_t nch = (int64_t)ch_sys.size();
    const int m = h->prm.gmres_restart;
    PR_TRY(dalloc(h, &h->ch_sys, nch));
    PR_TRY(dalloc(h, &h->ch_lo, nch));
    PR_TRY(dalloc(h, &h->ch_len, nch));
    PR_TRY(dalloc(h, &h->sys_ch0, nsys));
    PR_TRY(dalloc(h, &h->sys_nch, nsys));
    PR_TRY(dalloc(h, &h->bpart, (size_t)nch * 32));
    PR_TRY(dalloc(h, &h->bscal, (size_t)4 * nsys * kBStride));
    PR_TRY(dalloc(h, &h->bgm, (size_t)nsys * ((int64_t)(m + 1) * m + 4 * m + 2)));
    PR_TRY(dalloc(h, &h->bctl, (size_t)3 * nsys + 1));
    PR_TRY(dalloc(h, &h->bbase, nsys));
    PR_TRY(dalloc(h, &h->btol, nsys));
    PR_HIP(h, hipMemcpyAsync(h->ch_sys, ch_sys.data(), nch * sizeof(int32_t), hipMemcpyHostToDevice, st));
    PR_HIP(h, hipMemcpyAsync(h->ch_lo, ch_lo.data(), nch * sizeof(int64_t), hipMemcpyHostToDevice, st));
    PR_HIP(h, hipMemcpyAsync(h->ch_len, ch_len.data(), nch * sizeof(int32_t), hipMemcpyHostToDevice, st));
    PR_HIP(h, hipMemcpyAsync(h->sys_ch0, sys_ch0.data(), nsys * sizeof(int32_t), hipMemcpyHostToDevice, st));
    PR_HIP(h, hipMemcpyAsync(h->sys_nch, sys_nch.data(), nsys * sizeof(int32_t), hipMemcpyHostToDevice, st));
    PR_HIP(h, hipStreamSynchronize(st));
    h->nch = nch;
    h->nsys = (int)nsys;
    if (h->bgexec) {                 // a captured cycle holds the old chunk arrays
        (void)hipGraphExecDestroy(h->bgexec);
        h->bgexec = nullptr;
        h->bgraph_m = -1;
    }
    h->sys_ptr_host.assign(sptr, sptr + nsys + 1);
    h->sys_iters.assign(nsys, 0);
    h->sys_relres.assign(nsys, 0.0);
    return PR_OK;
}

int pr_get_system_info(pr_handle h, int64_t* iters, double* relres) {
    if (!h || h->nsys == 0) return pr_fail(h, PR_ERR_INVALID_ARG, "no systems set on this handle");
    if (iters) std::memcpy(iters, h->sys_iters.data(), h->nsys * sizeof(int64_t));
    if (relres) std::memcpy(relres, h->sys_relres.data(), h->nsys * sizeof(double));
    return PR_OK;
}

int solve_batch(pr_handle h, const double* b, double* x, double tol) {
    const double tstart = now_s();
    hipStream_t s = h->stream;
    // optional per-class device timing: 0 apply, 1 spmv, 2 orthogonalisation
    const bool timing = h->prm.timing != 0;
    // timing = k > 1: only every k-th Arnoldi step is bracketed (the events
    // themselves add a gap between kernels)
    const int tstride = h->prm.timing > 1 ? h->prm.timing : 1;
    bool tsel = timing;
    // a span records the cycle and Arnoldi step it belongs to, so that the
    // steps after every system stopped are not counted
    struct Span { int cls; hipEvent_t a, b; int64_t cyc; int j; };
    std::vector<Span> spans;
    std::vector<int64_t> done_cols;   // steps that ran (largest over the systems), per cycle
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
    const int ns = h->nsys;
    PR_TRY(pr_workspace_internal(h, m));
    // graph replay of whole restart cycles (not with per-kernel timing): the
    // capture needs a stream of its own, and b and x live in handle memory
    // so that one captured cycle serves every later solve
    const bool use_graph = h->prm.graph != 0 && !timing;
    if (use_graph) {
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
    const double* bw = use_graph ? h->gb : b;
    double* xw = use_graph ? h->gx : x;
    if (use_graph) launch_copy(h->gb, b, n, s);
    BGeom bg{h->nch, h->ch_sys, h->ch_lo, h->ch_len, ns, h->sys_ch0, h->sys_nch};
    double* V = h->V;
    double* w = h->w;
    double* r = h->t1;
    double* zt = h->t2;
    double* t3 = h->t2 + n;
    const int64_t ldv = h->ldv;
    double* H1 = h->bscal;
    double* H2 = H1 + (int64_t)ns * kBStride;
    double* HN = H2 + (int64_t)ns * kBStride;
    double* NR = HN + (int64_t)ns * kBStride;
    int32_t* sstop = h->bctl;
    int32_t* scols = sstop + ns;
    int32_t* act = scols + ns;
    int32_t* gstop = act + ns;
    double* R = h->bgm;
    double* cs = R + (int64_t)ns * (m + 1) * m;
    double* sn = cs + (int64_t)ns * m;
    double* gv = sn + (int64_t)ns * m;
    double* yv = gv + (int64_t)ns * (m + 1);
    double* est = yv + (int64_t)ns * m;
    std::vector<double> nr((size_t)ns * kBStride);
    std::vector<int32_t> cols_h(ns, 0), act_h(ns, 0);
    auto norms = [&](const double* v) -> int {
        launch_bgs(0, v, n, 1, const_cast<double*>(v), bg, nullptr, h->bpart, NR, nullptr, nullptr, s);
        PR_HIP(h, hipMemcpyAsync(nr.data(), NR, nr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        PR_HIP(h, hipStreamSynchronize(s));
        return PR_OK;
    };
    PR_TRY(norms(bw));
    std::vector<double> bn(ns), tol_abs(ns);
    for (int i = 0; i < ns; ++i) {
        bn[i] = std::sqrt(nr[(size_t)i * kBStride]);
        if (!std::isfinite(bn[i])) return pr_fail(h, PR_ERR_NONFINITE, "non-finite right-hand side");
        tol_abs[i] = tol * bn[i];
    }
    PR_HIP(h, hipMemcpyAsync(h->btol, tol_abs.data(), ns * sizeof(double), hipMemcpyHostToDevice, s));
    launch_zero(xw, n, s);
    launch_copy(r, bw, n, s);
    std::vector<int64_t> its(ns, 0);
    std::vector<double> rel(ns, 0.0);
    int64_t cycles = 0;
    const int64_t maxit = h->prm.max_iters;
    // One restart cycle of every active system, all on the device (each
    // Arnoldi step ends in the per-system Givens update and stopping test;
    // kernels of stopped systems, or of a stopped batch, return at once),
    // then x_s += M(V_s y_s) for every system that ran and r = b - A x.
    auto enqueue_cycle = [&]() -> int {
        launch_bcycle_init(ns, m, NR, act, gv, sstop, scols, gstop, s);
        launch_bscale(r, V, bg, NR, sstop, gstop, s);
        for (int j = 0; j < m; ++j) {
            tsel = timing && (tcyc * m + j) % tstride == 0;
            tj = j;
            double* vj = V + (int64_t)j * ldv;
            tbeg();
            PR_TRY(pr_precond_internal(h, vj, zt, t3, gstop));
            tend(0);
            tbeg();
            launch_spmv_sell(h->sell(), n, zt, nullptr, w, s, gstop);
            tend(1);
            tbeg();
            launch_bgs(0, V, ldv, j + 1, w, bg, nullptr, h->bpart, H1, sstop, gstop, s);
            launch_bgs(1, V, ldv, j + 1, w, bg, H1, h->bpart, H2, sstop, gstop, s);
            launch_bgs(2, V, ldv, j + 1, w, bg, H2, h->bpart, HN, sstop, gstop, s);
            launch_bscale(w, V + (int64_t)(j + 1) * ldv, bg, HN, sstop, gstop, s);
            tend(2);
            launch_bgivens(j, m, ns, H1, H2, HN, R, cs, sn, gv, est, sstop, scols, h->btol, h->bbase, maxit,
                           gstop, s);
        }
        launch_btrisolve(m, ns, R, gv, yv, scols, s);
        launch_bgemv(V, ldv, bg, yv, m, scols, r, s);
        PR_TRY(pr_precond_internal(h, r, zt, t3, nullptr));
        launch_axpy_dev(xw, zt, 1.0, n, s);
        launch_spmv_sell(h->sell(), n, xw, bw, r, s);
        return PR_OK;
    };
    for (;;) {
        PR_TRY(norms(r));
        if (cycles > 0) done_cols.push_back(*std::max_element(cols_h.begin(), cols_h.end()));
        bool any = false;
        for (int i = 0; i < ns; ++i) {
            if (cycles > 0) its[i] += cols_h[i];
            const double rn = std::sqrt(nr[(size_t)i * kBStride]);
            if (!std::isfinite(rn)) return pr_fail(h, PR_ERR_NONFINITE, "non-finite residual");
            rel[i] = bn[i] > 0.0 ? rn / bn[i] : 0.0;
            act_h[i] = (rel[i] > tol && its[i] < maxit) ? 1 : 0;
            any = any || act_h[i];
        }
        if (!any) break;
        ++cycles;
        ++tcyc;
        PR_HIP(h, hipMemcpyAsync(act, act_h.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PR_HIP(h, hipMemcpyAsync(h->bbase, its.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice, s));
        if (use_graph) {
            if (!h->bgexec || h->bgraph_m != m) {
                if (h->bgexec) {
                    (void)hipGraphExecDestroy(h->bgexec);
                    h->bgexec = nullptr;
                }
                hipGraph_t gr = nullptr;
                PR_HIP(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                const int rc = enqueue_cycle();
                const hipError_t ec = hipStreamEndCapture(s, &gr);
                if (rc < 0) return rc;
                if (ec != hipSuccess)
                    return pr_fail(h, PR_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
                const hipError_t ei = hipGraphInstantiate(&h->bgexec, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (ei != hipSuccess)
                    return pr_fail(h, PR_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
                h->bgraph_m = m;
            }
            PR_HIP(h, hipGraphLaunch(h->bgexec, s));
        } else {
            PR_TRY(enqueue_cycle());
        }
        PR_HIP(h, hipMemcpyAsync(cols_h.data(), scols, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    if (use_graph) launch_copy(x, xw, n, s);
    PR_HIP(h, hipStreamSynchronize(s));
    PR_HIP(h, hipGetLastError());
    h->sys_iters = its;
    h->sys_relres = rel;
    h->sinfo = pr_solve_info{};
    h->sinfo.iters = *std::max_element(its.begin(), its.end());
    h->sinfo.cycles = cycles;
    h->sinfo.reorth = (int32_t)h->sinfo.iters;   // the batch solve always projects twice
    h->sinfo.relres = *std::max_element(rel.begin(), rel.end());
    h->sinfo.relres_est = h->sinfo.relres;
    h->sinfo.status = h->sinfo.relres <= tol ? PR_OK : PR_NOT_CONVERGED;
    h->sinfo.seconds = now_s() - tstart;
    for (const Span& sp : spans) {
        float ms = 0.0f;
        if (sp.j >= 0 && (sp.cyc >= (int64_t)done_cols.size() || sp.j >= done_cols[sp.cyc])) continue;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) != hipSuccess) continue;
        if (sp.cls == 0) { h->sinfo.apply_ms += ms; h->sinfo.n_apply++; }
        if (sp.cls == 1) { h->sinfo.spmv_ms += ms; h->sinfo.n_spmv++; }
        if (sp.cls == 2) { h->sinfo.orth_ms += ms; h->sinfo.n_orth++; }
    }
    return h->sinfo.status;
}
