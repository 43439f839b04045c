// Dense per-patch kernels in FP64:
//  * batched inverse by Gauss-Jordan elimination with partial pivoting (the
//    factorisation of the database matrices; Section 4, Experiment 3 uses an
//    LU factorisation, whose explicit inverse is the same operator);
//  * the similarity criteria: d(A,B) = ||I - A B^{-1}||_2 (Eq.(5)) with the
//    largest singular value of E = I - A X from cyclic Jacobi on E^T E, and
//    the entrywise l1 / Frobenius differences (remark after Eq.(4));
//  * Algorithm 1 (tolerance construction) as device-resident rounds: the
//    lowest unresolved patch joins the database, then every unresolved patch
//    is tested against it.  This gives the sequential first-match result:
//    patch i is compared with database entries in append order and keeps the
//    first match.  A certified norm bound skips pairs that cannot match
//    (the subset search suggested after Algorithm 1).
#include "pr_internal.h"

#include <climits>

namespace {

constexpr int kMaxPs = 32;

// ---------------------------------------------------------------------------
// Gauss-Jordan inverse of one p x p matrix per group of G lanes; lane r of the
// group holds row r of [A | I] in registers.  Pivot: largest |a_ik| over rows
// not yet used, ties to the lowest row.  Row piv_k ends as row k of A^{-1}.
// ---------------------------------------------------------------------------
template <int MAXP, int G>
__device__ __forceinline__ int gj_invert(const double* __restrict__ A, double* __restrict__ X,
                                         int p, int r) {
    double a[MAXP], x[MAXP];
    const bool act = r < p;
#pragma unroll
    for (int c = 0; c < MAXP; ++c) {
        a[c] = (act && c < p) ? A[(int64_t)r * p + c] : 0.0;
        x[c] = (act && c == r) ? 1.0 : 0.0;
    }
    bool used = !act;
    int mycol = -1;
    int info = 0;
#pragma unroll
    for (int k = 0; k < MAXP; ++k) {
        if (k < p) {
            double cv = used ? -1.0 : fabs(a[k]);
            int ci = r;
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                const double ov = __shfl_xor(cv, o, G);
                const int oi = __shfl_xor(ci, o, G);
                if (ov > cv || (ov == cv && oi < ci)) {
                    cv = ov;
                    ci = oi;
                }
            }
            const int piv = ci;
            if (!(cv > 0.0) && info == 0) info = k + 1;
            const double pk = __shfl(a[k], piv, G);
            const double inv = 1.0 / pk;
            const double f = (r == piv) ? 0.0 : a[k] * inv;
#pragma unroll
            for (int c = 0; c < MAXP; ++c) {
                if (c < p) {
                    const double pa = __shfl(a[c], piv, G);
                    const double px = __shfl(x[c], piv, G);
                    if (r == piv) {
                        a[c] = pa * inv;
                        x[c] = px * inv;
                    } else {
                        a[c] = fma(-f, pa, a[c]);
                        x[c] = fma(-f, px, x[c]);
                    }
                }
            }
            if (r == piv) {
                used = true;
                mycol = k;
            }
        }
    }
    if (act && mycol >= 0) {
#pragma unroll
        for (int c = 0; c < MAXP; ++c)
            if (c < p) X[(int64_t)mycol * p + c] = x[c];
    }
    return info;
}

template <int MAXP, int G>
__global__ __launch_bounds__(256) void k_batch_inverse(int p, int64_t count, const double* __restrict__ A,
                                                       const int64_t* __restrict__ aoff,
                                                       const int32_t* __restrict__ sel,
                                                       const int64_t* __restrict__ pptr,
                                                       double* __restrict__ X,
                                                       const int64_t* __restrict__ xoff,
                                                       int32_t* __restrict__ info) {
    const int64_t gsz = (int64_t)blockDim.x / G;
    const int64_t grp = (int64_t)blockIdx.x * gsz + threadIdx.x / G;
    const int r = threadIdx.x % G;
    const int64_t stride = (int64_t)gridDim.x * gsz;
    for (int64_t i = grp; i < count; i += stride) {
        const int64_t m = sel ? sel[i] : i;
        const int pm = pptr ? (int)(pptr[m + 1] - pptr[m]) : p;
        const double* Am = A + (aoff ? aoff[m] : m * (int64_t)p * p);
        double* Xm = X + (xoff ? xoff[m] : m * (int64_t)p * p);
        const int inf = gj_invert<MAXP, G>(Am, Xm, pm, r);
        if (r == 0 && info) info[m] = inf;
    }
}

template <int MAXP, int G>
void run_inverse(int p, int64_t count, const double* A, const int64_t* aoff, const int32_t* sel,
                 const int64_t* pptr, double* X, const int64_t* xoff, int32_t* info, hipStream_t s) {
    const int per_block = 256 / G;
    int64_t blocks = (count + per_block - 1) / per_block;
    if (blocks > 65536) blocks = 65536;
    k_batch_inverse<MAXP, G><<<(unsigned)blocks, 256, 0, s>>>(p, count, A, aoff, sel, pptr, X, xoff, info);
}

// ---------------------------------------------------------------------------
// criterion helpers (one wavefront; LDS buffers of kMaxPs^2 doubles)
// ---------------------------------------------------------------------------

// E = I - A X into sE; returns ||E||_F^2 (wave-reduced).
__device__ __forceinline__ double form_E(const double* sA, const double* sX, double* sE, int p,
                                         int lane) {
    double fro2 = 0.0;
    for (int e = lane; e < p * p; e += PR_WAVE) {
        const int a = e / p, b = e % p;
        double acc = 0.0;
        for (int c = 0; c < p; ++c) acc = fma(sA[a * p + c], sX[c * p + b], acc);
        const double v = (a == b ? 1.0 : 0.0) - acc;
        sE[e] = v;
        fro2 += v * v;
    }
    return wave_sum(fro2);
}

// Largest column 2-norm of E squared (a lower bound on sigma_max^2).
__device__ __forceinline__ double max_col2(const double* sE, int p, int lane) {
    double m = 0.0;
    if (lane < p) {
        double s = 0.0;
        for (int a = 0; a < p; ++a) s += sE[a * p + lane] * sE[a * p + lane];
        m = s;
    }
    return wave_max(m);
}

// sigma_max(E)^2 as the largest eigenvalue of G = E^T E by cyclic Jacobi
// rotations; sG is overwritten.  Requires a one-wave block (uses barriers).
__device__ double sigma_max2_jacobi(const double* sE, double* sG, int p, int lane) {
    for (int e = lane; e < p * p; e += PR_WAVE) {
        const int a = e / p, b = e % p;
        double acc = 0.0;
        for (int c = 0; c < p; ++c) acc = fma(sE[c * p + a], sE[c * p + b], acc);
        sG[e] = acc;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = lane; e < p * p; e += PR_WAVE) {
            const int a = e / p, b = e % p;
            const double v = sG[e];
            if (a == b) dia += v * v; else off += v * v;
        }
        off = wave_sum(off);
        dia = wave_sum(dia);
        if (off <= 1e-32 * dia || off == 0.0) break;
        for (int i = 0; i < p - 1; ++i) {
            for (int j = i + 1; j < p; ++j) {
                const double gij = sG[i * p + j];
                if (fabs(gij) <= 1e-300) continue;      // uniform: every lane reads the same value
                const double gii = sG[i * p + i], gjj = sG[j * p + j];
                const double theta = (gjj - gii) / (2.0 * gij);
                double t;
                if (fabs(theta) > 1e150) {
                    t = 0.5 / theta;
                } else {
                    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                }
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                __syncthreads();
                if (lane < p) {
                    const double gki = sG[lane * p + i], gkj = sG[lane * p + j];
                    sG[lane * p + i] = c * gki - s * gkj;
                    sG[lane * p + j] = s * gki + c * gkj;
                }
                __syncthreads();
                if (lane < p) {
                    const double gik = sG[i * p + lane], gjk = sG[j * p + lane];
                    sG[i * p + lane] = c * gik - s * gjk;
                    sG[j * p + lane] = s * gik + c * gjk;
                }
                __syncthreads();
            }
        }
    }
    double m = lane < p ? sG[lane * p + lane] : 0.0;
    m = wave_max(m);
    return m > 0.0 ? m : 0.0;
}

__global__ __launch_bounds__(64) void k_criterion_batch(int p, int64_t count, int crit,
                                                        const double* __restrict__ A,
                                                        const double* __restrict__ B,
                                                        const double* __restrict__ X,
                                                        double* __restrict__ d) {
    __shared__ double sA[kMaxPs * kMaxPs];
    __shared__ double sX[kMaxPs * kMaxPs];
    __shared__ double sE[kMaxPs * kMaxPs];
    const int lane = threadIdx.x;
    const int64_t pp = (int64_t)p * p;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        if (crit == PR_CRIT_SPECTRAL) {
            for (int e = lane; e < pp; e += PR_WAVE) {
                sA[e] = A[i * pp + e];
                sX[e] = X[i * pp + e];
            }
            __syncthreads();
            form_E(sA, sX, sE, p, lane);
            __syncthreads();
            const double s2 = sigma_max2_jacobi(sE, sA, p, lane);
            if (lane == 0) d[i] = sqrt(s2);
            __syncthreads();
        } else {
            double acc = 0.0;
            for (int e = lane; e < pp; e += PR_WAVE) {
                const double v = A[i * pp + e] - B[i * pp + e];
                acc += (crit == PR_CRIT_L1) ? fabs(v) : v * v;
            }
            acc = wave_sum(acc);
            if (lane == 0) d[i] = (crit == PR_CRIT_L1) ? acc : sqrt(acc);
        }
    }
}

// ---------------------------------------------------------------------------
// Algorithm 1 rounds
// ---------------------------------------------------------------------------
// ctrl: [0] current entry's patch (or -1)  [1] lowest unresolved patch (next entry)
//       [2] entries so far (m)             [3] done flag
//       [4] number of candidates this round [5] error: singular entry patch + 1
// counters: [0] evaluations [1] exact singular values [2] key-bound skips
// win[0] = key of the current entry, win[1] = half-width of the key window

// R1: the lowest unresolved patch becomes database entry m; invert it.
__global__ __launch_bounds__(64) void k_alg1_open(int32_t* ctrl, double* win, int crit, double eps,
                                                  int64_t n_p, const int64_t* __restrict__ ptr,
                                                  const double* __restrict__ tiles,
                                                  const int64_t* __restrict__ toff, int uniform_ps,
                                                  const double* __restrict__ keynorm,
                                                  int32_t* __restrict__ status, int32_t* phi,
                                                  int32_t* reps, double* db, int64_t db_stride,
                                                  int32_t* ctrl_next) {
    if (ctrl[3]) return;
    const int lane = threadIdx.x;
    const int32_t r = *ctrl_next;
    if (r >= n_p) {
        if (lane == 0) {
            ctrl[3] = 1;
            ctrl[0] = -1;
        }
        return;
    }
    const int32_t m = ctrl[2];
    const int p = (int)(ptr[r + 1] - ptr[r]);
    const double* Ar = tiles + (uniform_ps ? (int64_t)r * uniform_ps * uniform_ps : toff[r]);
    double* Xm = db + (int64_t)m * db_stride;
    const int info = gj_invert<kMaxPs, PR_WAVE / 2>(Ar, Xm, p, lane < 32 ? lane : 64);
    // bound: spectral d >= |kA - kB| / (sqrt(p) ||B||_F) with k = ||.||_F ;
    // l1 / Frobenius: d >= |kA - kB| with k the same entrywise norm.
    const double kb = keynorm[r];
    double half;
    if (crit == PR_CRIT_SPECTRAL)
        half = eps * sqrt((double)p) * kb * (1.0 + 1e-10) + (p * p + 64) * 2.3e-16 * kb;
    else
        half = eps * (1.0 + 1e-10) + (p * p + 64) * 2.3e-16 * kb;
    __syncthreads();
    if (lane == 0) {
        if (info != 0 && ctrl[5] == 0) ctrl[5] = r + 1;
        reps[m] = r;
        phi[r] = m;
        status[r] = 1;
        ctrl[0] = r;
        ctrl[2] = m + 1;
        ctrl[4] = 0;
        win[0] = kb;
        win[1] = half;
        *ctrl_next = (int32_t)n_p;  // R2 lowers it to the next unresolved patch
    }
}

// R2a: key-bound filter over all unresolved patches; survivors go to cand[].
__global__ void k_alg1_filter(const int32_t* ctrl, const double* win, int64_t n_p,
                              const int64_t* __restrict__ ptr, const double* __restrict__ keynorm,
                              const int32_t* __restrict__ status, int32_t* cand, int32_t* ncand,
                              int32_t* ctrl_next, unsigned long long* counters) {
    if (ctrl[3]) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool skip = false;
    if (i < n_p && status[i] == 0) {
        const int32_t r = ctrl[0];
        const int pr = (int)(ptr[r + 1] - ptr[r]);
        const int pi = (int)(ptr[i + 1] - ptr[i]);
        if (pi == pr && fabs(keynorm[i] - win[0]) <= win[1]) {
            const int32_t slot = atomicAdd(ncand, 1);
            cand[slot] = (int32_t)i;
        } else {
            atomicMin(ctrl_next, (int32_t)i);
            skip = true;
        }
    }
    const unsigned long long nskip = __popcll(__ballot(skip));
    if ((threadIdx.x & (PR_WAVE - 1)) == 0 && nskip) atomicAdd(&counters[2], nskip);
}

// R2b: evaluate the criterion for every candidate (one wavefront per pair).
__global__ __launch_bounds__(64) void k_alg1_eval(const int32_t* ctrl, int crit, double eps,
                                                  const int64_t* __restrict__ ptr,
                                                  const double* __restrict__ tiles,
                                                  const int64_t* __restrict__ toff, int uniform_ps,
                                                  int32_t* status, int32_t* phi,
                                                  const double* __restrict__ db, int64_t db_stride,
                                                  const int32_t* __restrict__ cand,
                                                  const int32_t* __restrict__ ncand,
                                                  int32_t* ctrl_next,
                                                  unsigned long long* counters) {
    if (ctrl[3]) return;
    const int nc = *ncand;
    if ((int)blockIdx.x >= nc) return;
    __shared__ double sA[kMaxPs * kMaxPs];
    __shared__ double sX[kMaxPs * kMaxPs];
    __shared__ double sE[kMaxPs * kMaxPs];
    const int lane = threadIdx.x;
    const int32_t r = ctrl[0];
    const int32_t m = ctrl[2] - 1;
    const int p = (int)(ptr[r + 1] - ptr[r]);
    const int pp = p * p;
    const double* Br = tiles + (uniform_ps ? (int64_t)r * uniform_ps * uniform_ps : toff[r]);
    const double* Xm = db + (int64_t)m * db_stride;
    for (int e = lane; e < pp; e += PR_WAVE) sX[e] = (crit == PR_CRIT_SPECTRAL) ? Xm[e] : Br[e];
    __syncthreads();
    unsigned long long nev = 0, nex = 0;
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        const int32_t i = cand[c];
        const double* Ai = tiles + (uniform_ps ? (int64_t)i * uniform_ps * uniform_ps : toff[i]);
        bool match;
        ++nev;
        if (crit == PR_CRIT_SPECTRAL) {
            for (int e = lane; e < pp; e += PR_WAVE) sA[e] = Ai[e];
            __syncthreads();
            const double fro2 = form_E(sA, sX, sE, p, lane);
            __syncthreads();
            const double lb2 = max_col2(sE, p, lane);
            const double e2 = eps * eps;
            if (fro2 * (1.0 + 1e-12) < e2) {
                match = true;                       // sigma_max <= ||E||_F < eps
            } else if (lb2 * (1.0 - 1e-12) >= e2) {
                match = false;                      // sigma_max >= max column norm >= eps
            } else {
                const double s2 = sigma_max2_jacobi(sE, sA, p, lane);
                match = sqrt(s2) < eps;
                ++nex;
            }
            __syncthreads();
        } else {
            double acc = 0.0;
            for (int e = lane; e < pp; e += PR_WAVE) {
                const double v = Ai[e] - sX[e];
                acc += (crit == PR_CRIT_L1) ? fabs(v) : v * v;
            }
            acc = wave_sum(acc);
            const double dv = (crit == PR_CRIT_L1) ? acc : sqrt(acc);
            match = dv < eps;
        }
        if (lane == 0) {
            if (match) {
                phi[i] = m;
                status[i] = 1;
            } else {
                atomicMin(ctrl_next, i);
            }
        }
    }
    if (lane == 0) {
        atomicAdd(&counters[0], nev);
        if (nex) atomicAdd(&counters[1], nex);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

void launch_batch_inverse(int p, int64_t count, const double* A, const int64_t* aoff,
                          const int32_t* sel, const int64_t* pptr, double* X, const int64_t* xoff,
                          int32_t* info, hipStream_t s) {
    if (count <= 0) return;
    if (p <= 4) run_inverse<4, 4>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
    else if (p <= 8) run_inverse<8, 8>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
    else if (p <= 12) run_inverse<12, 16>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
    else if (p <= 16) run_inverse<16, 16>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
    else if (p <= 20) run_inverse<20, 32>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
    else if (p <= 24) run_inverse<24, 32>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
    else if (p <= 28) run_inverse<28, 32>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
    else run_inverse<32, 32>(p, count, A, aoff, sel, pptr, X, xoff, info, s);
}

void launch_batch_criterion(int p, int64_t count, int crit, const double* A, const double* B,
                            const double* X, double* d, hipStream_t s) {
    if (count <= 0) return;
    int64_t blocks = count < 65536 ? count : 65536;
    k_criterion_batch<<<(unsigned)blocks, 64, 0, s>>>(p, count, crit, A, B, X, d);
}

// Scratch layout inside Alg1Dev: ctrl int32[8] (ctrl[7] = next), win in counters' tail.
void launch_alg1_rounds(int rounds, const Alg1Dev& a, int crit, double eps, int64_t n_p,
                        const int64_t* ptr, const double* tiles, const int64_t* toff,
                        int uniform_ps, const double* keynorm, int32_t* phi, int32_t* reps,
                        double* db, int64_t db_stride, hipStream_t s) {
    int32_t* cand = a.cand;
    int32_t* ctrl = a.ctrl;
    int32_t* next = a.ctrl + 7;
    int32_t* ncand = a.ctrl + 4;
    double* win = reinterpret_cast<double*>(a.counters + 4);
    const unsigned fblocks = (unsigned)((n_p + 255) / 256);
    const unsigned eblocks = (unsigned)(n_p < 4096 ? n_p : 4096);
    for (int t = 0; t < rounds; ++t) {
        k_alg1_open<<<1, 64, 0, s>>>(ctrl, win, crit, eps, n_p, ptr, tiles, toff, uniform_ps,
                                      keynorm, a.status, phi, reps, db, db_stride, next);
        k_alg1_filter<<<fblocks, 256, 0, s>>>(ctrl, win, n_p, ptr, keynorm, a.status, cand, ncand,
                                              next, a.counters);
        k_alg1_eval<<<eblocks, 64, 0, s>>>(ctrl, crit, eps, ptr, tiles, toff, uniform_ps, a.status,
                                           phi, db, db_stride, cand, ncand, next, a.counters);
    }
}
