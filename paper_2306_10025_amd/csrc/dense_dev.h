// Dense per-patch device routines shared by the batched kernels and
// Algorithm 1: Gauss-Jordan inversion with partial pivoting and the
// criterion building blocks (E = I - A X, its Frobenius norm, a column-norm
// lower bound, and the exact largest singular value).
#pragma once

#include "pr_internal.h"

namespace pr_dev {

constexpr int kMaxPs = 32;
// squarings of the criterion bracket before the exact singular value
// (a bracket of relative width at most log(p) / 2^12 < 0.1 % in sigma^2)
constexpr int kSquarings = 12;

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
    // every load unconditional from a clamped address, the padding dropped
    // by a multiply (a load feeding a select gets sunk into a branch, and
    // each branch then waits for its load)
    const int64_t row = (int64_t)(act ? r : 0) * p;
#pragma unroll
    for (int c = 0; c < MAXP; ++c) a[c] = A[row + (c < p ? c : 0)];
#pragma unroll
    for (int c = 0; c < MAXP; ++c) {
        a[c] *= (act && c < p) ? 1.0 : 0.0;
        x[c] = (act && c == r) ? 1.0 : 0.0;
    }
    bool used = !act;
    int mycol = -1;
    int info = 0;
    // The pivot steps stay a loop (unrolled, the 32-row form was about 8,000
    // straight-line instructions, and one wavefront running it once per call
    // waited on instruction fetch).  Column k of this row is carried in ak:
    // step k picks column k + 1 out of the updated row with selects, so the
    // row stays in registers without dynamic indexing.
    double ak = a[0];
#pragma unroll 1
    for (int k = 0; k < p; ++k) {
        double cv = used ? -1.0 : fabs(ak);
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
        const double pk = __shfl(ak, piv, G);
        const double inv = 1.0 / pk;
        const double f = (r == piv) ? 0.0 : ak * inv;
        double next = 0.0;
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
            next = (c == k + 1) ? a[c] : next;
        }
        ak = next;
        if (r == piv) {
            used = true;
            mycol = k;
        }
    }
    if (act && mycol >= 0) {
#pragma unroll
        for (int c = 0; c < MAXP; ++c)
            if (c < p) X[(int64_t)mycol * p + c] = x[c];
    }
    return info;
}

// ---------------------------------------------------------------------------
// criterion helpers (one wavefront; LDS buffers of kMaxPs^2 doubles)
// ---------------------------------------------------------------------------

// dst[0..n) = src[0..n) for one wavefront, n <= kMaxPs^2: all loads are
// issued (from clamped, valid addresses) before the first store, instead of
// one load-wait-store round per element stride.
__device__ __forceinline__ void lds_load(double* dst, const double* __restrict__ src, int n, int lane) {
    constexpr int U = kMaxPs * kMaxPs / PR_WAVE;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = lane + u * PR_WAVE;
        v[u] = src[e < n ? e : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = lane + u * PR_WAVE;
        if (e < n) dst[e] = v[u];
    }
}

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

// Bracket [lo2, hi2] of lambda = sigma_max(E)^2 tightened by repeated
// squaring of G = E^T E, which is symmetric positive semidefinite with
// eigenvalues l_1 >= ... >= l_p >= 0.  With N_0 = G / tr G and
// N_k = N_{k-1}^2 / tr(N_{k-1}^2) (so N_k = G^(2^k) / tr G^(2^k)):
//   l_1^(2^k) <= tr G^(2^k)             (every other eigenvalue is >= 0),
//   l_1^(2^k) >= max_j (G^(2^k))_jj     (no diagonal entry of a PSD matrix
//                                        exceeds its largest eigenvalue),
// so log l_1 lies in [U_k + log(max_j (N_k)_jj) / 2^k, U_k], where
// U_k = log tr G + sum_{i=1..k} log tr(N_{i-1}^2) / 2^i, a bracket of width
// at most log(p) / 2^k.  done(lo2, hi2) is asked after each step; at most
// kmax squarings.  One wavefront; sG and sH are p x p LDS scratch; sE may be
// the same buffer as sH (E is consumed once G is formed).  Returns false
// when E is zero (then lo2 = hi2 = 0).
template <class Done>
__device__ bool sigma2_bracket(const double* sE, double* sG, double* sH, int p, int lane, int kmax,
                               double& lo2, double& hi2, Done done) {
    for (int e = lane; e < p * p; e += PR_WAVE) {
        const int a = e / p, b = e % p;
        double acc = 0.0;
        for (int c = 0; c < p; ++c) acc = fma(sE[c * p + a], sE[c * p + b], acc);
        sG[e] = acc;
    }
    __syncthreads();
    const double tr = wave_sum(lane < p ? sG[lane * p + lane] : 0.0);
    if (!(tr > 0.0)) {
        lo2 = hi2 = 0.0;
        return false;
    }
    hi2 = fmin(hi2, tr);
    lo2 = fmax(lo2, wave_max(lane < p ? sG[lane * p + lane] : 0.0));
    if (done(lo2, hi2)) return true;
    const double itr = 1.0 / tr;
    for (int e = lane; e < p * p; e += PR_WAVE) sG[e] *= itr;
    __syncthreads();
    double U = log(tr), w = 0.5;
    double* cur = sG;
    double* nxt = sH;
    for (int k = 1; k <= kmax; ++k) {
        for (int e = lane; e < p * p; e += PR_WAVE) {
            const int a = e / p, b = e % p;
            double acc = 0.0;
            for (int c = 0; c < p; ++c) acc = fma(cur[c * p + a], cur[c * p + b], acc);   // N symmetric
            nxt[e] = acc;
        }
        __syncthreads();
        const double t = wave_sum(lane < p ? nxt[lane * p + lane] : 0.0);   // in [1/p, 1]
        const double it = 1.0 / t;
        for (int e = lane; e < p * p; e += PR_WAVE) nxt[e] *= it;
        __syncthreads();
        U += w * log(t);
        const double md = wave_max(lane < p ? nxt[lane * p + lane] : 0.0);
        hi2 = fmin(hi2, exp(U));
        lo2 = fmax(lo2, exp(U + w * log(md)));
        w *= 0.5;
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (done(lo2, hi2)) break;
    }
    return true;
}

// sigma_max(E)^2 as the largest eigenvalue of G = E^T E by cyclic Jacobi
// rotations; sG is overwritten.  Requires a one-wave block (uses barriers).
__device__ inline double sigma_max2_jacobi(const double* sE, double* sG, int p, int lane) {
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

}  // namespace pr_dev
