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

typedef double pr_d4 __attribute__((ext_vector_type(4)));

// P = L R for p x p row-major matrices in LDS (p <= 32) on the FP64 matrix
// cores, 16 x 16 x 4 products accumulated over k in steps of 4; one
// wavefront with every lane active.  TL: L is read transposed (P = L^T R).
// Tile (ti, tj) of P (rows 16 ti.., columns 16 tj..) ends in c[2 ti + tj]
// (only c[0] when p <= 16): lane l holds rows l / 16 + 4 v, v = 0..3, of
// column l % 16 (the FP64 form interleaves the rows, unlike the 16 x 16 FP32
// products, whose lanes hold four consecutive rows).  Operand lanes: A element (row l % 16, k l / 16), B element
// (k l / 16, column l % 16).  Padding rows, columns and k are zero (loads
// from clamped, valid addresses times a 0/1 mask, so no load waits in a
// branch).
template <bool TL>
__device__ __forceinline__ void mm_wave(const double* sL, const double* sR, int p, int lane, pr_d4 c[4]) {
    const bool two = p > 16;
    const int li = lane & 15, lk = lane >> 4;
    const int i0 = li < p ? li : 0;
    const int i1 = 16 + li < p ? 16 + li : 0;
    const double m0 = li < p ? 1.0 : 0.0;
    const double m1 = 16 + li < p ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] = pr_d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < p; k0 += 4) {
        const int k = k0 + lk;
        const int kc = k < p ? k : 0;
        const double mk = k < p ? 1.0 : 0.0;
        const double a0 = (TL ? sL[kc * p + i0] : sL[i0 * p + kc]) * (mk * m0);
        const double b0 = sR[kc * p + i0] * (mk * m0);
        c[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c[0], 0, 0, 0);
        if (two) {
            const double a1 = (TL ? sL[kc * p + i1] : sL[i1 * p + kc]) * (mk * m1);
            const double b1 = sR[kc * p + i1] * (mk * m1);
            c[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c[1], 0, 0, 0);
            c[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c[2], 0, 0, 0);
            c[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c[3], 0, 0, 0);
        }
    }
}

// row and column of element v of tile t held by this lane (layout above)
__device__ __forceinline__ int mm_row(int t, int v, int lane) { return 16 * (t >> 1) + (lane >> 4) + 4 * v; }
__device__ __forceinline__ int mm_col(int t, int lane) { return 16 * (t & 1) + (lane & 15); }

// dst = scale * P for the tiles of mm_wave
__device__ __forceinline__ void mm_store(const pr_d4 c[4], double* dst, int p, int lane, double scale) {
    const int nt = p > 16 ? 4 : 1;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t >= nt) break;
        const int col = mm_col(t, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = mm_row(t, v, lane);
            if (row < p && col < p) dst[row * p + col] = scale * c[t][v];
        }
    }
}

// sum (wave-reduced) and largest value of the diagonal of P
__device__ __forceinline__ void mm_diag(const pr_d4 c[4], int p, int lane, double& sum, double& mx) {
    const int nt = p > 16 ? 4 : 1;
    double s = 0.0, m = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t >= nt) break;
        const int col = mm_col(t, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = mm_row(t, v, lane);
            if (row == col && row < p) {
                s += c[t][v];
                m = fmax(m, c[t][v]);
            }
        }
    }
    sum = wave_sum(s);
    mx = wave_max(m);
}

// E = I - A X into sE; returns ||E||_F^2 (wave-reduced) and, when lb2 is
// not null, the largest squared column norm of E (a lower bound on
// sigma_max(E)^2).  One wavefront, every lane active.
__device__ __forceinline__ double form_E(const double* sA, const double* sX, double* sE, int p, int lane,
                                         double* lb2 = nullptr) {
    pr_d4 c[4];
    mm_wave<false>(sA, sX, p, lane, c);
    const int nt = p > 16 ? 4 : 1;
    double fro2 = 0.0, cs0 = 0.0, cs1 = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t >= nt) break;
        const int col = mm_col(t, lane);
        double cs = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = mm_row(t, v, lane);
            if (row < p && col < p) {
                const double e = (row == col ? 1.0 : 0.0) - c[t][v];
                sE[row * p + col] = e;
                cs += e * e;
            }
        }
        fro2 += cs;
        if (t & 1) cs1 += cs; else cs0 += cs;
    }
    if (lb2) {
        // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the rows of the same columns
        cs0 += __shfl_xor(cs0, 16);
        cs0 += __shfl_xor(cs0, 32);
        cs1 += __shfl_xor(cs1, 16);
        cs1 += __shfl_xor(cs1, 32);
        *lb2 = wave_max(fmax(cs0, cs1));
    }
    return wave_sum(fro2);
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
    pr_d4 c[4];
    mm_wave<true>(sE, sE, p, lane, c);
    double tr, dmax;
    mm_diag(c, p, lane, tr, dmax);
    if (!(tr > 0.0)) {
        lo2 = hi2 = 0.0;
        return false;
    }
    hi2 = fmin(hi2, tr);
    lo2 = fmax(lo2, dmax);
    if (done(lo2, hi2)) return true;
    const double itr = 1.0 / tr;
    __syncthreads();                        // sG may be an operand buffer still being read
    mm_store(c, sG, p, lane, itr);
    __syncthreads();
    double U = log(tr), w = 0.5;
    double* cur = sG;
    double* nxt = sH;
    for (int k = 1; k <= kmax; ++k) {
        mm_wave<true>(cur, cur, p, lane, c);   // N^T N = N^2, N symmetric
        double t, md;
        mm_diag(c, p, lane, t, md);           // t in [1/p, 1]
        const double it = 1.0 / t;
        md *= it;
        mm_store(c, nxt, p, lane, it);
        __syncthreads();
        U += w * log(t);
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
    {
        pr_d4 c[4];
        mm_wave<true>(sE, sE, p, lane, c);
        __syncthreads();                    // sG may be an operand buffer still being read
        mm_store(c, sG, p, lane, 1.0);
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
