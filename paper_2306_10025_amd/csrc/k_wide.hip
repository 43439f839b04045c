// Patches with more than 32 dofs.  With q cells per patch and degree-p
// elements a patch has p_s = q (p+1)^d dofs (Section 2): 216 for the degree-5
// hexahedra of Experiment 3, several hundred in general.  Such a tile no
// longer fits one wavefront's registers or LDS (216^2 doubles are 373 KB), so
// every kernel here gives a patch (or a pair, or a group of patches) a block
// of 256 threads and keeps tiles, inverses and criterion products in device
// memory:
//  * extraction stages rows of the tile in LDS chunks and writes them out
//    coalesced; the boundary key is the 32-bit XOR fold of the mask of rows
//    with a single nonzero (equal to the mask itself up to 32 dofs);
//  * the inverse is Gauss-Jordan elimination with partial pivoting over the
//    whole column, in place in device memory, one block per matrix;
//  * Algorithm 1 opens one entry per round (the first open patch), so every
//    patch meets the entries in creation order, exactly as in the sequential
//    algorithm; a pair whose norm gap already exceeds what the criterion
//    allows is skipped; the entrywise criteria are one pass over the tile
//    pair; the spectral one forms E = I - A X on the FP64 matrix cores and
//    decides d < eps from a bracket on sigma_max(E)^2 (column norms and the
//    Frobenius norm, then repeated squaring of E^T E);
//  * the apply stacks up to 16 patches of one database entry, so
//    Y = X_j [r_1 .. r_16] runs on the matrix cores with X_j read transposed
//    (16 consecutive rows of one column per 16 lanes); when (almost) every
//    patch is its own entry a block streams its patch's X^T with vector FMAs.
#include "pr_internal.h"

namespace {

constexpr int kWT = 256;                 // threads per block
constexpr int kWW = kWT / PR_WAVE;       // waves per block
constexpr int kChunk = 8192;             // doubles of the extraction row buffer (64 KB)
constexpr int kSquaringsWide = 40;       // bracket width <= 2 log(p) / 2^40 in log sigma^2
constexpr double kGapSlack = 1e-10;      // relative slack of the pruning norm gap
constexpr int kRStride = 17;             // LDS row stride (doubles) of the staged residuals

typedef double wd4 __attribute__((ext_vector_type(4)));
typedef float wf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double block_sum(double v, double* sred) {
    v = wave_sum(v);
    __syncthreads();                      // sred may still be read by a previous call
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) sred[threadIdx.x / PR_WAVE] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWW; ++w) t += sred[w];
    return t;
}

__device__ __forceinline__ double block_max(double v, double* sred) {
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) sred[threadIdx.x / PR_WAVE] = v;
    __syncthreads();
    double t = sred[0];
#pragma unroll
    for (int w = 1; w < kWW; ++w) t = fmax(t, sred[w]);
    return t;
}

__device__ __forceinline__ int64_t tile_off(int64_t k, int p, const int64_t* toff, int uniform_ps) {
    return uniform_ps ? k * (int64_t)uniform_ps * uniform_ps : toff[k];
}

// ---------------------------------------------------------------------------
// validation of the patches above 32 dofs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWT) void k_validate_wide(const int64_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ dofs, int64_t n_p,
                                                       int64_t n, int32_t* flags) {
    __shared__ int32_t sd[kWideMaxPs];
    __shared__ int s_bad, s_dup;
    for (int64_t k = blockIdx.x; k < n_p; k += gridDim.x) {
        const int64_t s0 = ptr[k];
        const int p = (int)(ptr[k + 1] - s0);
        if (p <= 32 || p > kWideMaxPs) continue;          // the same for the whole block
        if (threadIdx.x == 0) {
            s_bad = 0;
            s_dup = 0;
        }
        __syncthreads();
        for (int a = threadIdx.x; a < p; a += kWT) {
            const int32_t g = dofs[s0 + a];
            sd[a] = g;
            if (g < 0 || g >= n) s_bad = 1;
        }
        __syncthreads();
        if (!s_bad)
            for (int a = threadIdx.x; a < p; a += kWT)
                for (int b = 0; b < a; ++b)
                    if (sd[b] == sd[a]) s_dup = 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_bad) atomicMin(&flags[2], (int32_t)k);
            else if (s_dup) atomicMin(&flags[3], (int32_t)k);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// extraction: A_k[a][b] = A[g_a][g_b], one block per patch
// ---------------------------------------------------------------------------
// The patch dofs go into an LDS hash map (dof -> local index, open
// addressing at load at most 1/2).  Rows go through an LDS buffer of kChunk
// doubles, kChunk / p rows at a time: the buffer is zeroed, each wavefront
// takes a row and its lanes read the CSR row with unit stride, look each
// column up in the map and drop the value into place, and the buffer is
// written to the tile with coalesced stores.  (Walking all the patch rows'
// nonzeros as one sequence, each entry finding its row and then its column
// by binary search, took 8.9 ms for Experiment 3's 8000 patches of 216
// dofs: about 14 dependent LDS reads per stored entry.)
constexpr int kExHash = 2 * kWideMaxPs;   // slots of the dof map

__device__ __forceinline__ int ex_hash(int32_t g) { return (int)(((uint32_t)g * 2654435761u) >> 22); }
static_assert(kExHash == 1024, "ex_hash yields 10 bits");

__global__ __launch_bounds__(kWT) void k_extract_wide(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, const double* __restrict__ val,
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ dofs, int64_t n_p,
    const int64_t* __restrict__ toff, int uniform_ps, double* __restrict__ tiles, uint32_t* __restrict__ keys,
    double* __restrict__ fnorm, double* __restrict__ l1norm, int32_t* flags) {
    __shared__ double sbuf[kChunk];
    __shared__ int32_t s_g[kWideMaxPs];
    __shared__ int32_t s_hk[kExHash];
    __shared__ int16_t s_hv[kExHash];
    __shared__ double sred[kWW];
    __shared__ uint32_t s_key;
    __shared__ int s_fin;
    const int tid = threadIdx.x, lane = tid & (PR_WAVE - 1), wv = tid / PR_WAVE;
    for (int64_t k = blockIdx.x; k < n_p; k += gridDim.x) {
        const int64_t s0 = ptr[k];
        const int p = (int)(ptr[k + 1] - s0);
        const int64_t t0 = tile_off(k, p, toff, uniform_ps);
        for (int h = tid; h < kExHash; h += kWT) s_hk[h] = -1;
        if (tid == 0) {
            s_key = 0u;
            s_fin = 1;
        }
        __syncthreads();
        for (int a = tid; a < p; a += kWT) {
            const int32_t g = dofs[s0 + a];
            s_g[a] = g;
            int h = ex_hash(g);
            while (true) {
                const int32_t old = atomicCAS(&s_hk[h], -1, g);
                if (old == -1) {
                    s_hv[h] = (int16_t)a;
                    break;
                }
                if (old == g) break;                 // repeated dof (validation rejects these)
                h = (h + 1) & (kExHash - 1);
            }
        }
        __syncthreads();
        const int R = p < kChunk / p ? p : kChunk / p;
        double sq = 0.0, ab = 0.0;
        bool fin = true;
        uint32_t key = 0u;
        for (int a0 = 0; a0 < p; a0 += R) {
            const int a1 = a0 + R < p ? a0 + R : p;
            const int ne = (a1 - a0) * p;
            for (int e = tid; e < ne; e += kWT) sbuf[e] = 0.0;
            __syncthreads();
            for (int a = a0 + wv; a < a1; a += kWW) {
                const int32_t g = s_g[a];
                const int64_t q1 = rowptr[g + 1];
                double* row = sbuf + (a - a0) * p;
                for (int64_t q = rowptr[g] + lane; q < q1; q += PR_WAVE) {
                    const int32_t c = col[q];
                    const double v = val[q];
                    int h = ex_hash(c);
                    while (true) {                   // ends at c or at an empty slot
                        const int32_t kh = s_hk[h];
                        if (kh == c) {
                            row[s_hv[h]] = v;
                            break;
                        }
                        if (kh == -1) break;
                        h = (h + 1) & (kExHash - 1);
                    }
                }
            }
            __syncthreads();
            double* dst = tiles + t0 + (int64_t)a0 * p;
            for (int e = tid; e < ne; e += kWT) {
                const double v = sbuf[e];
                dst[e] = v;
                sq += v * v;
                ab += fabs(v);
                fin = fin && isfinite(v);
            }
            for (int a = a0 + tid; a < a1; a += kWT) {
                const double* rw = sbuf + (a - a0) * p;
                int nz = 0;
                for (int b = 0; b < p; ++b) nz += (rw[b] != 0.0) ? 1 : 0;
                if (nz == 1) key ^= 1u << (a & 31);
            }
            __syncthreads();
        }
        if (key) atomicXor(&s_key, key);
        if (!fin) atomicAnd(&s_fin, 0);
        sq = block_sum(sq, sred);
        ab = block_sum(ab, sred);                        // its barriers also order s_key, s_fin
        if (tid == 0) {
            keys[k] = s_key;
            fnorm[k] = sqrt(sq);
            l1norm[k] = ab;
            if (!s_fin) atomicMin(&flags[5], (int32_t)k);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Gauss-Jordan inverse in place, partial pivoting over the whole column
// ---------------------------------------------------------------------------
// Step c: the pivot is the largest |M[r][c]| over rows r >= c (lowest r on
// ties); rows c and r are swapped; row c is divided by the pivot, with the
// pivot position taking 1 / pivot; every other row i loses M[i][c] times the
// new row c, with position c taking -M[i][c] / pivot.  After the last step M
// holds the inverse of the row-swapped matrix, and the column swaps undone in
// reverse order give A^{-1}.  Wave w updates rows w, w + 4, ...; a row whose
// factor is zero is unchanged and skipped.
__global__ __launch_bounds__(kWT) void k_gj_wide(int64_t count, const int32_t* __restrict__ list,
                                                 const int64_t* __restrict__ ptr, const double* __restrict__ tiles,
                                                 const int64_t* __restrict__ toff, int uniform_ps,
                                                 double* __restrict__ X, const int64_t* __restrict__ xoff,
                                                 int32_t* __restrict__ info) {
    __shared__ double s_row[kWideMaxPs];
    __shared__ double s_col[kWideMaxPs];
    __shared__ int32_t s_piv[kWideMaxPs];
    __shared__ double s_bv[kWW];
    __shared__ int s_bi[kWW];
    __shared__ int s_r;
    __shared__ double s_best;
    const int tid = threadIdx.x, lane = tid & (PR_WAVE - 1), w = tid / PR_WAVE;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t k = list ? list[i] : i;
        const int p = ptr ? (int)(ptr[k + 1] - ptr[k]) : uniform_ps;     // no ptr: a dense batch
        const double* src = tiles + tile_off(k, p, toff, uniform_ps);
        double* M = X + (xoff ? xoff[i] : i * (int64_t)p * p);
        for (int e = tid; e < p * p; e += kWT) M[e] = src[e];
        __syncthreads();
        int bad = 0;
        for (int c = 0; c < p; ++c) {
            double bv = -1.0;
            int bi = INT_MAX;
            for (int r = c + tid; r < p; r += kWT) {
                const double v = fabs(M[(int64_t)r * p + c]);
                if (v > bv) {
                    bv = v;
                    bi = r;
                }
            }
            for (int o = PR_WAVE >> 1; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int oi = __shfl_xor(bi, o);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            if (lane == 0) {
                s_bv[w] = bv;
                s_bi[w] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                for (int u = 1; u < kWW; ++u)
                    if (s_bv[u] > bv || (s_bv[u] == bv && s_bi[u] < bi)) {
                        bv = s_bv[u];
                        bi = s_bi[u];
                    }
                s_r = bi;
                s_best = bv;
                s_piv[c] = bi;
            }
            __syncthreads();
            if (!(s_best > 0.0)) {
                bad = c + 1;
                break;
            }
            const int r = s_r;
            if (r != c)
                for (int j = tid; j < p; j += kWT) {
                    double* a = M + (int64_t)c * p + j;
                    double* b = M + (int64_t)r * p + j;
                    const double t = *a;
                    *a = *b;
                    *b = t;
                }
            __syncthreads();
            const double pv = M[(int64_t)c * p + c];
            for (int j = tid; j < p; j += kWT) {
                s_row[j] = (j == c ? 1.0 : M[(int64_t)c * p + j]) / pv;
                s_col[j] = (j == c) ? 0.0 : M[(int64_t)j * p + c];
            }
            __syncthreads();
            for (int j = tid; j < p; j += kWT) M[(int64_t)c * p + j] = s_row[j];
            for (int r2 = w; r2 < p; r2 += kWW) {
                const double f = s_col[r2];
                if (f == 0.0) continue;                    // also skips row c
                double* Mi = M + (int64_t)r2 * p;
                // the row's loads (lane + 64 u, p <= 512) are all issued
                // before its stores
                double v[kWideMaxPs / PR_WAVE];
#pragma unroll
                for (int u = 0; u < kWideMaxPs / PR_WAVE; ++u) {
                    const int j = lane + PR_WAVE * u;
                    v[u] = Mi[j < p ? j : 0];
                }
#pragma unroll
                for (int u = 0; u < kWideMaxPs / PR_WAVE; ++u) {
                    const int j = lane + PR_WAVE * u;
                    if (j < p) Mi[j] = (j == c ? 0.0 : v[u]) - f * s_row[j];
                }
            }
            __syncthreads();
        }
        if (!bad) {
            for (int c = p - 1; c >= 0; --c) {
                const int r = s_piv[c];
                if (r == c) continue;
                for (int r2 = tid; r2 < p; r2 += kWT) {
                    double* a = M + (int64_t)r2 * p + c;
                    double* b = M + (int64_t)r2 * p + r;
                    const double t = *a;
                    *a = *b;
                    *b = t;
                }
                __syncthreads();
            }
        }
        if (tid == 0) info[i] = bad;
        __syncthreads();
    }
}

// Gauss-Jordan with the matrix in registers (p <= TR MA and p <= 32 MB):
// TR x 32 threads, thread (tr, tc) holding rows tr + TR a and columns
// tc + 32 b (block-cyclic, so every step keeps all threads busy).  Rows stay
// in place: step c takes as pivot the largest |M[r][c]| over the rows not yet
// used (lowest r on ties), divides row r by it (position c taking 1 / pivot)
// and takes M[i][c] times the new row r from every other row i (position c
// taking -M[i][c] / pivot).  Row r_c then holds row c of the inverse with its
// columns in pivot order: X[c][r_k] = M[r_c][k].  The pivot column and row
// reach every thread through LDS, so no step touches device memory, and
// register indices stay compile-time (a runtime row is matched against each
// slot by an unrolled comparison).
template <int TR, int MA, int MB>
__global__ __launch_bounds__(TR * 32) void k_gj_reg(int64_t count, const int32_t* __restrict__ list,
                                                    const int64_t* __restrict__ ptr, const double* __restrict__ tiles,
                                                    const int64_t* __restrict__ toff, int uniform_ps,
                                                    double* __restrict__ X, const int64_t* __restrict__ xoff,
                                                    int32_t* __restrict__ info) {
    __shared__ double s_col[TR * MA];
    __shared__ double s_raw[32 * MB];
    __shared__ double s_pv[TR];
    __shared__ int s_pi[TR];
    __shared__ int32_t s_piv[TR * MA];      // r_c
    __shared__ int32_t s_inv[TR * MA];      // c of row r_c
    __shared__ int s_r;
    __shared__ double s_best;
    const int tid = threadIdx.x, tc = tid & 31, tr = tid >> 5;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t k = list ? list[i] : i;
        const int p = ptr ? (int)(ptr[k + 1] - ptr[k]) : uniform_ps;
        const double* src = tiles + tile_off(k, p, toff, uniform_ps);
        double* M = X + (xoff ? xoff[i] : i * (int64_t)p * p);
        double m[MA][MB];
        // one row slot's loads at a time (the compiler barrier keeps all
        // MA MB loads, each with its address, from being in flight at once)
#pragma unroll
        for (int a = 0; a < MA; ++a) {
            const int r = tr + TR * a;
            const double* row = src + (int64_t)(r < p ? r : 0) * p;
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                const int c = tc + 32 * b;
                const bool ok = r < p && c < p;
                const double v = row[ok ? c : 0];
                m[a][b] = ok ? v : 0.0;
            }
            __asm__ volatile("" ::: "memory");
        }
        uint32_t used = 0;                  // bit a: row tr + TR a was a pivot
        int bad = 0;
        for (int c = 0; c < p; ++c) {
            const int cb = c >> 5, cc = c & 31;
            // pivot column to LDS (every row), then the TR owners pick their best
            if (tc == cc) {
                double bv = -1.0;
                int bi = INT_MAX;
#pragma unroll
                for (int a = 0; a < MA; ++a) {
                    const int r = tr + TR * a;
                    double v = 0.0;
#pragma unroll
                    for (int b = 0; b < MB; ++b) v = (b == cb) ? m[a][b] : v;
                    if (r < p) s_col[r] = v;
                    if (r < p && !((used >> a) & 1u) && fabs(v) > bv) {
                        bv = fabs(v);
                        bi = r;
                    }
                }
                s_pv[tr] = bv;
                s_pi[tr] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                double bv = s_pv[0];
                int bi = s_pi[0];
                for (int u = 1; u < TR; ++u)
                    if (s_pv[u] > bv || (s_pv[u] == bv && s_pi[u] < bi)) {
                        bv = s_pv[u];
                        bi = s_pi[u];
                    }
                s_r = bi;
                s_best = bv;
                s_piv[c] = bi;
                if (bi < p) s_inv[bi] = c;
            }
            __syncthreads();
            if (!(s_best > 0.0)) {
                bad = c + 1;
                break;
            }
            const int r = s_r;
            const int ra = r / TR, rr = r - ra * TR;
            if (tr == rr) {
#pragma unroll
                for (int a = 0; a < MA; ++a)
                    if (a == ra)
#pragma unroll
                        for (int b = 0; b < MB; ++b) s_raw[tc + 32 * b] = m[a][b];
                used |= 1u << ra;
            }
            __syncthreads();
            const double ipv = 1.0 / s_col[r];              // one division per step
            double rv[MB];
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                const int j = tc + 32 * b;
                rv[b] = j < p ? (j == c ? ipv : s_raw[j] * ipv) : 0.0;
            }
#pragma unroll
            for (int a = 0; a < MA; ++a) {
                const int row = tr + TR * a;
                if (row >= p) continue;
                if (row == r) {
#pragma unroll
                    for (int b = 0; b < MB; ++b) m[a][b] = rv[b];
                } else {
                    const double f = s_col[row];
#pragma unroll
                    for (int b = 0; b < MB; ++b) {
                        const int j = tc + 32 * b;
                        m[a][b] = (j == c ? 0.0 : m[a][b]) - f * rv[b];
                    }
                }
            }
            __syncthreads();                               // s_col, s_raw are rewritten next step
        }
        if (!bad) {
            // X[c][r_k] = M[r_c][k]: rows by s_inv, columns by s_piv
            int oc[MB];
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                const int c = tc + 32 * b;
                oc[b] = c < p ? s_piv[c] : 0;
            }
#pragma unroll
            for (int a = 0; a < MA; ++a) {
                const int r = tr + TR * a;
                double* row = M + (int64_t)(r < p ? s_inv[r] : 0) * p;
#pragma unroll
                for (int b = 0; b < MB; ++b)
                    if (r < p && tc + 32 * b < p) row[oc[b]] = m[a][b];
                __asm__ volatile("" ::: "memory");
            }
        }
        if (tid == 0) info[i] = bad;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// P = op(L) R for p x p row-major matrices in device memory on the FP64
// matrix cores: the block's waves take 32 x 32 output blocks round-robin,
// each four 16 x 16 x 4 products accumulated over k in steps of 4 (operand
// lanes: L element (row l % 16, k l / 16), R element (k l / 16, column
// l % 16); result lanes: rows l / 16 + 4 v of column l % 16).  TL: op(L) =
// L^T.  Padding rows, columns and k read clamped (valid) addresses times a
// 0/1 mask.  out(row, col, value) receives every element with row, col < p.
// ---------------------------------------------------------------------------
template <bool TL, class Out>
__device__ __forceinline__ void wg_mm(const double* __restrict__ L, const double* __restrict__ R, int p, Out out) {
    const int lane = threadIdx.x & (PR_WAVE - 1), w = threadIdx.x / PR_WAVE;
    const int li = lane & 15, lk = lane >> 4;
    const int nb = (p + 31) >> 5;
    for (int b = w; b < nb * nb; b += kWW) {
        const int bi = b / nb, bj = b - bi * nb;
        int ri[2], cj[2];
        double mr[2], mc[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int r = 32 * bi + 16 * t + li, c = 32 * bj + 16 * t + li;
            ri[t] = r < p ? r : 0;
            mr[t] = r < p ? 1.0 : 0.0;
            cj[t] = c < p ? c : 0;
            mc[t] = c < p ? 1.0 : 0.0;
        }
        wd4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[a][c] = wd4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < p; k0 += 4) {
            const int k = k0 + lk;
            const int kc = k < p ? k : 0;
            const double mk = k < p ? 1.0 : 0.0;
            double av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = (TL ? L[(int64_t)kc * p + ri[t]] : L[(int64_t)ri[t] * p + kc]) * (mk * mr[t]);
                bv[t] = R[(int64_t)kc * p + cj[t]] * (mk * mc[t]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int col = 32 * bj + 16 * c + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * bi + 16 * a + lk + 4 * v;
                    if (row < p && col < p) out(row, col, acc[a][c][v]);
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Algorithm 1, one round: entry m (patch U[0]) against the open patches
// U[1..nu]
// ---------------------------------------------------------------------------
// A pair is a candidate only when both patches have the same size.  Pruning
// (d can only be larger than the bound, so the pair cannot match):
//   l1:        d = sum |A - B| >= |sum|A| - sum|B||
//   Frobenius: d = ||A - B||_F >= | ||A||_F - ||B||_F |
//   spectral:  d = ||(B - A) B^{-1}||_2 >= ||B - A||_2 / ||B||_2
//                >= | ||A||_F - ||B||_F | / (sqrt(p) ||B||_F)
// each with a relative slack of kGapSlack for the rounding of the norms.
__device__ __forceinline__ bool a1w_pruned(int crit, double eps, double nA, double nB, int p) {
    const double gap = fabs(nA - nB) - kGapSlack * (nA + nB);
    if (crit == PR_CRIT_SPECTRAL) return gap > sqrt((double)p) * nB * eps * (1.0 + kGapSlack);
    return gap > eps * (1.0 + kGapSlack);
}

__global__ __launch_bounds__(kWT) void k_a1w_entrywise(int64_t nu, const int32_t* __restrict__ U, int32_t m,
                                                       int crit, double eps, const int64_t* __restrict__ ptr,
                                                       const double* __restrict__ tiles,
                                                       const int64_t* __restrict__ toff, int uniform_ps,
                                                       const double* __restrict__ keynorm,
                                                       int32_t* __restrict__ phi, int64_t* __restrict__ keep,
                                                       unsigned long long* counters) {
    __shared__ double sred[kWW];
    const int32_t ks = U[0];
    const int pk = (int)(ptr[ks + 1] - ptr[ks]);
    const double* B = tiles + tile_off(ks, pk, toff, uniform_ps);
    const double nB = keynorm[ks];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        phi[ks] = m;
        keep[nu] = 0;
    }
    for (int64_t u = blockIdx.x; u < nu; u += gridDim.x) {
        const int32_t k = U[1 + u];
        const int p = (int)(ptr[k + 1] - ptr[k]);
        if (p != pk) {                                      // other size: no candidate
            if (threadIdx.x == 0) keep[u] = 1;
            continue;
        }
        if (a1w_pruned(crit, eps, keynorm[k], nB, p)) {
            if (threadIdx.x == 0) {
                keep[u] = 1;
                atomicAdd(&counters[1], 1ull);
            }
            continue;
        }
        const double* A = tiles + tile_off(k, p, toff, uniform_ps);
        double s = 0.0;
        for (int e = threadIdx.x; e < p * p; e += kWT) {
            const double d = A[e] - B[e];
            s += (crit == PR_CRIT_L1) ? fabs(d) : d * d;
        }
        s = block_sum(s, sred);
        const double dv = (crit == PR_CRIT_L1) ? s : sqrt(s);
        if (threadIdx.x == 0) {
            const bool match = dv < eps;
            keep[u] = match ? 0 : 1;
            if (match) phi[k] = m;
            atomicAdd(&counters[0], 1ull);
        }
    }
}

// Spectral criterion d = ||I - A X||_2 with X = B^{-1}.  E = I - A X goes to
// the block's scratch; sigma_max(E)^2 lies in [largest squared column norm,
// ||E||_F^2].  When eps^2 is inside, G = E^T E is formed and N_0 = G / c
// (c = ||E||_F^2) squared repeatedly, N_k = N_{k-1}^2 / tr(N_{k-1}^2):
// with U_k = log c + sum_{i<=k} log tr(N_{i-1}^2) / 2^i,
//   log lambda_1 <= U_k                         (tr of a PSD power),
//   log lambda_1 >= U_k + log max_j (N_k)_jj / 2^k (largest diagonal entry),
// a bracket of width at most 2 log(p) / 2^k.  After kSquaringsWide steps an
// open bracket (d within about 1e-11 of eps) is decided at its geometric
// midpoint (counted in counters[3]).
__global__ __launch_bounds__(kWT) void k_a1w_spectral(int64_t nu, const int32_t* __restrict__ U, int32_t m,
                                                      double eps, const int64_t* __restrict__ ptr,
                                                      const double* __restrict__ tiles,
                                                      const int64_t* __restrict__ toff, int uniform_ps,
                                                      const double* __restrict__ fnorm,
                                                      const double* __restrict__ Xm, double* __restrict__ scratch,
                                                      int pmax, int32_t* __restrict__ phi,
                                                      int64_t* __restrict__ keep, unsigned long long* counters) {
    __shared__ double sred[kWW];
    const int32_t ks = U[0];
    const int pk = (int)(ptr[ks + 1] - ptr[ks]);
    const double nB = fnorm[ks];
    const double e2 = eps * eps;
    double* E = scratch + (int64_t)blockIdx.x * 2 * pmax * pmax;
    double* H = E + (int64_t)pmax * pmax;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        phi[ks] = m;
        keep[nu] = 0;
    }
    for (int64_t u = blockIdx.x; u < nu; u += gridDim.x) {
        const int32_t k = U[1 + u];
        const int p = (int)(ptr[k + 1] - ptr[k]);
        if (p != pk) {
            if (threadIdx.x == 0) keep[u] = 1;
            continue;
        }
        if (a1w_pruned(PR_CRIT_SPECTRAL, eps, fnorm[k], nB, p)) {
            if (threadIdx.x == 0) {
                keep[u] = 1;
                atomicAdd(&counters[1], 1ull);
            }
            continue;
        }
        const double* A = tiles + tile_off(k, p, toff, uniform_ps);
        wg_mm<false>(A, Xm, p, [&](int r, int c, double v) { E[(int64_t)r * p + c] = (r == c ? 1.0 : 0.0) - v; });
        __syncthreads();
        double cmax = 0.0, fro = 0.0;
        for (int c = threadIdx.x; c < p; c += kWT) {
            double s = 0.0;
            for (int r = 0; r < p; ++r) {
                const double v = E[(int64_t)r * p + c];
                s += v * v;
            }
            cmax = fmax(cmax, s);
            fro += s;
        }
        double lo2 = block_max(cmax, sred);
        double hi2 = block_sum(fro, sred);
        const double c0 = hi2;
        bool match = hi2 < e2;
        bool open = !match && !(lo2 >= e2);
        if (open) {
            if (threadIdx.x == 0) atomicAdd(&counters[2], 1ull);
            const double ic = 1.0 / c0;
            wg_mm<true>(E, E, p, [&](int r, int c, double v) { H[(int64_t)r * p + c] = v * ic; });
            __syncthreads();
            double Uk = log(c0), wk = 0.5;
            double* cur = H;
            double* nxt = E;
            for (int it = 1; it <= kSquaringsWide && open; ++it) {
                double tr = 0.0, md = 0.0;
                wg_mm<true>(cur, cur, p, [&](int r, int c, double v) {
                    nxt[(int64_t)r * p + c] = v;
                    if (r == c) {
                        tr += v;
                        md = fmax(md, v);
                    }
                });
                tr = block_sum(tr, sred);
                md = block_max(md, sred);
                const double it_ = 1.0 / tr;
                for (int64_t e = threadIdx.x; e < (int64_t)p * p; e += kWT) nxt[e] *= it_;
                __syncthreads();
                Uk += wk * log(tr);
                hi2 = fmin(hi2, exp(Uk));
                lo2 = fmax(lo2, exp(Uk + wk * log(md * it_)));
                wk *= 0.5;
                double* t = cur;
                cur = nxt;
                nxt = t;
                if (hi2 < e2) {
                    match = true;
                    open = false;
                } else if (lo2 >= e2) {
                    open = false;
                }
            }
            if (open) {
                match = sqrt(lo2) * sqrt(hi2) < e2;
                if (threadIdx.x == 0) atomicAdd(&counters[3], 1ull);
            }
        }
        if (threadIdx.x == 0) {
            keep[u] = match ? 0 : 1;
            if (match) phi[k] = m;
            atomicAdd(&counters[0], 1ull);
        }
        __syncthreads();                                   // E and H are rewritten by the next pair
    }
}

__global__ void k_a1w_compact(int64_t nu, const int32_t* __restrict__ U, const int64_t* __restrict__ keep,
                              const int64_t* __restrict__ excl, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu && keep[i]) out[excl[i]] = U[i];
}

// column-major copy of every entry, 32 x 32 tiles through LDS
__global__ __launch_bounds__(kWT) void k_transpose_db(int64_t m_p, const double* __restrict__ db,
                                                      const int64_t* __restrict__ dboff,
                                                      const int32_t* __restrict__ dbps,
                                                      double* __restrict__ out64, float* __restrict__ out32) {
    __shared__ double st[32][33];
    for (int64_t j = blockIdx.x; j < m_p; j += gridDim.x) {
        const int p = dbps[j];
        const int64_t off = dboff[j];
        const int nt = (p + 31) >> 5;
        for (int t = 0; t < nt * nt; ++t) {
            const int ta = t / nt, tc = t - ta * nt;
            for (int e = threadIdx.x; e < 1024; e += kWT) {
                const int a = 32 * ta + (e >> 5), c = 32 * tc + (e & 31);
                st[e >> 5][e & 31] = (a < p && c < p) ? db[off + (int64_t)a * p + c] : 0.0;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < 1024; e += kWT) {
                const int c = 32 * tc + (e >> 5), a = 32 * ta + (e & 31);
                if (a < p && c < p) {
                    const double v = st[e & 31][e >> 5];
                    if (out64) out64[off + (int64_t)c * p + a] = v;
                    if (out32) out32[off + (int64_t)c * p + a] = (float)v;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
// Slot of local row a of grouped patch s (the layout of the two-stage
// scatter: tiles of 16 patches, row-plane by row-plane)
__device__ __forceinline__ int64_t yslot_w(int64_t s, int a, int pmax) {
    return (((s >> 4) * pmax + a) << 4) + (s & 15);
}

__device__ __forceinline__ int64_t goff_of(const int64_t* goff, int pst, int64_t s) {
    return goff ? goff[s] : s * (int64_t)pst;
}

struct WideGeom {
    const int32_t* gdofs;
    const int64_t* goff;
    int pst;
    const int32_t* gphi;
    const int64_t* dboff;
    const int32_t* stop;
    int ypm;
};

template <typename T>
__device__ __forceinline__ void mfma_w(T a, T b, wd4& acc);
template <>
__device__ __forceinline__ void mfma_w<double>(double a, double b, wd4& acc) {
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// Work unit (item, row range): the item is (entry j, grouped positions
// start .. start + cnt - 1, cnt <= 16, p) and the range 64 rows of
// Y = X_j R, one 16-row block per wave, on the FP64 matrix cores (16 x 16 x 4
// products).  R, the members' restricted residuals, is staged in LDS k-major
// (16 members per row, stride kRStride, rows to a multiple of 32, zero past
// p), gathered in two phases (eight dof indices per thread, then their eight
// values).  Each wave streams its 16 rows of X_j^T (the column-major
// database: 16 consecutive values per k) from L2 eight k-steps at a time, so
// eight loads are in flight before their products, and sums even and odd
// k-steps in two chains.  FP32 storage: X_j and the residual are FP32
// values, widened exactly, and the products accumulate in FP64.  Output
// lanes hold rows l / 16 + 4 v of member l % 16.
constexpr int kRowsPerUnit = 64;

__host__ __device__ inline size_t wide_apply_lds(int pmax) {
    return (size_t)((pmax + 31) & ~31) * kRStride * sizeof(double);
}

template <typename TX, bool TWO>
__global__ __launch_bounds__(kWT) void k_apply_wide_mfma(const int32_t* __restrict__ items, int64_t n_items,
                                                         int nrange, WideGeom g, const TX* __restrict__ dbt,
                                                         const double* __restrict__ W, double omega,
                                                         const double* __restrict__ r, double* __restrict__ z,
                                                         TX* __restrict__ Y) {
    extern __shared__ double sR[];
    if (g.stop && *g.stop) return;
    const int tid = threadIdx.x, lane = tid & (PR_WAVE - 1), w = tid / PR_WAVE;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t units = n_items * nrange;
    for (int64_t bi = blockIdx.x; bi < units; bi += gridDim.x) {
        const int64_t it = bi / nrange;
        const int row0 = (int)(bi - it * nrange) * kRowsPerUnit;
        const int j = items[4 * it], start = items[4 * it + 1], cnt = items[4 * it + 2], p = items[4 * it + 3];
        if (row0 >= p) continue;                           // the same for the whole block
        const int p32 = (p + 31) & ~31;
        const int tot = 16 * p32;
        for (int base = 0; base < tot; base += 8 * kWT) {
            int32_t gi[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + tid + u * kWT;
                const int mbr = e / p32, k = e - mbr * p32;
                const bool ok = e < tot && mbr < cnt && k < p;
                gi[u] = ok ? g.gdofs[goff_of(g.goff, g.pst, start + mbr) + k] : -1;
            }
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double x = r[gi[u] >= 0 ? gi[u] : 0];
                v[u] = gi[u] >= 0 ? x : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + tid + u * kWT;
                if (e < tot) {
                    const int mbr = e / p32, k = e - mbr * p32;
                    double x = v[u];
                    if constexpr (sizeof(TX) == 4) x = (double)(float)x;   // FP32 operands
                    sR[k * kRStride + mbr] = x;
                }
            }
        }
        __syncthreads();
        const int rb0 = row0 + 16 * w;
        if (rb0 < p) {                                     // the same for the whole wave
            const TX* XT = dbt + g.dboff[j];
            const int row = rb0 + li;
            const int rc = row < p ? row : 0;
            wd4 acc0 = wd4{0.0, 0.0, 0.0, 0.0}, acc1 = wd4{0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < p32; k0 += 32) {
                double av[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = k0 + 4 * u + lk;
                    const int kc = k < p ? k : 0;              // k past p meets staged zeros
                    av[u] = (double)XT[(int64_t)kc * p + rc];
                    bv[u] = sR[k * kRStride + li];
                }
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    mfma_w<double>(av[u], bv[u], acc0);
                    mfma_w<double>(av[u + 1], bv[u + 1], acc1);
                }
            }
            if (li < cnt) {
                const int64_t s = start + li;
                const int64_t o = goff_of(g.goff, g.pst, s);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int orow = rb0 + lk + 4 * v;
                    const double y = acc0[v] + acc1[v];
                    if (orow < p) {
                        if (TWO) {
                            Y[yslot_w(s, orow, g.ypm)] = (TX)y;
                        } else {
                            const int32_t gd = g.gdofs[o + orow];
                            atomicAdd(&z[gd], omega * W[gd] * y);
                        }
                    }
                }
            }
        }
        __syncthreads();                                   // sR is restaged by the next unit
    }
}

// One grouped position per block: y[a] = sum_k X^T[k][a] r_k with the
// restricted residual in LDS and X^T streamed (coalesced over a).
template <typename TX, bool TWO>
__global__ __launch_bounds__(kWT) void k_apply_wide_vec(int64_t n_p, WideGeom g, const TX* __restrict__ dbt,
                                                        const double* __restrict__ W, double omega,
                                                        const double* __restrict__ r, double* __restrict__ z,
                                                        TX* __restrict__ Y) {
    __shared__ double sr[kWideMaxPs];
    if (g.stop && *g.stop) return;
    const int tid = threadIdx.x;
    for (int64_t s = blockIdx.x; s < n_p; s += gridDim.x) {
        const int64_t o = goff_of(g.goff, g.pst, s);
        const int p = g.goff ? (int)(g.goff[s + 1] - o) : g.pst;
        for (int k = tid; k < p; k += kWT) {
            const double v = r[g.gdofs[o + k]];
            sr[k] = sizeof(TX) == 4 ? (double)(float)v : v;          // FP32 operands
        }
        __syncthreads();
        const TX* XT = dbt + g.dboff[g.gphi[s]];
        for (int a = tid; a < p; a += kWT) {
            double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
            int k = 0;
            for (; k + 4 <= p; k += 4) {
                acc0 = fma((double)XT[(int64_t)k * p + a], sr[k], acc0);
                acc1 = fma((double)XT[(int64_t)(k + 1) * p + a], sr[k + 1], acc1);
                acc2 = fma((double)XT[(int64_t)(k + 2) * p + a], sr[k + 2], acc2);
                acc3 = fma((double)XT[(int64_t)(k + 3) * p + a], sr[k + 3], acc3);
            }
            for (; k < p; ++k) acc0 = fma((double)XT[(int64_t)k * p + a], sr[k], acc0);
            const double acc = (acc0 + acc1) + (acc2 + acc3);
            if (TWO) {
                Y[yslot_w(s, a, g.ypm)] = (TX)acc;
            } else {
                const int32_t gd = g.gdofs[o + a];
                atomicAdd(&z[gd], omega * W[gd] * acc);
            }
        }
        __syncthreads();
    }
}

inline unsigned grid_of(int64_t work, int64_t cap) {
    return (unsigned)(work < 1 ? 1 : (work < cap ? work : cap));
}

}  // namespace

void launch_validate_wide(const int64_t* ptr, const int32_t* dofs, int64_t n_p, int64_t n, int32_t* flags,
                          hipStream_t s) {
    if (n_p <= 0) return;
    k_validate_wide<<<grid_of(n_p, 8192), kWT, 0, s>>>(ptr, dofs, n_p, n, flags);
}

void launch_extract_wide(const int64_t* rowptr, const int32_t* col, const double* val, const int64_t* ptr,
                         const int32_t* dofs, int64_t n_p, const int64_t* toff, int uniform_ps, double* tiles,
                         uint32_t* keys, double* fnorm, double* l1norm, int32_t* flags, hipStream_t s) {
    if (n_p <= 0) return;
    k_extract_wide<<<grid_of(n_p, 8192), kWT, 0, s>>>(rowptr, col, val, ptr, dofs, n_p, toff, uniform_ps, tiles,
                                                       keys, fnorm, l1norm, flags);
}

void launch_gj_wide(int64_t count, const int32_t* list, const int64_t* ptr, const double* tiles,
                    const int64_t* toff, int uniform_ps, int pmax, double* X, const int64_t* xoff, int32_t* info,
                    hipStream_t s) {
    if (count <= 0) return;
    // the matrix in registers up to 216 dofs (Experiment 3's size), in device memory above
    const unsigned nb = grid_of(count, 4096);
    if (pmax <= 128)
        k_gj_reg<16, 8, 4><<<nb, 512, 0, s>>>(count, list, ptr, tiles, toff, uniform_ps, X, xoff, info);
    else if (pmax <= 192)
        k_gj_reg<32, 6, 6><<<nb, 1024, 0, s>>>(count, list, ptr, tiles, toff, uniform_ps, X, xoff, info);
    else if (pmax <= 216)
        k_gj_reg<24, 9, 7><<<nb, 768, 0, s>>>(count, list, ptr, tiles, toff, uniform_ps, X, xoff, info);
    else
        k_gj_wide<<<nb, kWT, 0, s>>>(count, list, ptr, tiles, toff, uniform_ps, X, xoff, info);
}

int64_t a1w_spectral_grid(int64_t nu) { return nu < 1 ? 1 : (nu < 512 ? nu : 512); }

void launch_a1w_round(int64_t nu, const int32_t* U, int32_t m, int crit, double eps, const int64_t* ptr,
                      const double* tiles, const int64_t* toff, int uniform_ps, const double* fnorm,
                      const double* l1norm, const double* Xm, double* scratch, int64_t grid, int pmax,
                      int32_t* phi, int64_t* keep, unsigned long long* counters, hipStream_t s) {
    if (crit == PR_CRIT_SPECTRAL) {
        k_a1w_spectral<<<(unsigned)grid, kWT, 0, s>>>(nu, U, m, eps, ptr, tiles, toff, uniform_ps, fnorm, Xm,
                                                      scratch, pmax, phi, keep, counters);
    } else {
        const double* keynorm = crit == PR_CRIT_L1 ? l1norm : fnorm;
        k_a1w_entrywise<<<grid_of(nu, 4096), kWT, 0, s>>>(nu, U, m, crit, eps, ptr, tiles, toff, uniform_ps,
                                                          keynorm, phi, keep, counters);
    }
}

void launch_a1w_compact(int64_t nu, const int32_t* U, const int64_t* keep, const int64_t* excl, int32_t* out,
                        hipStream_t s) {
    if (nu <= 0) return;
    k_a1w_compact<<<(unsigned)((nu + 255) / 256), 256, 0, s>>>(nu, U, keep, excl, out);
}

void launch_transpose_db(int64_t m_p, const double* db, const int64_t* dboff, const int32_t* dbps,
                         double* out64, float* out32, hipStream_t s) {
    if (m_p <= 0) return;
    k_transpose_db<<<grid_of(m_p, 8192), kWT, 0, s>>>(m_p, db, dboff, dbps, out64, out32);
}

void launch_apply_wide(int prec, bool two_stage, const ApplyLaunch& a, hipStream_t s) {
    WideGeom g{a.gdofs, a.goff, a.pst, a.gphi, a.dboff, a.stop, a.maxp};
    const int64_t cap = a.grid_cap > 0 ? a.grid_cap : 65536;
    if (a.wide == 2) {
        const unsigned nb = grid_of(a.n_p, cap);
        if (prec == PR_FP64) {
            if (two_stage) k_apply_wide_vec<double, true><<<nb, kWT, 0, s>>>(a.n_p, g, a.db_t, a.W, a.omega, a.r, a.z, (double*)a.Y);
            else k_apply_wide_vec<double, false><<<nb, kWT, 0, s>>>(a.n_p, g, a.db_t, a.W, a.omega, a.r, a.z, (double*)nullptr);
        } else {
            if (two_stage) k_apply_wide_vec<float, true><<<nb, kWT, 0, s>>>(a.n_p, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)a.Y);
            else k_apply_wide_vec<float, false><<<nb, kWT, 0, s>>>(a.n_p, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)nullptr);
        }
        return;
    }
    if (a.n_items <= 0) return;
    const int nrange = (a.maxp + kRowsPerUnit - 1) / kRowsPerUnit;
    const unsigned nb = grid_of(a.n_items * nrange, cap);
    const size_t lds = wide_apply_lds(a.maxp);
    static bool lds_set = false;                           // above 64 KB from p = 481
    if (!lds_set) {
        const int most = (int)wide_apply_lds(kWideMaxPs);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_wide_mfma<double, true>), hipFuncAttributeMaxDynamicSharedMemorySize, most);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_wide_mfma<double, false>), hipFuncAttributeMaxDynamicSharedMemorySize, most);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_wide_mfma<float, true>), hipFuncAttributeMaxDynamicSharedMemorySize, most);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_wide_mfma<float, false>), hipFuncAttributeMaxDynamicSharedMemorySize, most);
        lds_set = true;
    }
    if (prec == PR_FP64) {
        if (two_stage) k_apply_wide_mfma<double, true><<<nb, kWT, lds, s>>>(a.items, a.n_items, nrange, g, a.db_t, a.W, a.omega, a.r, a.z, (double*)a.Y);
        else k_apply_wide_mfma<double, false><<<nb, kWT, lds, s>>>(a.items, a.n_items, nrange, g, a.db_t, a.W, a.omega, a.r, a.z, (double*)nullptr);
    } else {
        if (two_stage) k_apply_wide_mfma<float, true><<<nb, kWT, lds, s>>>(a.items, a.n_items, nrange, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)a.Y);
        else k_apply_wide_mfma<float, false><<<nb, kWT, lds, s>>>(a.items, a.n_items, nrange, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)nullptr);
    }
}
