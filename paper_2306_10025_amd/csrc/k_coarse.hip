// Two-level combination preconditioner (Eq.(2)) on the device:
//   M_combo^{-1} r = M~^{-1} r + P0 A0^{-1} R0 r,   R0 = P0^T,  A0 = R0 A P0,
// with A0 solved directly, as in the first two numerical experiments.
//
// Setup: R0 by a transpose of P0; A0 = R0 (A P0) in two sparse products, one
// row per wavefront each, with a fixed summation order per entry
// (deterministic); then a direct solver:
//  - small A0 (dense form): its explicit inverse;
//  - otherwise A0 is banded (|v - w| <= b for every entry), so with blocks of
//    s >= b rows it is block tridiagonal, and block LU without pivoting across
//    blocks (A0 is symmetric positive definite for the diffusion problems)
//    keeps the inverses of the Schur complements
//        S_0 = D_0,  S_i = D_i - L_i S_{i-1}^{-1} U_{i-1},
//    where D_i, L_i, U_i are the diagonal, sub- and super-diagonal blocks.
//  Dense inverses: blocked Gauss-Jordan in place, 32-wide panels, the rank-32
//  updates on the FP64 matrix cores (16 x 16 x 4 MFMA), partial pivoting
//  inside each 32 x 32 pivot block (Gauss-Jordan in registers).
// The banded form also keeps G_i = S_i^{-1} L_i and H_i = S_i^{-1} U_i, so
// that the sequential sweeps are dense matrix-vector products only.
// Apply: r0 = R0 r; u_i = S_i^{-1} r0_i for every block at once; forward
// sweep w_i = u_i - G_i w_{i-1}; backward sweep x_i = w_i - H_i x_{i+1};
// z += P0 x.  Every kernel returns at once when the solve's stop flag is set
// (graph replays).
#include "dense_dev.h"

#include <climits>

namespace {

using namespace pr_dev;

inline unsigned nbk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__device__ __forceinline__ bool stopped(const int32_t* stop) { return stop && *stop; }

// ---- interpolation checks ----------------------------------------------------
// flags[0]: row_ptr not monotone or wrong ends; [1]: column out of [0, n0);
// [2]: non-finite value
__global__ void k_interp_check(int64_t n, int64_t n0, int64_t nnz, const int64_t* __restrict__ rp,
                               const int32_t* __restrict__ ci, const double* __restrict__ v,
                               int32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) flags[0] = 1;
    if (i >= n) return;
    const int64_t a = rp[i], b = rp[i + 1];
    if (b < a || a < 0 || b > nnz) {
        flags[0] = 1;
        return;
    }
    for (int64_t e = a; e < b; ++e) {
        const int32_t c = ci[e];
        if (c < 0 || c >= n0) flags[1] = 1;
        if (!isfinite(v[e])) flags[2] = 1;
    }
}

// ---- transpose of a CSR matrix (n rows, m columns) --------------------------
__global__ void k_tr_count(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           int64_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) atomicAdd((unsigned long long*)&cnt[ci[e]], 1ull);
}

__global__ void k_tr_fill(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ v, const int64_t* __restrict__ tp,
                          int64_t* __restrict__ fill, int32_t* __restrict__ tc, double* __restrict__ tv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t c = ci[e];
        const int64_t pos = tp[c] + (int64_t)atomicAdd((unsigned long long*)&fill[c], 1ull);
        tc[pos] = (int32_t)i;
        tv[pos] = v[e];
    }
}

// Rows of the transpose in ascending column.  The fill order depends on
// timing, so each row is rewritten from the filled copy (uc, uv) by rank, one
// wavefront per row: an entry's rank is the number of entries before it in
// (column, value bits, position) order.  Equal columns come only from a
// column repeated within one input row; the value bits then order them, and
// entries equal in both are interchangeable, so the row is the same whatever
// the fill order.  Quadratic in the row length, read from the cache.
__global__ __launch_bounds__(256) void k_tr_rank(int64_t m, const int64_t* __restrict__ tp,
                                                 const int32_t* __restrict__ uc, const double* __restrict__ uv,
                                                 int32_t* __restrict__ tc, double* __restrict__ tv) {
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / PR_WAVE) + threadIdx.x / PR_WAVE;
    const int lane = threadIdx.x & (PR_WAVE - 1);
    if (r >= m) return;
    const int64_t a = tp[r], len = tp[r + 1] - a;
    for (int64_t e = lane; e < len; e += PR_WAVE) {
        const int32_t c = uc[a + e];
        const double v = uv[a + e];
        const unsigned long long vb = (unsigned long long)__double_as_longlong(v);
        int64_t rk = 0;
        for (int64_t f = 0; f < len; ++f) {
            const int32_t cf = uc[a + f];
            if (cf == c) {
                const unsigned long long fb = (unsigned long long)__double_as_longlong(uv[a + f]);
                rk += (fb < vb || (fb == vb && f < e)) ? 1 : 0;
            } else {
                rk += cf < c ? 1 : 0;
            }
        }
        tc[a + rk] = c;
        tv[a + rk] = v;
    }
}

// ---- Galerkin product A0 = R0 A P0, one wavefront per coarse row -------------
constexpr int kGalSlots = 256;   // distinct coarse columns one coarse row may reach

__device__ __forceinline__ int gal_hash(int32_t w) { return (int)(((uint32_t)w * 2654435761u) >> 24); }

// Row v of A0 from the lane-owned sums acc[q] of the columns of rank
// q * 64 + lane (nk columns, ascending in sorted[]): entries at most drop
// times the row's largest magnitude are dropped (rounding residue of couplings
// that vanish exactly); the rest go to out + v * kGalSlots in column order.
__device__ __forceinline__ void gal_emit(const double (&acc)[kGalSlots / PR_WAVE], int nk,
                                         const int32_t* sorted, double drop, int64_t v, int32_t* ocnt,
                                         int32_t* ocol, double* oval) {
    constexpr int Q = kGalSlots / PR_WAVE;
    const int lane = threadIdx.x & (PR_WAVE - 1);
    double mx = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (q * PR_WAVE + lane < nk) mx = fmax(mx, fabs(acc[q]));
    mx = wave_max(mx);
    const double lim = drop * mx;
    int base = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = q * PR_WAVE + lane;
        const bool keep = r < nk && fabs(acc[q]) > lim;
        const unsigned long long m = __ballot(keep);
        if (keep) {
            const int pos = base + __popcll(m & below);
            ocol[v * kGalSlots + pos] = sorted[r];
            oval[v * kGalSlots + pos] = acc[q];
        }
        base += __popcll(m);
    }
    if (lane == 0) ocnt[v] = base;
}

// Pass 1 collects the coarse columns w reachable from row v (R0 row v, then A
// rows, then P0 rows) in an LDS hash set; they are ranked in ascending order.
// Pass 2: lane l owns the columns of rank l, l + 64, ...; every lane walks the
// same stream of products r_vi a_ij p_jw in the same order and adds those of
// its columns, so each entry is summed in one fixed order.  The general form,
// for interpolations whose rows of A P0 reach more than kApSlots columns.
__global__ __launch_bounds__(64) void k_galerkin(
    int64_t n0, const int64_t* __restrict__ rrp, const int32_t* __restrict__ rci, const double* __restrict__ rv,
    const int64_t* __restrict__ arp, const int32_t* __restrict__ aci, const double* __restrict__ av,
    const int64_t* __restrict__ prp, const int32_t* __restrict__ pci, const double* __restrict__ pv,
    double drop, int32_t* __restrict__ ocnt, int32_t* __restrict__ ocol, double* __restrict__ oval,
    int32_t* __restrict__ overflow) {
    __shared__ int32_t keys[kGalSlots];
    __shared__ int32_t rank[kGalSlots];
    __shared__ int32_t sorted[kGalSlots];
    const int lane = threadIdx.x;
    constexpr int Q = kGalSlots / PR_WAVE;
    for (int64_t v = blockIdx.x; v < n0; v += gridDim.x) {
        for (int s = lane; s < kGalSlots; s += PR_WAVE) keys[s] = -1;
        __syncthreads();
        bool over = false;
        const int64_t r0 = rrp[v], r1 = rrp[v + 1];
        for (int64_t er = r0; er < r1; ++er) {
            const int32_t i = rci[er];
            for (int64_t ea = arp[i] + lane; ea < arp[i + 1]; ea += PR_WAVE) {
                const int32_t j = aci[ea];
                for (int64_t ep = prp[j]; ep < prp[j + 1]; ++ep) {
                    const int32_t w = pci[ep];
                    int h = gal_hash(w);
                    int probes = 0;
                    while (true) {
                        const int32_t old = atomicCAS(&keys[h], -1, w);
                        if (old == -1 || old == w) break;
                        h = (h + 1) & (kGalSlots - 1);
                        if (++probes >= kGalSlots) {
                            over = true;
                            break;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (__ballot(over)) {
            if (lane == 0) atomicOr(overflow, 1);
            if (lane == 0) ocnt[v] = 0;
            __syncthreads();
            continue;
        }
        // rank of every present key
        int nk = 0;
        for (int s = lane; s < kGalSlots; s += PR_WAVE) {
            const int32_t k = keys[s];
            int r = -1;
            if (k >= 0) {
                r = 0;
                for (int t = 0; t < kGalSlots; ++t) {
                    const int32_t o = keys[t];
                    r += (o >= 0 && o < k) ? 1 : 0;
                }
                sorted[r] = k;
                ++nk;
            }
            rank[s] = r;
        }
        nk = wave_sum(nk);
        __syncthreads();
        // pass 2: owned accumulators
        double acc[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] = 0.0;
        for (int64_t er = r0; er < r1; ++er) {
            const int32_t i = rci[er];
            const double ri = rv[er];
            for (int64_t ea = arp[i]; ea < arp[i + 1]; ++ea) {
                const int32_t j = aci[ea];
                const double ra = ri * av[ea];
                for (int64_t ep = prp[j]; ep < prp[j + 1]; ++ep) {
                    const int32_t w = pci[ep];
                    int h = gal_hash(w);
                    while (keys[h] != w) h = (h + 1) & (kGalSlots - 1);
                    const int rk = rank[h];
                    const double t = ra * pv[ep];
#pragma unroll
                    for (int q = 0; q < Q; ++q) acc[q] += (rk == q * PR_WAVE + lane) ? t : 0.0;
                }
            }
        }
        gal_emit(acc, nk, sorted, drop, v, ocnt, ocol, oval);
        __syncthreads();
    }
}

// ---- Galerkin product in two products: B = A P0, then A0 = R0 B ------------
constexpr int kApSlots = 32;      // distinct coarse columns one row of A P0 may reach
constexpr int kApHash = 2 * kApSlots;

__device__ __forceinline__ int ap_hash(int32_t w) { return (int)(((uint32_t)w * 2654435761u) >> 26); }

// B = A P0, one wavefront per fine row i.  Pass 1 collects the row's coarse
// columns (the P0 rows of A's columns) in an LDS hash set and ranks them.
// Pass 2: lane l takes A's entries l, l + 64, ... and adds a_ij p_jw into its
// own partial of column w; lane s then adds the 64 partials of the column of
// rank s in lane order, so each entry is summed in one fixed order.  Output:
// row i at out + i * kApSlots, columns ascending, bcnt[i] of them; a row with
// more than kApSlots columns sets *overflow (and writes bcnt[i] = 0).
__global__ __launch_bounds__(64) void k_ap(int64_t n, const int64_t* __restrict__ arp,
                                           const int32_t* __restrict__ aci, const double* __restrict__ av,
                                           const int64_t* __restrict__ prp, const int32_t* __restrict__ pci,
                                           const double* __restrict__ pv, int32_t* __restrict__ bcnt,
                                           int32_t* __restrict__ bcol, double* __restrict__ bval,
                                           int32_t* __restrict__ overflow) {
    __shared__ int32_t keys[kApHash];
    __shared__ int32_t rank[kApHash];
    __shared__ int32_t sorted[kApSlots];
    __shared__ double part[kApSlots * PR_WAVE];
    const int lane = threadIdx.x;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        for (int t = lane; t < kApHash; t += PR_WAVE) keys[t] = -1;
        __syncthreads();
        const int64_t a0 = arp[i], a1 = arp[i + 1];
        bool over = false;
        for (int64_t ea = a0 + lane; ea < a1; ea += PR_WAVE) {
            const int32_t j = aci[ea];
            for (int64_t ep = prp[j]; ep < prp[j + 1]; ++ep) {
                const int32_t w = pci[ep];
                int h = ap_hash(w);
                int probes = 0;
                while (true) {
                    const int32_t old = atomicCAS(&keys[h], -1, w);
                    if (old == -1 || old == w) break;
                    h = (h + 1) & (kApHash - 1);
                    if (++probes >= kApHash) {
                        over = true;
                        break;
                    }
                }
            }
        }
        __syncthreads();
        int nk = 0;
        for (int t = lane; t < kApHash; t += PR_WAVE) {
            const int32_t k = keys[t];
            int r = -1;
            if (k >= 0) {
                r = 0;
                for (int u = 0; u < kApHash; ++u) {
                    const int32_t o = keys[u];
                    r += (o >= 0 && o < k) ? 1 : 0;
                }
                if (r < kApSlots) sorted[r] = k;
                ++nk;
            }
            rank[t] = r;
        }
        nk = wave_sum(nk);
        if (__ballot(over) || nk > kApSlots) {
            if (lane == 0) {
                atomicOr(overflow, 1);
                bcnt[i] = 0;
            }
            __syncthreads();
            continue;
        }
        for (int r = 0; r < nk; ++r) part[r * PR_WAVE + lane] = 0.0;
        __syncthreads();
        for (int64_t ea = a0 + lane; ea < a1; ea += PR_WAVE) {
            const int32_t j = aci[ea];
            const double aij = av[ea];
            for (int64_t ep = prp[j]; ep < prp[j + 1]; ++ep) {
                const int32_t w = pci[ep];
                int h = ap_hash(w);
                while (keys[h] != w) h = (h + 1) & (kApHash - 1);
                part[rank[h] * PR_WAVE + lane] += aij * pv[ep];
            }
        }
        __syncthreads();
        if (lane < nk) {
            double sum = 0.0;
            for (int l = 0; l < PR_WAVE; ++l) sum += part[lane * PR_WAVE + l];
            bcol[i * kApSlots + lane] = sorted[lane];
            bval[i * kApSlots + lane] = sum;
        }
        if (lane == 0) bcnt[i] = nk;
        __syncthreads();
    }
}

// A0 = R0 B, one wavefront per coarse row v.  Pass 1 collects the columns of
// the B rows that R0 row v names (lanes over R0's entries) in an LDS hash set
// and ranks them.  Pass 2: the two half-waves take R0's entries in turn (the
// first the even positions, the second the odd); the lanes of a half-wave
// take the entries of that B row (at most kApSlots, distinct columns) and add
// r_vi b_iw into the half-wave's sum of column w, so no two lanes of one step
// touch one sum.  The two halves are added at the end: a fixed order again.
__global__ __launch_bounds__(64) void k_rb(int64_t n0, const int64_t* __restrict__ rrp,
                                           const int32_t* __restrict__ rci, const double* __restrict__ rv,
                                           const int32_t* __restrict__ bcnt, const int32_t* __restrict__ bcol,
                                           const double* __restrict__ bval, double drop,
                                           int32_t* __restrict__ ocnt, int32_t* __restrict__ ocol,
                                           double* __restrict__ oval, int32_t* __restrict__ overflow) {
    static_assert(kApSlots <= PR_WAVE / 2, "a B row fits one half-wave");
    __shared__ int32_t keys[kGalSlots];
    __shared__ int32_t rank[kGalSlots];
    __shared__ int32_t sorted[kGalSlots];
    __shared__ double sums[2][kGalSlots];
    const int lane = threadIdx.x;
    const int half = lane / (PR_WAVE / 2), t = lane % (PR_WAVE / 2);
    constexpr int Q = kGalSlots / PR_WAVE;
    for (int64_t v = blockIdx.x; v < n0; v += gridDim.x) {
        for (int s = lane; s < kGalSlots; s += PR_WAVE) {
            keys[s] = -1;
            sums[0][s] = 0.0;
            sums[1][s] = 0.0;
        }
        __syncthreads();
        bool over = false;
        const int64_t r0 = rrp[v], r1 = rrp[v + 1];
        for (int64_t er = r0 + lane; er < r1; er += PR_WAVE) {
            const int32_t i = rci[er];
            const int c = bcnt[i];
            for (int u = 0; u < c; ++u) {
                const int32_t w = bcol[(int64_t)i * kApSlots + u];
                int h = gal_hash(w);
                int probes = 0;
                while (true) {
                    const int32_t old = atomicCAS(&keys[h], -1, w);
                    if (old == -1 || old == w) break;
                    h = (h + 1) & (kGalSlots - 1);
                    if (++probes >= kGalSlots) {
                        over = true;
                        break;
                    }
                }
            }
        }
        __syncthreads();
        if (__ballot(over)) {
            if (lane == 0) {
                atomicOr(overflow, 1);
                ocnt[v] = 0;
            }
            __syncthreads();
            continue;
        }
        int nk = 0;
        for (int s = lane; s < kGalSlots; s += PR_WAVE) {
            const int32_t k = keys[s];
            int r = -1;
            if (k >= 0) {
                r = 0;
                for (int u = 0; u < kGalSlots; ++u) {
                    const int32_t o = keys[u];
                    r += (o >= 0 && o < k) ? 1 : 0;
                }
                sorted[r] = k;
                ++nk;
            }
            rank[s] = r;
        }
        nk = wave_sum(nk);
        __syncthreads();
        for (int64_t er = r0 + half; er < r1; er += 2) {
            const int32_t i = rci[er];
            const double ri = rv[er];
            if (t < bcnt[i]) {
                const int32_t w = bcol[(int64_t)i * kApSlots + t];
                const double b = bval[(int64_t)i * kApSlots + t];
                int h = gal_hash(w);
                while (keys[h] != w) h = (h + 1) & (kGalSlots - 1);
                double* sp = &sums[half][rank[h]];
                *sp = fma(ri, b, *sp);
            }
        }
        __syncthreads();
        double acc[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] = sums[0][q * PR_WAVE + lane] + sums[1][q * PR_WAVE + lane];
        gal_emit(acc, nk, sorted, drop, v, ocnt, ocol, oval);
        __syncthreads();
    }
}

__global__ void k_rows_compact(int64_t n0, const int64_t* __restrict__ rp, const int32_t* __restrict__ icol,
                               const double* __restrict__ ival, int32_t* __restrict__ ocol,
                               double* __restrict__ oval) {
    const int64_t v = blockIdx.x;
    if (v >= n0) return;
    const int64_t a = rp[v], len = rp[v + 1] - a;
    for (int64_t e = threadIdx.x; e < len; e += blockDim.x) {
        ocol[a + e] = icol[v * kGalSlots + e];
        oval[a + e] = ival[v * kGalSlots + e];
    }
}

__global__ void k_cnt_to_i64(int64_t n, const int32_t* __restrict__ c, int64_t* __restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = c[i];
    else if (i == n) o[i] = 0;
}

// largest |v - w| over the entries of A0
__global__ void k_bandwidth(int64_t n0, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            int32_t* __restrict__ bw) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int b = 0;
    if (v < n0)
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) b = max(b, (int)abs((int64_t)ci[e] - v));
    b = wave_max(b);
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) atomicMax(bw, b);
}

// ---- dense blocks -----------------------------------------------------------
// S (s x s) = D_bi - L_bi H_{bi-1} with H_{bi-1} = Sinv_{bi-1} U_{bi-1} given
// (Hprev; S = D_0 for bi = 0): S[a][c] = A0[bi s + a][bi s + c] - sum over the
// entries (r, v) of A0 row bi s + a in block bi - 1 of v H[r][c].  Rows or
// columns beyond n0 form an identity.
__global__ void k_block_schur_h(int64_t n0, int s, int bi, const int64_t* __restrict__ rp,
                                const int32_t* __restrict__ ci, const double* __restrict__ v,
                                const double* __restrict__ Hprev, double* __restrict__ S) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)s * s) return;
    const int a = (int)(q / s), c = (int)(q % s);
    const int64_t ga = (int64_t)bi * s + a, gc = (int64_t)bi * s + c;
    if (ga >= n0 || gc >= n0) {
        S[q] = (a == c) ? 1.0 : 0.0;
        return;
    }
    const int64_t r0 = (int64_t)(bi - 1) * s;
    double d = 0.0, acc = 0.0;
    for (int64_t e = rp[ga]; e < rp[ga + 1]; ++e) {
        const int64_t col = ci[e];
        const double val = v[e];
        if (col == gc) d = val;
        if (Hprev && col >= r0 && col < r0 + s) acc += val * Hprev[(col - r0) * s + c];
    }
    S[q] = d - acc;
}

// out (s x s) = Sinv_bi C where C = block (bi, bj) of A0, read by columns
// from the transpose: out[a][c] = sum over the entries (r, v) of A0^T row
// bj s + c with r in block bi of Sinv[a][r - bi s] v.
__global__ void k_block_coupling(int64_t n0, int s, int bi, int bj, const int64_t* __restrict__ trp,
                                 const int32_t* __restrict__ tci, const double* __restrict__ tv,
                                 const double* __restrict__ Sinv, double* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)s * s) return;
    const int a = (int)(q / s), c = (int)(q % s);
    const int64_t gc = (int64_t)bj * s + c;
    const int64_t r0 = (int64_t)bi * s;
    double acc = 0.0;
    if (gc < n0)
        for (int64_t e = trp[gc]; e < trp[gc + 1]; ++e) {
            const int64_t r = tci[e];
            if (r >= r0 && r < r0 + s) acc += Sinv[(int64_t)a * s + (r - r0)] * tv[e];
        }
    out[q] = acc;
}

// dense n0 x n0 (padded to np) copy of A0, identity on the padding
__global__ void k_dense_from_csr(int64_t n0, int64_t np, const int64_t* __restrict__ rp,
                                 const int32_t* __restrict__ ci, const double* __restrict__ v,
                                 double* __restrict__ M) {
    for (int64_t a = blockIdx.x; a < np; a += gridDim.x) {
        double* row = M + a * np;
        for (int64_t c = threadIdx.x; c < np; c += blockDim.x) row[c] = (a >= n0 && a == c) ? 1.0 : 0.0;
        __syncthreads();
        if (a < n0)
            for (int64_t e = rp[a] + threadIdx.x; e < rp[a + 1]; e += blockDim.x) row[ci[e]] = v[e];
        __syncthreads();
    }
}

// ---- blocked Gauss-Jordan inverse in place (s multiple of 32) ----------------
// Inverse of the 32 x 32 row-major matrix in sP into sI by Gauss-Jordan
// elimination with partial pivoting, one wavefront holding the augmented
// matrix [P | I] by rows: lane r < 32 holds row r of P, lane 32 + r row r of
// the identity half, 32 doubles each.  Step k: the pivot is the largest
// |a_rk| over the rows not yet used (lowest row on ties), found by a DPP
// max within rows of 16 lanes and a ballot of the lanes holding it; the
// pivot row goes through LDS (sRow, 64 doubles) to every lane, and each lane
// updates its row with its factor a_rk: a_rc -= a_rk (p_c / p_k), the pivot
// row itself becoming p_c / p_k.  Row piv_k of the right half ends as row k
// of the inverse.  The step loop is unrolled, so no register is indexed at
// run time.  (Lane c holding column c instead made the pivot search a
// 32-step chain in one lane's registers and every row update a select by
// the pivot index: 1.5 us per step, 50 us per inverse.)  Returns nonzero on
// a zero pivot.
__device__ __forceinline__ double bcast(double v, int src) {
    const int2 t = *reinterpret_cast<const int2*>(&v);
    int2 r;
    r.x = __builtin_amdgcn_readlane(t.x, src);
    r.y = __builtin_amdgcn_readlane(t.y, src);
    return *reinterpret_cast<const double*>(&r);
}

// v of the lane `n` below in the same row of 16 (own value past the row's
// start): DPP row_shr:n on both halves
template <int N>
__device__ __forceinline__ double dpp_row_shr(double v) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8, "row_shr by 1, 2, 4 or 8");
    const int2 t = *reinterpret_cast<const int2*>(&v);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(t.x, t.x, 0x110 + N, 0xf, 0xf, false);
    r.y = __builtin_amdgcn_update_dpp(t.y, t.y, 0x110 + N, 0xf, 0xf, false);
    return *reinterpret_cast<const double*>(&r);
}

__device__ int reg_gj32(const double* sP, double* sI, int* srow, double* sRow, int lane) {
    const int h = lane >> 5, r = lane & 31;
    double a[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) a[c] = h == 0 ? sP[r * 32 + c] : (c == r ? 1.0 : 0.0);
    bool used = false;
    int bad = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        // pivot: largest |a_rk| over the unused rows (lanes 0..31)
        const double ak = a[k];
        const double mag = fabs(ak);
        const double v = (h == 0 && !used && mag >= 0.0) ? mag : -1.0;    // NaN never pivots
        double m = fmax(v, dpp_row_shr<1>(v));
        m = fmax(m, dpp_row_shr<2>(m));
        m = fmax(m, dpp_row_shr<4>(m));
        m = fmax(m, dpp_row_shr<8>(m));
        const double best = fmax(bcast(m, 15), bcast(m, 31));
        const uint64_t hold = __ballot(h == 0 && !used && v == best);
        const int piv = (int)__builtin_ctzll(hold);
        if (!(best > 0.0)) bad = 1;
        if (r == piv) used = true;
        if (lane == 0) srow[piv] = k;
        // factor of this lane's row: a_rk, held by lane r
        const double f = __shfl(ak, r);
        // the pivot row (both halves) to every lane
        if (r == piv) {
#pragma unroll
            for (int c = 0; c < 32; ++c) sRow[h * 32 + c] = a[c];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");    // one wavefront: LDS in order
        __builtin_amdgcn_wave_barrier();
        const double inv = 1.0 / sRow[k];
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            const double pv = sRow[h * 32 + c] * inv;
            a[c] = (r == piv) ? pv : fma(-f, pv, a[c]);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (h == 1) {
#pragma unroll
        for (int c = 0; c < 32; ++c) sI[srow[r] * 32 + c] = a[c];
    }
    __syncthreads();
    return bad;
}

// Panel k: P = M[k][k] (32 x 32 tile) is inverted in LDS; the row panel becomes
// M[k][j] <- P^{-1} M[k][j]; the column panel's old tiles go to C.
__global__ __launch_bounds__(64) void k_gj_panel(double* __restrict__ M, int s, int k,
                                                 double* __restrict__ Pinv, double* __restrict__ C,
                                                 int32_t* __restrict__ info) {
    __shared__ double sP[32 * 32];
    __shared__ double sI[32 * 32];
    __shared__ double sT[32 * 32];
    __shared__ int srow[32];
    __shared__ double sRow[64];
    const int lane = threadIdx.x;
    const int j = blockIdx.x;
    const int64_t ks = (int64_t)k * 32;
    for (int e = lane; e < 1024; e += PR_WAVE) sP[e] = M[(ks + e / 32) * s + ks + e % 32];
    __syncthreads();
    const int bad = reg_gj32(sP, sI, srow, sRow, lane);
    if (bad && lane == 0) atomicOr(info, 1);
    if (j == k) {
        for (int e = lane; e < 1024; e += PR_WAVE) Pinv[e] = sI[e];
        return;
    }
    const int64_t js = (int64_t)j * 32;
    for (int e = lane; e < 1024; e += PR_WAVE) {
        sT[e] = M[(ks + e / 32) * s + js + e % 32];
        C[(int64_t)j * 1024 + e] = M[(js + e / 32) * s + ks + e % 32];
    }
    __syncthreads();
    pr_d4 c[4];
    mm_wave<false>(sI, sT, 32, lane, c);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = mm_col(t, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = mm_row(t, v, lane);
            M[(ks + row) * s + js + col] = c[t][v];
        }
    }
}

// Every tile (I, J) with I != k: M[I][J] -= C[I] M[k][J] (J != k) or
// M[I][k] = -C[I] P^{-1}; tile (k, k) becomes P^{-1}.
__global__ __launch_bounds__(64) void k_gj_update(double* __restrict__ M, int s, int k,
                                                  const double* __restrict__ Pinv,
                                                  const double* __restrict__ C) {
    __shared__ double sC[32 * 32];
    __shared__ double sB[32 * 32];
    const int lane = threadIdx.x;
    const int nt = s / 32;
    const int I = blockIdx.x / nt, J = blockIdx.x % nt;
    const int64_t is = (int64_t)I * 32, js = (int64_t)J * 32, ks = (int64_t)k * 32;
    if (I == k) {
        if (J == k)
            for (int e = lane; e < 1024; e += PR_WAVE) M[(ks + e / 32) * s + ks + e % 32] = Pinv[e];
        return;
    }
    for (int e = lane; e < 1024; e += PR_WAVE) {
        sC[e] = C[(int64_t)I * 1024 + e];
        sB[e] = (J == k) ? Pinv[e] : M[(ks + e / 32) * s + js + e % 32];
    }
    __syncthreads();
    pr_d4 c[4];
    mm_wave<false>(sC, sB, 32, lane, c);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = mm_col(t, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = mm_row(t, v, lane);
            double* dst = &M[(is + row) * s + js + col];
            *dst = (J == k) ? -c[t][v] : *dst - c[t][v];
        }
    }
}

// ---- apply ------------------------------------------------------------------
// sum_c row[c] x[c] over c < s by one wavefront, lane l adding columns
// l, l + 64, ... in order (then a wave sum); eight columns' loads are issued
// before their products (a loop of one load pair per step waited for each:
// sixteen round trips per 1024-column row)
__device__ __forceinline__ double row_dot(const double* __restrict__ row, const double* __restrict__ x, int64_t s,
                                          int lane) {
    constexpr int U = 8;
    double acc = 0.0;
    for (int64_t c0 = lane; c0 < s; c0 += U * PR_WAVE) {
        double mv[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = c0 + (int64_t)u * PR_WAVE;
            const int64_t cc = c < s ? c : 0;
            mv[u] = row[cc];
            xv[u] = x[cc];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c0 + (int64_t)u * PR_WAVE < s) acc = fma(mv[u], xv[u], acc);
    }
    return wave_sum(acc);
}

// y[r] = sum_e v[e] x[c[e]] (one wavefront per row); rows >= m untouched
__global__ __launch_bounds__(256) void k_csr_rows_wave(int64_t m, const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       const int32_t* stop) {
    if (stopped(stop)) return;
    const int lane = threadIdx.x & (PR_WAVE - 1);
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PR_WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / PR_WAVE;
    for (int64_t r = w0; r < m; r += nw) {
        double acc = 0.0;
        for (int64_t e = rp[r] + lane; e < rp[r + 1]; e += PR_WAVE) acc += v[e] * x[ci[e]];
        acc = wave_sum(acc);
        if (lane == 0) y[r] = acc;
    }
}

// z[i] += sum_e v[e] x[c[e]] (one thread per row)
__global__ void k_csr_rows_add(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const double* __restrict__ v, const double* __restrict__ x,
                               double* __restrict__ z, const int32_t* stop) {
    if (stopped(stop)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * x[ci[e]];
    z[i] += acc;
}

// out[0..np) = X in (dense, np x np row-major); 4 rows per wave pass
__global__ __launch_bounds__(256) void k_dense_gemv(int64_t np, const double* __restrict__ X,
                                                    const double* __restrict__ in, double* __restrict__ out,
                                                    const int32_t* stop) {
    if (stopped(stop)) return;
    const int lane = threadIdx.x & (PR_WAVE - 1);
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PR_WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / PR_WAVE;
    for (int64_t r = w0; r < np; r += nw) {
        const double acc = row_dot(X + r * np, in, np, lane);
        if (lane == 0) out[r] = acc;
    }
}

// u_i = Sinv_i r0_i for every block i at once (one wavefront per row)
__global__ __launch_bounds__(256) void k_band_diag(int s, int nb, const double* __restrict__ Sinv,
                                                   const double* __restrict__ r0, double* __restrict__ u,
                                                   const int32_t* stop) {
    if (stopped(stop)) return;
    const int lane = threadIdx.x & (PR_WAVE - 1);
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PR_WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / PR_WAVE;
    const int64_t rows = (int64_t)nb * s;
    for (int64_t g = w0; g < rows; g += nw) {
        const int64_t bi = g / s, a = g % s;
        const double acc = row_dot(Sinv + bi * s * s + a * s, r0 + bi * s, s, lane);
        if (lane == 0) u[g] = acc;
    }
}

// out_i = in_i - M_i x_j (x_j the neighbouring block: j = i - 1 forward with
// M = G_i = Sinv_i L_i, j = i + 1 backward with M = H_i = Sinv_i U_i); one
// wavefront per row
__global__ __launch_bounds__(256) void k_band_couple(int s, const double* __restrict__ M,
                                                     const double* __restrict__ in, const double* __restrict__ xj,
                                                     double* __restrict__ out, const int32_t* stop) {
    if (stopped(stop)) return;
    const int lane = threadIdx.x & (PR_WAVE - 1);
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PR_WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / PR_WAVE;
    for (int64_t a = w0; a < s; a += nw) {
        const double acc = M ? row_dot(M + a * s, xj, s, lane) : 0.0;
        if (lane == 0) out[a] = in[a] - acc;
    }
}

}  // namespace

// ---- launchers ---------------------------------------------------------------

void launch_interp_check(int64_t n, int64_t n0, int64_t nnz, const int64_t* rp, const int32_t* ci,
                         const double* v, int32_t* flags, hipStream_t st) {
    k_interp_check<<<nbk(n + 1, 256), 256, 0, st>>>(n, n0, nnz, rp, ci, v, flags);
}

// transpose: tp int64[m+1] (out), tc/tv [nnz] (out); cnt, fill: int64[m+1],
// uc/uv [nnz] scratch
int launch_csr_transpose(int64_t n, int64_t m, const int64_t* rp, const int32_t* ci, const double* v,
                         int64_t* tp, int32_t* tc, double* tv, int64_t* cnt, int64_t* fill, int32_t* uc,
                         double* uv, int64_t* scan_scr, hipStream_t st) {
    if (hipMemsetAsync(cnt, 0, (m + 1) * sizeof(int64_t), st) != hipSuccess) return -1;
    if (hipMemsetAsync(fill, 0, (m + 1) * sizeof(int64_t), st) != hipSuccess) return -1;
    if (n > 0) k_tr_count<<<nbk(n, 256), 256, 0, st>>>(n, rp, ci, cnt);
    launch_exclusive_scan_i64(cnt, tp, m + 1, scan_scr, st);
    if (n > 0) k_tr_fill<<<nbk(n, 256), 256, 0, st>>>(n, rp, ci, v, tp, fill, uc, uv);
    if (m > 0) k_tr_rank<<<nbk(m, 4), 256, 0, st>>>(m, tp, uc, uv, tc, tv);
    return 0;
}

int coarse_gal_slots() { return kGalSlots; }

void launch_galerkin(int64_t n0, const int64_t* rrp, const int32_t* rci, const double* rv, const int64_t* arp,
                     const int32_t* aci, const double* av, const int64_t* prp, const int32_t* pci,
                     const double* pv, double drop, int32_t* ocnt, int32_t* ocol, double* oval,
                     int32_t* overflow, hipStream_t st) {
    if (n0 <= 0) return;
    const unsigned g = (unsigned)(n0 < 16384 ? n0 : 16384);
    k_galerkin<<<g, 64, 0, st>>>(n0, rrp, rci, rv, arp, aci, av, prp, pci, pv, drop, ocnt, ocol, oval, overflow);
}

int coarse_ap_slots() { return kApSlots; }

void launch_ap(int64_t n, const int64_t* arp, const int32_t* aci, const double* av, const int64_t* prp,
               const int32_t* pci, const double* pv, int32_t* bcnt, int32_t* bcol, double* bval,
               int32_t* overflow, hipStream_t st) {
    if (n <= 0) return;
    const unsigned g = (unsigned)(n < 65536 ? n : 65536);
    k_ap<<<g, 64, 0, st>>>(n, arp, aci, av, prp, pci, pv, bcnt, bcol, bval, overflow);
}

void launch_rb(int64_t n0, const int64_t* rrp, const int32_t* rci, const double* rv, const int32_t* bcnt,
               const int32_t* bcol, const double* bval, double drop, int32_t* ocnt, int32_t* ocol, double* oval,
               int32_t* overflow, hipStream_t st) {
    if (n0 <= 0) return;
    const unsigned g = (unsigned)(n0 < 16384 ? n0 : 16384);
    k_rb<<<g, 64, 0, st>>>(n0, rrp, rci, rv, bcnt, bcol, bval, drop, ocnt, ocol, oval, overflow);
}

void launch_rows_finish(int64_t n0, const int32_t* cnt32, int64_t* cnt64, int64_t* rp, int64_t* scan_scr,
                        hipStream_t st) {
    k_cnt_to_i64<<<nbk(n0 + 1, 256), 256, 0, st>>>(n0, cnt32, cnt64);
    launch_exclusive_scan_i64(cnt64, rp, n0 + 1, scan_scr, st);
}

void launch_rows_compact(int64_t n0, const int64_t* rp, const int32_t* icol, const double* ival, int32_t* ocol,
                         double* oval, hipStream_t st) {
    if (n0 > 0) k_rows_compact<<<(unsigned)n0, 64, 0, st>>>(n0, rp, icol, ival, ocol, oval);
}

void launch_bandwidth(int64_t n0, const int64_t* rp, const int32_t* ci, int32_t* bw, hipStream_t st) {
    k_bandwidth<<<nbk(n0, 256), 256, 0, st>>>(n0, rp, ci, bw);
}

void launch_dense_from_csr(int64_t n0, int64_t np, const int64_t* rp, const int32_t* ci, const double* v,
                           double* M, hipStream_t st) {
    k_dense_from_csr<<<(unsigned)(np < 16384 ? np : 16384), 256, 0, st>>>(n0, np, rp, ci, v, M);
}

// in-place inverse of the s x s row-major matrix M (s a multiple of 32)
void launch_gj_inverse(double* M, int s, double* Pinv, double* C, int32_t* info, hipStream_t st) {
    const int nt = s / 32;
    for (int k = 0; k < nt; ++k) {
        k_gj_panel<<<nt, 64, 0, st>>>(M, s, k, Pinv, C, info);
        k_gj_update<<<nt * nt, 64, 0, st>>>(M, s, k, Pinv, C);
    }
}

void launch_csr_rows_wave(int64_t m, const int64_t* rp, const int32_t* ci, const double* v, const double* x,
                          double* y, const int32_t* stop, hipStream_t st) {
    if (m <= 0) return;
    const int64_t blocks = (m + 3) / 4;
    k_csr_rows_wave<<<(unsigned)(blocks < 8192 ? blocks : 8192), 256, 0, st>>>(m, rp, ci, v, x, y, stop);
}

void launch_csr_rows_add(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, const double* x,
                         double* z, const int32_t* stop, hipStream_t st) {
    if (n > 0) k_csr_rows_add<<<nbk(n, 256), 256, 0, st>>>(n, rp, ci, v, x, z, stop);
}

void launch_dense_gemv(int64_t np, const double* X, const double* in, double* out, const int32_t* stop,
                       hipStream_t st) {
    const int64_t blocks = (np + 3) / 4;
    k_dense_gemv<<<(unsigned)(blocks < 8192 ? blocks : 8192), 256, 0, st>>>(np, X, in, out, stop);
}

void launch_block_schur_h(int64_t n0, int s, int bi, const int64_t* rp, const int32_t* ci, const double* v,
                          const double* Hprev, double* S, hipStream_t st) {
    k_block_schur_h<<<nbk((int64_t)s * s, 256), 256, 0, st>>>(n0, s, bi, rp, ci, v, Hprev, S);
}

void launch_block_coupling(int64_t n0, int s, int bi, int bj, const int64_t* trp, const int32_t* tci,
                           const double* tv, const double* Sinv, double* out, hipStream_t st) {
    k_block_coupling<<<nbk((int64_t)s * s, 256), 256, 0, st>>>(n0, s, bi, bj, trp, tci, tv, Sinv, out);
}

// x = A0^{-1} r0 from the block LU: u_i = Sinv_i r0_i (all blocks together);
// w_0 = u_0, w_i = u_i - G_i w_{i-1}; x_{nb-1} = w_{nb-1},
// x_i = w_i - H_i x_{i+1}.  G, H: nb blocks of s x s (G_0, H_{nb-1} unused).
void launch_band_solve(int s, int nb, const double* Sinv, const double* G, const double* H, const double* r0,
                        double* u, double* w, double* x, const int32_t* stop, hipStream_t st) {
    const int64_t blk = (int64_t)s * s;
    const int64_t rows = (int64_t)nb * s;
    const int64_t b1 = (rows + 3) / 4;
    k_band_diag<<<(unsigned)(b1 < 16384 ? b1 : 16384), 256, 0, st>>>(s, nb, Sinv, r0, u, stop);
    const unsigned g = (unsigned)((s + 3) / 4);
    // the first forward and the last backward step couple to nothing (M null)
    for (int i = 0; i < nb; ++i)
        k_band_couple<<<g, 256, 0, st>>>(s, i == 0 ? nullptr : G + blk * i, u + (int64_t)i * s,
                                         i == 0 ? u : w + (int64_t)(i - 1) * s, w + (int64_t)i * s, stop);
    for (int i = nb - 1; i >= 0; --i)
        k_band_couple<<<g, 256, 0, st>>>(s, i == nb - 1 ? nullptr : H + blk * i, w + (int64_t)i * s,
                                         i == nb - 1 ? w : x + (int64_t)(i + 1) * s, x + (int64_t)i * s, stop);
}
