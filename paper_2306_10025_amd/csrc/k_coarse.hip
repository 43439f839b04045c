// Two-level combination preconditioner (Eq.(2)) on the device:
//   M_combo^{-1} r = M~^{-1} r + P0 A0^{-1} R0 r,   R0 = P0^T,  A0 = R0 A P0,
// with A0 solved directly, as in the first two numerical experiments.
//
// Setup: R0 by a transpose of P0; A0 one coarse row per wavefront with a
// fixed summation order per entry (deterministic); then a direct solver:
//  - small A0 (dense form): its explicit inverse;
//  - otherwise A0 is banded (|v - w| <= b for every entry), so with blocks of
//    s >= b rows it is block tridiagonal, and block LU without pivoting across
//    blocks (A0 is symmetric positive definite for the diffusion problems)
//    keeps the inverses of the Schur complements
//        S_0 = D_0,  S_i = D_i - L_i S_{i-1}^{-1} U_{i-1},
//    where D_i, L_i, U_i are the diagonal, sub- and super-diagonal blocks.
//  Dense inverses: blocked Gauss-Jordan in place, 32-wide panels, the rank-32
//  updates on the FP64 matrix cores (16 x 16 x 4 MFMA), partial pivoting
//  inside each 32 x 32 pivot block.
// Apply: r0 = R0 r; forward sweep w_i = S_i^{-1} (r0_i - L_i w_{i-1});
// backward sweep x_i = w_i - S_i^{-1} U_i x_{i+1}; z += P0 x.  Every kernel
// returns at once when the solve's stop flag is set (graph replays).
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

// rows of the transpose in ascending column (the fill order depends on timing)
__global__ void k_tr_sort(int64_t m, const int64_t* __restrict__ tp, int32_t* __restrict__ tc,
                          double* __restrict__ tv) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int64_t a = tp[r], b = tp[r + 1];
    for (int64_t e = a + 1; e < b; ++e) {
        const int32_t kc = tc[e];
        const double kv = tv[e];
        int64_t q = e - 1;
        while (q >= a && tc[q] > kc) {
            tc[q + 1] = tc[q];
            tv[q + 1] = tv[q];
            --q;
        }
        tc[q + 1] = kc;
        tv[q + 1] = kv;
    }
}

// ---- Galerkin product A0 = R0 A P0, one wavefront per coarse row -------------
constexpr int kGalSlots = 256;   // distinct coarse columns one coarse row may reach

__device__ __forceinline__ int gal_hash(int32_t w) { return (int)(((uint32_t)w * 2654435761u) >> 24); }

// Pass 1 collects the coarse columns w reachable from row v (R0 row v, then A
// rows, then P0 rows) in an LDS hash set; they are ranked in ascending order.
// Pass 2: lane l owns the columns of rank l, l + 64, ...; every lane walks the
// same stream of products r_vi a_ij p_jw in the same order and adds those of
// its columns, so each entry is summed in one fixed order.  Entries at most
// drop times the row's largest magnitude are dropped (rounding residue of
// couplings that vanish exactly).  Output: row v at out + v * kGalSlots.
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
// S (s x s, row-major) = block (bi, bj) of A0 minus Y U (when Y is given):
// S[a][c] = A0[bi s + a][bj s + c] - sum_r Y[a][r] A0[(bi - 1) s + r][bi s + c];
// rows or columns beyond n0 form an identity (padding of the last block).
__global__ void k_block_schur(int64_t n0, int s, int bi, const int64_t* __restrict__ rp,
                              const int32_t* __restrict__ ci, const double* __restrict__ v,
                              const int64_t* __restrict__ trp, const int32_t* __restrict__ tci,
                              const double* __restrict__ tv, const double* __restrict__ Y,
                              double* __restrict__ S) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)s * s) return;
    const int a = (int)(q / s), c = (int)(q % s);
    const int64_t ga = (int64_t)bi * s + a, gc = (int64_t)bi * s + c;
    if (ga >= n0 || gc >= n0) {
        S[q] = (a == c) ? 1.0 : 0.0;
        return;
    }
    // A0[ga][gc] by binary search in the sorted row
    int64_t lo = rp[ga], hi = rp[ga + 1];
    double d = 0.0;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t cm = ci[mid];
        if (cm == gc) {
            d = v[mid];
            break;
        }
        if (cm < gc) lo = mid + 1;
        else hi = mid;
    }
    if (Y && bi > 0) {
        // column gc of A0 = row gc of its transpose; rows r of block bi - 1
        const int64_t r0 = (int64_t)(bi - 1) * s;
        double acc = 0.0;
        for (int64_t e = trp[gc]; e < trp[gc + 1]; ++e) {
            const int64_t r = tci[e];
            if (r >= r0 && r < r0 + s) acc += Y[(int64_t)a * s + (r - r0)] * tv[e];
        }
        d -= acc;
    }
    S[q] = d;
}

// Y (s x s) = L_bi Sinv_prev: row a of Y sums the rows of Sinv_prev named by
// the entries of A0 row bi s + a that fall in block bi - 1
__global__ void k_block_lsinv(int64_t n0, int s, int bi, const int64_t* __restrict__ rp,
                              const int32_t* __restrict__ ci, const double* __restrict__ v,
                              const double* __restrict__ Sprev, double* __restrict__ Y) {
    for (int a = blockIdx.x; a < s; a += gridDim.x) {
        const int64_t ga = (int64_t)bi * s + a;
        const int64_t c0 = (int64_t)(bi - 1) * s;
        for (int c = threadIdx.x; c < s; c += blockDim.x) {
            double acc = 0.0;
            if (ga < n0)
                for (int64_t e = rp[ga]; e < rp[ga + 1]; ++e) {
                    const int64_t col = ci[e];
                    if (col >= c0 && col < c0 + s) acc += v[e] * Sprev[(col - c0) * s + c];
                }
            Y[(int64_t)a * s + c] = acc;
        }
    }
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
// Panel k: P = M[k][k] (32 x 32 tile) is inverted in LDS; the row panel becomes
// M[k][j] <- P^{-1} M[k][j]; the column panel's old tiles go to C.
__global__ __launch_bounds__(64) void k_gj_panel(double* __restrict__ M, int s, int k,
                                                 double* __restrict__ Pinv, double* __restrict__ C,
                                                 int32_t* __restrict__ info) {
    __shared__ double sP[32 * 32];
    __shared__ double sI[32 * 32];
    __shared__ double sT[32 * 32];
    const int lane = threadIdx.x;
    const int j = blockIdx.x;
    const int64_t ks = (int64_t)k * 32;
    for (int e = lane; e < 1024; e += PR_WAVE) sP[e] = M[(ks + e / 32) * s + ks + e % 32];
    __syncthreads();
    const int bad = gj_invert<32, 32>(sP, sI, 32, lane & 31);
    __syncthreads();
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
        const double* row = X + r * np;
        double acc = 0.0;
        for (int64_t c = lane; c < np; c += PR_WAVE) acc += row[c] * in[c];
        acc = wave_sum(acc);
        if (lane == 0) out[r] = acc;
    }
}

// Block step of the banded solve.  fwd: y = r0_i - L_i w_{i-1};
// w_i = Sinv_i y.  bwd: t = U_i x_{i+1}; x_i = w_i - Sinv_i t (the last block
// copies x = w).  Every workgroup forms the s-vector in LDS, then its waves
// take rows of Sinv_i.
template <bool FWD>
__global__ __launch_bounds__(256) void k_band_step(int64_t n0, int s, int nb, int bi,
                                                   const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ Sinv,
                                                   const double* __restrict__ r0, double* __restrict__ w,
                                                   double* __restrict__ x, const int32_t* stop) {
    extern __shared__ double sy[];
    if (stopped(stop)) return;
    const int64_t base = (int64_t)bi * s;
    if (!FWD && bi == nb - 1) {
        for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < s;
             a += (int64_t)gridDim.x * blockDim.x)
            x[base + a] = w[base + a];
        return;
    }
    // neighbour block: i - 1 (forward) or i + 1 (backward)
    const int64_t nbase = FWD ? base - s : base + s;
    const double* nv = FWD ? w : x;
    for (int a = threadIdx.x; a < s; a += blockDim.x) {
        const int64_t g = base + a;
        double acc = 0.0;
        if (g < n0 && (FWD ? bi > 0 : true))
            for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
                const int64_t c = ci[e];
                if (c >= nbase && c < nbase + s) acc += v[e] * nv[c];
            }
        sy[a] = FWD ? ((g < n0 ? r0[g] : 0.0) - acc) : acc;
    }
    __syncthreads();
    const int lane = threadIdx.x & (PR_WAVE - 1);
    const int wv = threadIdx.x / PR_WAVE;
    const int nwv = blockDim.x / PR_WAVE;
    const double* Si = Sinv + (int64_t)bi * s * s;
    for (int64_t row = (int64_t)blockIdx.x * nwv + wv; row < s; row += (int64_t)gridDim.x * nwv) {
        const double* sr = Si + row * s;
        double acc = 0.0;
        for (int c = lane; c < s; c += PR_WAVE) acc += sr[c] * sy[c];
        acc = wave_sum(acc);
        if (lane == 0) {
            if (FWD) w[base + row] = acc;
            else x[base + row] = w[base + row] - acc;
        }
    }
}

}  // namespace

// ---- launchers ---------------------------------------------------------------

void launch_interp_check(int64_t n, int64_t n0, int64_t nnz, const int64_t* rp, const int32_t* ci,
                         const double* v, int32_t* flags, hipStream_t st) {
    k_interp_check<<<nbk(n + 1, 256), 256, 0, st>>>(n, n0, nnz, rp, ci, v, flags);
}

// transpose: tp int64[m+1] (out), tc/tv [nnz] (out); cnt, fill: int64[m+1] scratch
int launch_csr_transpose(int64_t n, int64_t m, const int64_t* rp, const int32_t* ci, const double* v,
                         int64_t* tp, int32_t* tc, double* tv, int64_t* cnt, int64_t* fill,
                         int64_t* scan_scr, hipStream_t st) {
    if (hipMemsetAsync(cnt, 0, (m + 1) * sizeof(int64_t), st) != hipSuccess) return -1;
    if (hipMemsetAsync(fill, 0, (m + 1) * sizeof(int64_t), st) != hipSuccess) return -1;
    if (n > 0) k_tr_count<<<nbk(n, 256), 256, 0, st>>>(n, rp, ci, cnt);
    launch_exclusive_scan_i64(cnt, tp, m + 1, scan_scr, st);
    if (n > 0) k_tr_fill<<<nbk(n, 256), 256, 0, st>>>(n, rp, ci, v, tp, fill, tc, tv);
    if (m > 0) k_tr_sort<<<nbk(m, 256), 256, 0, st>>>(m, tp, tc, tv);
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

void launch_block_schur(int64_t n0, int s, int bi, const int64_t* rp, const int32_t* ci, const double* v,
                        const int64_t* trp, const int32_t* tci, const double* tv, const double* Y, double* S,
                        hipStream_t st) {
    k_block_schur<<<nbk((int64_t)s * s, 256), 256, 0, st>>>(n0, s, bi, rp, ci, v, trp, tci, tv, Y, S);
}

void launch_block_lsinv(int64_t n0, int s, int bi, const int64_t* rp, const int32_t* ci, const double* v,
                        const double* Sprev, double* Y, hipStream_t st) {
    k_block_lsinv<<<(unsigned)(s < 4096 ? s : 4096), 256, 0, st>>>(n0, s, bi, rp, ci, v, Sprev, Y);
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

void launch_band_solve(int64_t n0, int s, int nb, const int64_t* rp, const int32_t* ci, const double* v,
                       const double* Sinv, const double* r0, double* w, double* x, const int32_t* stop,
                       hipStream_t st) {
    // one workgroup per 8 rows of S_i^{-1} (4 waves, 2 rows each per pass)
    const unsigned g = (unsigned)((s + 7) / 8);
    const size_t lds = (size_t)s * sizeof(double);
    for (int i = 0; i < nb; ++i)
        k_band_step<true><<<g, 256, lds, st>>>(n0, s, nb, i, rp, ci, v, Sinv, r0, w, x, stop);
    for (int i = nb - 1; i >= 0; --i)
        k_band_step<false><<<g, 256, lds, st>>>(n0, s, nb, i, rp, ci, v, Sinv, r0, w, x, stop);
}
