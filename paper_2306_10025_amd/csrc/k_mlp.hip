// Learned predictor of a patch's database entry (the neural shortcut to the
// database construction that the closing remarks of Section 3.2 and Section 5
// point to), with hand-written inference and training kernels:
//  * patch invariants as features (one wavefront per patch);
//  * dense layers as GEMMs, either FP32 FMA or FP16 MFMA (32x32x8) with FP32
//    accumulation, with the bias, ReLU and ReLU-derivative mask fused into
//    the epilogue;
//  * softmax cross-entropy and its gradient, top-k selection, Adam;
//  * the exact criterion on the predicted candidates (accept on d < eps) and
//    the in-order scan of the database for patches the prediction missed.
#include "dense_dev.h"

#include <climits>

namespace {

using namespace pr_dev;

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// features (F = 3 pmax + 1): A_aa / m, sum_b |A_ab| / m, single-entry row bit,
// log m, with m = mean_a |A_aa| (1 when 0); slots beyond p stay 0
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_mlp_features(int64_t n_p, const int64_t* __restrict__ ptr,
                                                     const double* __restrict__ tiles,
                                                     const int64_t* __restrict__ toff, int ups,
                                                     const uint32_t* __restrict__ bkeys, int pmax,
                                                     float* __restrict__ out) {
    const int lane = threadIdx.x;
    const int F = 3 * pmax + 1;
    for (int64_t k = blockIdx.x; k < n_p; k += gridDim.x) {
        const int p = (int)(ptr[k + 1] - ptr[k]);
        const double* A = tiles + (ups ? k * (int64_t)ups * ups : toff[k]);
        double d = 0.0, rs = 0.0;
        if (lane < p) {
            d = A[(int64_t)lane * p + lane];
            for (int b = 0; b < p; ++b) rs += fabs(A[(int64_t)lane * p + b]);
        }
        double m = wave_sum(lane < p ? fabs(d) : 0.0) / (double)p;
        if (m == 0.0) m = 1.0;
        const uint32_t key = bkeys[k];
        float* o = out + k * (int64_t)F;
#pragma unroll
        for (int rep = 0; rep < 2; ++rep) {          // F <= 97 < 128
            const int f = lane + rep * PR_WAVE;
            const int sec = f / pmax, a = f % pmax;
            const double vd = __shfl(d, a);
            const double vr = __shfl(rs, a);
            if (f < F) {
                float v = 0.0f;
                if (sec == 3) v = (float)log(m);
                else if (a < p) v = (float)(sec == 0 ? vd / m : sec == 1 ? vr / m : (double)((key >> a) & 1u));
                o[f] = v;
            }
        }
    }
}

// per-feature mean and std over the rows listed (fixed order, FP64 sums)
__global__ void k_mlp_moments(int64_t nrows, const int32_t* __restrict__ rows, const float* __restrict__ X,
                              int F, float* __restrict__ mu, float* __restrict__ sd) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double s = 0.0;
    for (int64_t r = 0; r < nrows; ++r) s += (double)X[(int64_t)rows[r] * F + f];
    const double mean = s / (double)nrows;
    double v = 0.0;
    for (int64_t r = 0; r < nrows; ++r) {
        const double t = (double)X[(int64_t)rows[r] * F + f] - mean;
        v += t * t;
    }
    double st = sqrt(v / (double)nrows);
    if (st == 0.0) st = 1.0;
    mu[f] = (float)mean;
    sd[f] = (float)st;
}

// Xn[r] = (X[rows[r]] - mu) / sd; optional gathers of the labels and row keys
__global__ void k_mlp_gather(int64_t nrows, const int32_t* __restrict__ rows, const float* __restrict__ X,
                             int F, const float* __restrict__ mu, const float* __restrict__ sd,
                             float* __restrict__ Xn, const int32_t* __restrict__ lab_src,
                             int32_t* __restrict__ lab, const int32_t* __restrict__ key_src,
                             int32_t* __restrict__ key) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * F) return;
    const int64_t r = t / F;
    const int f = (int)(t % F);
    const int64_t i = rows[r];
    Xn[t] = (X[i * F + f] - mu[f]) / sd[f];
    if (f == 0) {
        if (lab) lab[r] = lab_src[r];
        if (key) key[r] = key_src[i];
    }
}

// ---------------------------------------------------------------------------
// C[m][n] = alpha sum_k op(A)[m][k] op(B)[k][n] (+ bias[n]), then ReLU, then
// times (mask[m][n] > 0).  op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k];
// op(B)[k][n] = TB ? B[n ldb + k] : B[k ldb + n].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gemm_store(float acc, float alpha, int m, int n, float* C, int ldc,
                                           const float* bias, int relu, const float* mask, int ldm) {
    float v = alpha * acc;
    if (bias) v += bias[n];
    if (relu) v = fmaxf(v, 0.0f);
    if (mask && !(mask[(int64_t)m * ldm + n] > 0.0f)) v = 0.0f;
    C[(int64_t)m * ldc + n] = v;
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f32(int M, int N, int K, const float* __restrict__ A, int lda,
                                                  const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                  int ldc, float alpha, const float* __restrict__ bias,
                                                  int relu, const float* __restrict__ mask, int ldm) {
    const int n = blockIdx.x * 16 + (threadIdx.x & 15);
    const int m = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (m >= M || n >= N) return;
    float acc = 0.0f;
    for (int k = 0; k < K; ++k) {
        const float a = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
        const float b = TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
        acc = fmaf(a, b, acc);
    }
    gemm_store(acc, alpha, m, n, C, ldc, bias, relu, mask, ldm);
}

// one wavefront per 32 x 32 tile of C; operands rounded to FP16 (nearest
// even) on load, products accumulated in FP32 by v_mfma_f32_32x32x8_f16.
// Lane l supplies A[m0 + l%32][k0 + 4(l/32) + t] and B[k0 + 4(l/32) + t][n0 + l%32]
// (t < 4) and holds C[m0 + 8(v/4) + 4(l/32) + v%4][n0 + l%32] (v < 16).
template <bool TA, bool TB>
__global__ __launch_bounds__(64) void k_gemm_f16(int M, int N, int K, const float* __restrict__ A, int lda,
                                                 const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                 int ldc, float alpha, const float* __restrict__ bias,
                                                 int relu, const float* __restrict__ mask, int ldm) {
    const int lane = threadIdx.x;
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    const int mi = m0 + (lane & 31), nj = n0 + (lane & 31), kh = 4 * (lane >> 5);
    f16v acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    // K in groups of U steps of 8: every load of a group is issued before
    // its products.  Loads are unconditional from clamped indices and the
    // values outside the matrices are dropped afterwards (a load under a
    // condition becomes a branch whose join waits for it).
    constexpr int U = 4;
    const int mc = mi < M ? mi : M - 1, nc = nj < N ? nj : N - 1;
    for (int kg = 0; kg < K; kg += 8 * U) {
        float av[U][4], bv[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = kg + 8 * u + kh + t;
                const int kc = k < K ? k : K - 1;
                av[u][t] = TA ? A[(int64_t)kc * lda + mc] : A[(int64_t)mc * lda + kc];
                bv[u][t] = TB ? B[(int64_t)nc * ldb + kc] : B[(int64_t)kc * ldb + nc];
            }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            h4 a, b;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // a multiply by 0/1, not a select: the compiler sinks a load
                // whose value a select may discard into a branch
                const int k = kg + 8 * u + kh + t;
                a[t] = (_Float16)(av[u][t] * ((mi < M && k < K) ? 1.0f : 0.0f));
                b[t] = (_Float16)(bv[u][t] * ((nj < N && k < K) ? 1.0f : 0.0f));
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x8f16(a, b, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int m = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int n = n0 + (lane & 31);
        if (m < M && n < N) gemm_store(acc[v], alpha, m, n, C, ldc, bias, relu, mask, ldm);
    }
}

// ---------------------------------------------------------------------------
// softmax cross-entropy over the allowed classes (rkey[r] == ckey[c], or all):
// loss_r = log sum exp(l) - l[y]; G = (softmax - onehot(y)) * scale
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_softmax_ce(int B, int C, const float* __restrict__ L, int ldl,
                                                   const int32_t* __restrict__ y,
                                                   const int32_t* __restrict__ rkey,
                                                   const int32_t* __restrict__ ckey, float* __restrict__ G,
                                                   int ldg, double* __restrict__ loss_rows, float scale) {
    const int lane = threadIdx.x;
    for (int r = blockIdx.x; r < B; r += gridDim.x) {
        const float* l = L + (int64_t)r * ldl;
        const int key = rkey ? rkey[r] : 0;
        double mx = -INFINITY;
        for (int c = lane; c < C; c += PR_WAVE)
            if (!ckey || ckey[c] == key) mx = fmax(mx, (double)l[c]);
        mx = wave_max(mx);
        double s = 0.0;
        for (int c = lane; c < C; c += PR_WAVE)
            if (!ckey || ckey[c] == key) s += exp((double)l[c] - mx);
        s = wave_sum(s);
        const int yr = y[r];
        const bool ok = yr >= 0 && yr < C;     // a label outside the classes gives a NaN loss
        if (lane == 0) loss_rows[r] = ok ? log(s) + mx - (double)l[yr] : NAN;
        if (G) {
            for (int c = lane; c < C; c += PR_WAVE) {
                double g = (!ckey || ckey[c] == key) ? exp((double)l[c] - mx) / s : 0.0;
                if (c == yr) g -= 1.0;
                G[(int64_t)r * ldg + c] = (float)(g * scale);
            }
        }
    }
}

// bias gradient: scale times the column sums
// (block of 256 threads per 64 columns: 4 row phases, each summing rows
// r = phase, phase + 4, ... in FP64, then the phases added in order)
__global__ __launch_bounds__(256) void k_colsum(int B, int N, const float* __restrict__ G, int ldg, float scale,
                                                float* __restrict__ out) {
    __shared__ double s_p[4][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    double s = 0.0;
    if (n < N) {
        int r = ph;
        for (; r + 12 < B; r += 16) {       // four independent loads in flight
            const float g0 = G[(int64_t)r * ldg + n], g1 = G[(int64_t)(r + 4) * ldg + n];
            const float g2 = G[(int64_t)(r + 8) * ldg + n], g3 = G[(int64_t)(r + 12) * ldg + n];
            s += (double)g0;
            s += (double)g1;
            s += (double)g2;
            s += (double)g3;
        }
        for (; r < B; r += 4) s += (double)G[(int64_t)r * ldg + n];
    }
    s_p[ph][c] = s;
    __syncthreads();
    if (ph == 0 && n < N) out[n] = (float)((((s_p[0][c] + s_p[1][c]) + s_p[2][c]) + s_p[3][c]) * (double)scale);
}

// Adam (Kingma and Ba): bc1 = 1 - b1^t, bc2 = 1 - b2^t
__global__ void k_adam(int64_t n, float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// SplitMix64 output number `idx + 1` of the stream seeded with `seed`
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// W uniform in [-a, a] with a = sqrt(6 / fan_in) (He-uniform), or 0
__global__ void k_init_uniform(int64_t n, float* __restrict__ W, float a, uint64_t seed, uint64_t base) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u = (double)(splitmix_at(seed, base + (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
    W[i] = (float)((2.0 * u - 1.0) * a);
}

// top-k allowed classes per row: largest logit first, lower index on ties
__global__ __launch_bounds__(64) void k_topk(int64_t R, int C, const float* __restrict__ L, int ldl, int k,
                                             const int32_t* __restrict__ rkey, const int32_t* __restrict__ ckey,
                                             int32_t* __restrict__ out) {
    const int lane = threadIdx.x;
    for (int64_t r = blockIdx.x; r < R; r += gridDim.x) {
        const float* l = L + r * ldl;
        const int key = rkey ? rkey[r] : 0;
        int picked[8];
        for (int t = 0; t < k; ++t) {
            float bv = -INFINITY;
            int bi = INT_MAX;
            for (int c = lane; c < C; c += PR_WAVE) {
                if (ckey && ckey[c] != key) continue;
                bool used = false;
                for (int q = 0; q < t; ++q) used |= (picked[q] == c);
                if (used) continue;
                const float v = l[c];
                if (bi == INT_MAX || v > bv) {
                    bv = v;
                    bi = c;
                }
            }
#pragma unroll
            for (int o = PR_WAVE / 2; o > 0; o >>= 1) {
                const float ov = __shfl_xor(bv, o);
                const int oi = __shfl_xor(bi, o);
                if (oi != INT_MAX && (bi == INT_MAX || ov > bv || (ov == bv && oi < bi))) {
                    bv = ov;
                    bi = oi;
                }
            }
            picked[t] = (bi == INT_MAX) ? -1 : bi;
            if (lane == 0) out[r * k + t] = picked[t];
        }
    }
}

// exact test of one pair (wavefront-wide); sA holds A_i; returns d < eps.
// sX, sE, sH: p x p LDS scratch.
__device__ bool pair_matches(int crit, double eps, const double* sA, double* sX, double* sE, double* sH,
                             const double* Xr, const double* Br, int p, int lane, unsigned long long& nev,
                             unsigned long long& nex, unsigned long long& nsq) {
    const int pp = p * p;
    ++nev;
    if (crit == PR_CRIT_SPECTRAL) {
        lds_load(sX, Xr, pp, lane);
        __syncthreads();
        double lb2;
        const double fro2 = form_E(sA, sX, sE, p, lane, &lb2);
        __syncthreads();
        const double e2 = eps * eps;
        auto decided = [e2](double lo, double hi) {
            return hi * (1.0 + 1e-11) < e2 || lo * (1.0 - 1e-11) >= e2;
        };
        double lo = lb2, hi = fro2;
        if (!decided(lo, hi)) {
            sigma2_bracket(sE, sX, sH, p, lane, kSquarings, lo, hi, decided);   // E kept in sE
            ++nsq;
        }
        bool match;
        if (decided(lo, hi)) {
            match = hi * (1.0 + 1e-11) < e2;
        } else {
            __syncthreads();
            match = sqrt(sigma_max2_jacobi(sE, sX, p, lane)) < eps;
            ++nex;
        }
        __syncthreads();
        return match;
    }
    double acc = 0.0;
    for (int e = lane; e < pp; e += PR_WAVE) {
        const double v = sA[e] - Br[e];
        acc += (crit == PR_CRIT_L1) ? fabs(v) : v * v;
    }
    acc = wave_sum(acc);
    return ((crit == PR_CRIT_L1) ? acc : sqrt(acc)) < eps;
}

struct PairGeom {
    const int64_t* ptr;
    const double* tiles;
    const int64_t* toff;
    int ups;
    const int32_t* entries;   // entry patch ids (training database, append order)
    int64_t n0;
    const double* X0;         // FP64 inverses of the entries, stride apart
    int64_t stride;
    int crit;
    double eps;
};

__device__ __forceinline__ const double* tile_of(const PairGeom& g, int64_t i) {
    return g.tiles + (g.ups ? i * (int64_t)g.ups * g.ups : g.toff[i]);
}

// mode 0: try the predicted candidates cand[q*k .. q*k+k) in rank order;
// mode 1: scan every entry in append order, skipping pairs the norm-key bound
// rules out.  The first d < eps sets repof[i] to the entry's patch.
__global__ __launch_bounds__(64, 2) void k_mlp_match(int mode, int64_t nq, const int32_t* __restrict__ qids,
                                                  const int32_t* __restrict__ cand, int k, PairGeom g,
                                                  const double* __restrict__ keynorm,
                                                  int32_t* __restrict__ repof, int32_t* __restrict__ resolved,
                                                  unsigned long long* __restrict__ counters) {
    __shared__ double sA[kMaxPs * kMaxPs];
    __shared__ double sX[kMaxPs * kMaxPs];
    __shared__ double sE[kMaxPs * kMaxPs];
    __shared__ double sH[kMaxPs * kMaxPs];
    const int lane = threadIdx.x;
    unsigned long long nev = 0, nex = 0, nsq = 0;
    for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int32_t i = qids[q];
        const int p = (int)(g.ptr[i + 1] - g.ptr[i]);
        const double* Ai = tile_of(g, i);
        lds_load(sA, Ai, p * p, lane);
        __syncthreads();
        const double ki = keynorm[i];
        const double c = (p * p + 64) * 2.3e-16;
        int32_t hit = -1;
        const int64_t nt = mode == 0 ? k : g.n0;
        for (int64_t t = 0; t < nt && hit < 0; ++t) {
            const int64_t j = mode == 0 ? cand[q * k + t] : t;
            if (j < 0 || j >= g.n0) continue;
            const int32_t r = g.entries[j];
            if ((int)(g.ptr[r + 1] - g.ptr[r]) != p) continue;
            if (mode == 1) {
                const double kr = keynorm[r];
                const double kmx = fmax(ki, kr);
                const double half = (g.crit == PR_CRIT_SPECTRAL) ? (g.eps * sqrt((double)p) * (1.0 + 1e-10) + c) * kmx
                                                                 : g.eps * (1.0 + 1e-10) + c * kmx;
                if (fabs(ki - kr) > half) continue;
            }
            if (pair_matches(g.crit, g.eps, sA, sX, sE, sH, g.X0 + j * g.stride, tile_of(g, r), p, lane, nev,
                             nex, nsq))
                hit = r;
        }
        if (lane == 0) {
            resolved[q] = hit >= 0 ? 1 : 0;
            if (hit >= 0) repof[i] = hit;
        }
        __syncthreads();
    }
    if (lane == 0) {
        atomicAdd(&counters[0], nev);
        if (nex) atomicAdd(&counters[1], nex);
        if (nsq) atomicAdd(&counters[3], nsq);
    }
}

// list compaction in order: out = ids[q] with keep[q] != want
__global__ void k_flag_not(int64_t n, const int32_t* __restrict__ keep, int want, int64_t* __restrict__ f) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) f[q] = (keep[q] == want) ? 1 : 0;
    else if (q == n) f[q] = 0;
}

__global__ void k_compact(int64_t n, const int32_t* __restrict__ ids, const int64_t* __restrict__ f,
                          const int64_t* __restrict__ pos, int32_t* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n && f[q]) out[pos[q]] = ids[q];
}

// dst[ids[q]] = src[ids[q]]
__global__ void k_copy_at(int64_t n, const int32_t* __restrict__ ids, const int32_t* __restrict__ src,
                          int32_t* __restrict__ dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[ids[q]] = src[ids[q]];
}

// out[q] = map[src[ids[q]]]  (labels of training rows, phi of all patches)
__global__ void k_map_at(int64_t n, const int32_t* __restrict__ ids, const int32_t* __restrict__ src,
                         const int32_t* __restrict__ map, int32_t* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int32_t i = ids ? ids[q] : (int32_t)q;
    out[q] = map[src[i]];
}

// size of each patch (row keys) and of each entry (class keys)
__global__ void k_sizes(int64_t n, const int32_t* __restrict__ ids, const int64_t* __restrict__ ptr,
                        int32_t* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t i = ids ? ids[q] : q;
    out[q] = (int32_t)(ptr[i + 1] - ptr[i]);
}

// dst rows r = src rows idx[r] (training minibatch), with labels and keys
__global__ void k_rows_gather(int64_t n, const int32_t* __restrict__ idx, const float* __restrict__ src, int F,
                              float* __restrict__ dst, const int32_t* __restrict__ lsrc, int32_t* __restrict__ ldst,
                              const int32_t* __restrict__ ksrc, int32_t* __restrict__ kdst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * F) return;
    const int64_t r = t / F;
    const int f = (int)(t % F);
    const int64_t q = idx[r];
    dst[t] = src[q * F + f];
    if (f == 0) {
        ldst[r] = lsrc[q];
        if (kdst) kdst[r] = ksrc[q];
    }
}

__global__ void k_set_at(int64_t n, const int32_t* __restrict__ ids, int32_t v, int32_t* __restrict__ dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[ids[q]] = v;
}

// training accuracy: top-1 equals the label
__global__ void k_count_eq(int64_t n, const int32_t* __restrict__ a, int sa, const int32_t* __restrict__ b,
                           unsigned long long* __restrict__ cnt) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n && a[q * sa] == b[q]) atomicAdd(cnt, 1ull);
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_mlp_features(int64_t n_p, const int64_t* ptr, const double* tiles, const int64_t* toff, int ups,
                         const uint32_t* bkeys, int pmax, float* out, hipStream_t s) {
    const unsigned g = (unsigned)(n_p < 65536 ? n_p : 65536);
    k_mlp_features<<<g, 64, 0, s>>>(n_p, ptr, tiles, toff, ups, bkeys, pmax, out);
}

void launch_mlp_moments(int64_t nrows, const int32_t* rows, const float* X, int F, float* mu, float* sd,
                        hipStream_t s) {
    k_mlp_moments<<<nb(F, 64), 64, 0, s>>>(nrows, rows, X, F, mu, sd);
}

void launch_mlp_gather(int64_t nrows, const int32_t* rows, const float* X, int F, const float* mu,
                       const float* sd, float* Xn, const int32_t* lab_src, int32_t* lab, const int32_t* key_src,
                       int32_t* key, hipStream_t s) {
    if (nrows <= 0) return;
    k_mlp_gather<<<nb(nrows * F, 256), 256, 0, s>>>(nrows, rows, X, F, mu, sd, Xn, lab_src, lab, key_src, key);
}

void launch_gemm(int prec, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B,
                 int ldb, float* C, int ldc, float alpha, const float* bias, int relu, const float* mask,
                 int ldm, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    if (prec == PR_FP16) {
        dim3 grid(nb(N, 32), nb(M, 32));
#define PR_G16(a, b) \
    k_gemm_f16<a, b><<<grid, 64, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, alpha, bias, relu, mask, ldm)
        if (!ta && !tb) PR_G16(false, false);
        else if (!ta && tb) PR_G16(false, true);
        else if (ta && !tb) PR_G16(true, false);
        else PR_G16(true, true);
#undef PR_G16
    } else {
        dim3 grid(nb(N, 16), nb(M, 16));
#define PR_G32(a, b) \
    k_gemm_f32<a, b><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, alpha, bias, relu, mask, ldm)
        if (!ta && !tb) PR_G32(false, false);
        else if (!ta && tb) PR_G32(false, true);
        else if (ta && !tb) PR_G32(true, false);
        else PR_G32(true, true);
#undef PR_G32
    }
}

void launch_softmax_ce(int B, int C, const float* L, int ldl, const int32_t* y, const int32_t* rkey,
                       const int32_t* ckey, float* G, int ldg, double* loss_rows, float scale, hipStream_t s) {
    if (B <= 0) return;
    k_softmax_ce<<<(unsigned)(B < 65536 ? B : 65536), 64, 0, s>>>(B, C, L, ldl, y, rkey, ckey, G, ldg, loss_rows,
                                                                  scale);
}

void launch_colsum(int B, int N, const float* G, int ldg, float scale, float* out, hipStream_t s) {
    if (N > 0) k_colsum<<<nb(N, 64), 256, 0, s>>>(B, N, G, ldg, scale, out);
}

void launch_adam(int64_t n, float* P, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, hipStream_t s) {
    k_adam<<<nb(n, 256), 256, 0, s>>>(n, P, g, m, v, lr, b1, b2, eps, bc1, bc2);
}

void launch_init_uniform(int64_t n, float* W, float a, uint64_t seed, uint64_t base, hipStream_t s) {
    if (n > 0) k_init_uniform<<<nb(n, 256), 256, 0, s>>>(n, W, a, seed, base);
}

void launch_topk(int64_t R, int C, const float* L, int ldl, int k, const int32_t* rkey, const int32_t* ckey,
                 int32_t* out, hipStream_t s) {
    if (R <= 0) return;
    k_topk<<<(unsigned)(R < 65536 ? R : 65536), 64, 0, s>>>(R, C, L, ldl, k, rkey, ckey, out);
}

void launch_mlp_match(int mode, int64_t nq, const int32_t* qids, const int32_t* cand, int k,
                      const int64_t* ptr, const double* tiles, const int64_t* toff, int ups,
                      const int32_t* entries, int64_t n0, const double* X0, int64_t stride, int crit, double eps,
                      const double* keynorm, int32_t* repof, int32_t* resolved, unsigned long long* counters,
                      hipStream_t s) {
    if (nq <= 0) return;
    PairGeom g{ptr, tiles, toff, ups, entries, n0, X0, stride, crit, eps};
    k_mlp_match<<<(unsigned)(nq < 16384 ? nq : 16384), 64, 0, s>>>(mode, nq, qids, cand, k, g, keynorm, repof,
                                                                   resolved, counters);
}

void launch_compact_flags(int64_t n, const int32_t* keep, int want, int64_t* f, hipStream_t s) {
    k_flag_not<<<nb(n + 1, 256), 256, 0, s>>>(n, keep, want, f);
}

void launch_compact(int64_t n, const int32_t* ids, const int64_t* f, const int64_t* pos, int32_t* out,
                    hipStream_t s) {
    if (n > 0) k_compact<<<nb(n, 256), 256, 0, s>>>(n, ids, f, pos, out);
}

void launch_copy_at(int64_t n, const int32_t* ids, const int32_t* src, int32_t* dst, hipStream_t s) {
    if (n > 0) k_copy_at<<<nb(n, 256), 256, 0, s>>>(n, ids, src, dst);
}

void launch_map_at(int64_t n, const int32_t* ids, const int32_t* src, const int32_t* map, int32_t* out,
                   hipStream_t s) {
    if (n > 0) k_map_at<<<nb(n, 256), 256, 0, s>>>(n, ids, src, map, out);
}

void launch_sizes(int64_t n, const int32_t* ids, const int64_t* ptr, int32_t* out, hipStream_t s) {
    if (n > 0) k_sizes<<<nb(n, 256), 256, 0, s>>>(n, ids, ptr, out);
}

void launch_count_eq(int64_t n, const int32_t* a, int sa, const int32_t* b, unsigned long long* cnt,
                     hipStream_t s) {
    if (n > 0) k_count_eq<<<nb(n, 256), 256, 0, s>>>(n, a, sa, b, cnt);
}

void launch_rows_gather(int64_t n, const int32_t* idx, const float* src, int F, float* dst, const int32_t* lsrc,
                        int32_t* ldst, const int32_t* ksrc, int32_t* kdst, hipStream_t s) {
    if (n > 0) k_rows_gather<<<nb(n * F, 256), 256, 0, s>>>(n, idx, src, F, dst, lsrc, ldst, ksrc, kdst);
}

void launch_set_at(int64_t n, const int32_t* ids, int32_t v, int32_t* dst, hipStream_t s) {
    if (n > 0) k_set_at<<<nb(n, 256), 256, 0, s>>>(n, ids, v, dst);
}
