// FP64 vector kernels of the outer GMRES solve: CSR sparse matrix-vector
// product (optionally fused with a residual), block-partitioned multi-dot
// products with a fixed reduction order (results do not depend on timing),
// Gram-Schmidt updates, scaling and small basis combinations.
#include "pr_internal.h"

namespace {

constexpr int kRedThreads = 256;
constexpr int kMaxVec = 32;   // Krylov vectors per multidot call

// y = A x (b == nullptr) or y = b - A x; L lanes per row.
template <int L>
__global__ __launch_bounds__(256) void k_spmv(const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ val, int64_t n,
                                              const double* __restrict__ x,
                                              const double* __restrict__ b, double* __restrict__ y) {
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
    const int sub = threadIdx.x % L;
    if (row >= n) return;
    const int64_t s = rowptr[row], e = rowptr[row + 1];
    double acc = 0.0;
    for (int64_t q = s + sub; q < e; q += L) acc = fma(val[q], x[col[q]], acc);
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
    if (sub == 0) y[row] = b ? b[row] - acc : acc;
}

// partial[blk * nv + i] = sum over the block's rows of V_i * w ; then a
// second kernel sums the block partials in fixed order.
__global__ __launch_bounds__(kRedThreads) void k_multidot(const double* __restrict__ V, int64_t ldv,
                                                          int nv, const double* __restrict__ w,
                                                          int64_t n, double* __restrict__ partial) {
    __shared__ double s_red[kRedThreads / PR_WAVE][kMaxVec];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    double acc[kMaxVec];
#pragma unroll
    for (int i = 0; i < kMaxVec; ++i) acc[i] = 0.0;
    for (int64_t q = lo + threadIdx.x; q < hi; q += kRedThreads) {
        const double wv = w[q];
#pragma unroll
        for (int i = 0; i < kMaxVec; ++i)
            if (i < nv) acc[i] = fma(V[(int64_t)i * ldv + q], wv, acc[i]);
    }
    const int lane = threadIdx.x & (PR_WAVE - 1), wid = threadIdx.x / PR_WAVE;
#pragma unroll
    for (int i = 0; i < kMaxVec; ++i) {
        if (i < nv) {
            const double v = wave_sum(acc[i]);
            if (lane == 0) s_red[wid][i] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        double t = 0.0;
        for (int w2 = 0; w2 < kRedThreads / PR_WAVE; ++w2) t += s_red[w2][threadIdx.x];
        partial[(int64_t)blockIdx.x * nv + threadIdx.x] = t;
    }
}

__global__ void k_reduce_partials(const double* __restrict__ partial, int nblk, int nv,
                                  double* __restrict__ out) {
    const int i = threadIdx.x;
    if (i >= nv) return;
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += partial[(int64_t)b * nv + i];
    out[i] = t;
}

// w += sign * sum_i h_i V_i
__global__ void k_update(double* __restrict__ w, const double* __restrict__ V, int64_t ldv, int nv,
                         const double* __restrict__ h, double sign, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double acc = w[q];
    for (int i = 0; i < nv; ++i) acc = fma(sign * h[i], V[(int64_t)i * ldv + q], acc);
    w[q] = acc;
}

// dst = src / sqrt(denom[0])   (denom holds a squared norm)
__global__ void k_scale(const double* __restrict__ src, double* __restrict__ dst,
                        const double* __restrict__ denom, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double d = sqrt(denom[0]);
    dst[q] = d > 0.0 ? src[q] / d : 0.0;
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = fma(a, x[q], y[q]);
}

__global__ void k_gemv_small(const double* __restrict__ V, int64_t ldv, int nv,
                             const double* __restrict__ c, int64_t n, double* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc = fma(c[i], V[(int64_t)i * ldv + q], acc);
    out[q] = acc;
}

__global__ void k_zero(double* x, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) x[q] = 0.0;
}

// ---------------------------------------------------------------------------
// Fused Gram-Schmidt passes (classical Gram-Schmidt applied twice):
//   MODE 0: out_i = V_i . w                       (i < nv)
//   MODE 1: w <- w - sum_i c_i V_i ; out_i = V_i . w   (each V_i loaded once)
//   MODE 2: w <- w - sum_i c_i V_i ; out_0 = w . w
// Each block reduces its rows; the last block to finish (ticket counter)
// sums the block partials in a fixed order, so results do not depend on
// timing.  The counter is returned to zero by that block.
// ---------------------------------------------------------------------------
constexpr int kGsThreads = 256;

template <int MODE>
__global__ __launch_bounds__(kGsThreads) void k_gs(const double* __restrict__ V, int64_t ldv, int nv,
                                                   double* __restrict__ w, int64_t n,
                                                   const double* __restrict__ c,
                                                   double* __restrict__ partial,
                                                   unsigned int* __restrict__ counter,
                                                   double* __restrict__ out) {
    constexpr int NO = (MODE == 2) ? 1 : kMaxVec;
    __shared__ double s_red[kGsThreads / PR_WAVE][kMaxVec];
    __shared__ bool s_last;
    const int nout = (MODE == 2) ? 1 : nv;
    double cf[kMaxVec];
    if (MODE >= 1) {
#pragma unroll
        for (int i = 0; i < kMaxVec; ++i) cf[i] = (i < nv) ? c[i] : 0.0;
    }
    double acc[NO];
#pragma unroll
    for (int i = 0; i < NO; ++i) acc[i] = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    for (int64_t q = lo + threadIdx.x; q < hi; q += kGsThreads) {
        double wq = w[q];
        if (MODE == 0) {
#pragma unroll
            for (int i = 0; i < kMaxVec; ++i)
                if (i < nv) acc[i] = fma(V[(int64_t)i * ldv + q], wq, acc[i]);
        } else {
            double v[kMaxVec];
#pragma unroll
            for (int i = 0; i < kMaxVec; ++i) v[i] = (i < nv) ? V[(int64_t)i * ldv + q] : 0.0;
#pragma unroll
            for (int i = 0; i < kMaxVec; ++i)
                if (i < nv) wq = fma(-cf[i], v[i], wq);
            w[q] = wq;
            if (MODE == 1) {
#pragma unroll
                for (int i = 0; i < kMaxVec; ++i)
                    if (i < nv) acc[i] = fma(v[i], wq, acc[i]);
            } else {
                acc[0] = fma(wq, wq, acc[0]);
            }
        }
    }
    const int lane = threadIdx.x & (PR_WAVE - 1), wid = threadIdx.x / PR_WAVE;
#pragma unroll
    for (int i = 0; i < NO; ++i) {
        if (i < nout) {
            const double t = wave_sum(acc[i]);
            if (lane == 0) s_red[wid][i] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nout) {
        double t = 0.0;
        for (int w2 = 0; w2 < kGsThreads / PR_WAVE; ++w2) t += s_red[w2][threadIdx.x];
        partial[(int64_t)blockIdx.x * kMaxVec + threadIdx.x] = t;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int ticket = atomicAdd(counter, 1u);
        s_last = (ticket == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // last block: out_i = sum_b partial[b][i], fixed partition and tree
    double tot[NO];
#pragma unroll
    for (int i = 0; i < NO; ++i) tot[i] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kGsThreads) {
#pragma unroll
        for (int i = 0; i < NO; ++i)
            if (i < nout) tot[i] += partial[(int64_t)b * kMaxVec + i];
    }
#pragma unroll
    for (int i = 0; i < NO; ++i) {
        if (i < nout) {
            const double t = wave_sum(tot[i]);
            if (lane == 0) s_red[wid][i] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nout) {
        double t = 0.0;
        for (int w2 = 0; w2 < kGsThreads / PR_WAVE; ++w2) t += s_red[w2][threadIdx.x];
        out[threadIdx.x] = t;
    }
    if (threadIdx.x == 0) *counter = 0u;
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_spmv(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n,
                 const double* x, const double* b, double* y, int avg_nnz, hipStream_t s) {
    if (n <= 0) return;
    if (avg_nnz <= 6)
        k_spmv<4><<<nb(n * 4, 256), 256, 0, s>>>(rowptr, col, val, n, x, b, y);
    else if (avg_nnz <= 14)
        k_spmv<8><<<nb(n * 8, 256), 256, 0, s>>>(rowptr, col, val, n, x, b, y);
    else if (avg_nnz <= 40)
        k_spmv<16><<<nb(n * 16, 256), 256, 0, s>>>(rowptr, col, val, n, x, b, y);
    else
        k_spmv<32><<<nb(n * 32, 256), 256, 0, s>>>(rowptr, col, val, n, x, b, y);
}

int reduce_blocks(int64_t n) {
    int64_t b = (n + 4095) / 4096;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

void launch_multidot(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
                     double* partial, double* out, hipStream_t s) {
    const int nbk = reduce_blocks(n);
    for (int base = 0; base < nv; base += kMaxVec) {
        const int cnt = nv - base < kMaxVec ? nv - base : kMaxVec;
        k_multidot<<<nbk, kRedThreads, 0, s>>>(V + (int64_t)base * ldv, ldv, cnt, w, n, partial);
        k_reduce_partials<<<1, kMaxVec, 0, s>>>(partial, nbk, cnt, out + base);
    }
}

void launch_update(double* w, const double* V, int64_t ldv, int nv, const double* h, double sign,
                   int64_t n, hipStream_t s) {
    if (n > 0 && nv > 0) k_update<<<nb(n, 256), 256, 0, s>>>(w, V, ldv, nv, h, sign, n);
}

void launch_scale(const double* src, double* dst, const double* denom, int64_t n, hipStream_t s) {
    if (n > 0) k_scale<<<nb(n, 256), 256, 0, s>>>(src, dst, denom, n);
}

void launch_axpy_dev(double* y, const double* x, double a, int64_t n, hipStream_t s) {
    if (n > 0) k_axpy<<<nb(n, 256), 256, 0, s>>>(y, x, a, n);
}

void launch_gemv_small(const double* V, int64_t ldv, int nv, const double* coef, int64_t n,
                       double* out, hipStream_t s) {
    if (n > 0) k_gemv_small<<<nb(n, 256), 256, 0, s>>>(V, ldv, nv, coef, n, out);
}

void launch_zero(double* x, int64_t n, hipStream_t s) {
    if (n > 0) k_zero<<<nb(n, 256), 256, 0, s>>>(x, n);
}

int gs_blocks(int64_t n) {
    int64_t b = (n + 2047) / 2048;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

// mode 0: out = V^T w ; mode 1: w -= V c, out = V^T w ; mode 2: w -= V c, out[0] = w.w
// partial: gs_blocks(n) * 32 doubles; counter: one zeroed unsigned int.
void launch_gs(int mode, const double* V, int64_t ldv, int nv, double* w, int64_t n, const double* c,
               double* partial, unsigned int* counter, double* out, hipStream_t s) {
    const int nbk = gs_blocks(n);
    for (int base = 0; base < nv || (nv == 0 && base == 0); base += kMaxVec) {
        const int cnt = nv - base < kMaxVec ? nv - base : kMaxVec;
        const double* Vb = V + (int64_t)base * ldv;
        if (mode == 0)
            k_gs<0><<<nbk, kGsThreads, 0, s>>>(Vb, ldv, cnt, w, n, c, partial, counter, out + base);
        else if (mode == 1)
            k_gs<1><<<nbk, kGsThreads, 0, s>>>(Vb, ldv, cnt, w, n, c + base, partial, counter, out + base);
        else
            k_gs<2><<<nbk, kGsThreads, 0, s>>>(Vb, ldv, cnt, w, n, c + base, partial, counter, out);
        if (nv == 0) break;
    }
}
