// Dense per-patch kernels in FP64:
//  * batched inverse by Gauss-Jordan elimination with partial pivoting (the
//    factorisation of the database matrices; Section 4, Experiment 3 uses an
//    LU factorisation, whose explicit inverse is the same operator);
//  * the similarity criteria: d(A,B) = ||I - A B^{-1}||_2 (Eq.(5)) with the
//    largest singular value of E = I - A X from cyclic Jacobi on E^T E, and
//    the entrywise l1 / Frobenius differences (remark after Eq.(4));
// (Algorithm 1 itself is in k_alg1.hip.)
#include "dense_dev.h"

#include <climits>

namespace {

using namespace pr_dev;

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

