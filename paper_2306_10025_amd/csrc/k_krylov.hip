// FP64 kernels of the outer GMRES solve (right preconditioning, Section 4):
// sliced-ELL sparse matrix-vector product (optionally fused with a residual),
// fused classical Gram-Schmidt passes with block-partitioned reductions in a
// fixed order (results do not depend on timing), the Givens rotations and
// the small triangular solve on the device, and basis combinations.
//
// Kernels that run inside an Arnoldi step take a `stop` flag (device int);
// once the device-side Givens update has met the stopping test they return
// at once, so the host can enqueue a whole restart cycle without waiting.
#include "pr_internal.h"

namespace {

constexpr int kMaxVec = 32;   // Krylov vectors per Gram-Schmidt launch
constexpr int kGsThreads = 256;
constexpr int kEndThreads = 256;   // step-end kernels
constexpr int kEndBlocks = 1024;

__device__ __forceinline__ bool stopped(const int32_t* stop) { return stop && *stop; }

// ---------------------------------------------------------------------------
// Hybrid sliced ELLPACK copy of A: slices of 64 rows, one wavefront each,
// column-major inside a slice (every lane streams its row at unit stride
// across the wave).  Each slice takes one of two forms:
//   diagonal (sfmt 1): the sorted distinct offsets d = col - row of the
//     slice's entries, one int32 per slice column, and a value for every
//     (row, offset), 0 where the row has no entry there: 8 bytes per stored
//     value, the column computed as row + d;
//   column (sfmt 0): each row's entries padded to the slice's longest row,
//     with their column indices: 12 bytes per stored value.
// The plan takes the diagonal form when it stores fewer bytes
// (8 ndiag <= 12 mlen) and ndiag <= kSellMaxDiag.  Matrices
// of structured meshes put most slices in the diagonal form; mixed
// discretisations (several field types per row block) stay in the column
// form.  Padding and absent diagonal entries hold 0 and contribute exact
// zeros for finite x.
// ---------------------------------------------------------------------------
constexpr int kPlanThreads = 256;
constexpr int kPlanTab = 1024;      // LDS hash set of a slice's offsets
constexpr int kMaxDiag = kSellMaxDiag;   // distinct offsets of one diagonal slice

__device__ __forceinline__ uint32_t offset_hash(int32_t d) { return ((uint32_t)d * 2654435761u) >> 22; }

// One block per slice (block ns writes the scan's closing 0): slen[sl] = 64 *
// stored columns, sfmt[sl], the slice's sorted distinct offsets in
// dtmp[sl * kMaxDiag ..] (diagonal form), and the totals in acc: [0] diagonal
// slices, [1] their offsets, [2] entries of column-form slices.  The offsets
// go into an LDS hash set (four lanes per row); a slice with more than fits
// the set takes the column form.
__global__ __launch_bounds__(kPlanThreads) void k_sell_plan(const int64_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ col, int64_t n,
                                                            int64_t* __restrict__ slen, int32_t* __restrict__ sfmt,
                                                            int32_t* __restrict__ dtmp,
                                                            int32_t* __restrict__ cnnz) {
    __shared__ int32_t tab[kPlanTab];
    __shared__ int32_t lst[kPlanThreads];
    __shared__ int s_mlen, s_nnz, s_cnt, s_over, s_pos;
    const int64_t ns = (n + 63) / 64;
    const int64_t sl = blockIdx.x;
    const int t = threadIdx.x;
    if (sl >= ns) {
        if (t == 0) slen[ns] = 0;
        return;
    }
    const int64_t r0 = sl * 64;
    const int rows = (int)(n - r0 < 64 ? n - r0 : 64);
    if (t == 0) {
        s_mlen = 0;
        s_nnz = 0;
        s_cnt = 0;
        s_over = 0;
        s_pos = 0;
    }
    for (int e = t; e < kPlanTab; e += kPlanThreads) tab[e] = INT_MAX;
    lst[t] = INT_MAX;
    __syncthreads();
    // four lanes per row: rows w * 16 .. w * 16 + 15 for wavefront w
    const int i = (t >> 6) * 16 + ((t & 63) >> 2), sub = t & 3;
    int64_t a = 0, l = 0;
    if (i < rows) {
        a = rowptr[r0 + i];
        l = rowptr[r0 + i + 1] - a;
        if (sub == 0) {
            atomicMax(&s_mlen, (int)l);
            atomicAdd(&s_nnz, (int)l);
        }
    }
    __syncthreads();
    // a row holds distinct offsets, so a slice whose longest row exceeds
    // kMaxDiag takes the column form without collecting its offsets
    const bool collect = s_mlen <= kMaxDiag;
    // rows of a slice mostly share their offsets: each step the wavefront
    // reduces its 64 offsets to one lane per distinct value, and a slot is
    // read before the atomic is tried; collection stops once the slice has
    // more offsets than the diagonal form allows
    int64_t lmax = collect ? l : 0;
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(lmax, o);
        lmax = u > lmax ? u : lmax;
    }
    for (int64_t k0 = 0; k0 < lmax; k0 += 4) {
        if (s_cnt > kMaxDiag) break;                 // one LDS read for the whole wavefront
        const int64_t k = k0 + sub;
        bool pending = k < l;
        const int32_t d = (int32_t)((int64_t)col[pending ? a + k : 0] - (r0 + i));
        for (;;) {
            const uint64_t m = __ballot(pending);
            if (m == 0) break;
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int32_t dl = __shfl(d, leader);
            if (pending && d == dl) pending = false;
            if ((t & 63) == leader) {
                uint32_t slot = offset_hash(dl);
                for (int probe = 0; probe < kPlanTab; ++probe) {
                    const int32_t seen = tab[slot];
                    if (seen == dl) break;
                    if (seen == INT_MAX) {
                        const int32_t prev = atomicCAS(&tab[slot], INT_MAX, dl);
                        if (prev == INT_MAX) {
                            atomicAdd(&s_cnt, 1);
                            break;
                        }
                        if (prev == dl) break;
                    }
                    slot = (slot + 1) & (kPlanTab - 1);
                    if (probe == kPlanTab - 1) s_over = 1;     // the set is full
                }
            }
        }
    }
    __syncthreads();
    const int mlen = s_mlen, ndiag = s_cnt;
    int fmt = (collect && !s_over && mlen > 0 && 2 * ndiag <= 3 * mlen && ndiag <= kMaxDiag) ? 1 : 0;
    // long rows of very different lengths (high-order cells: 216 to 1331
    // entries in one slice) would pad the column form by more than 30 %: the
    // slice's rows are then read from the CSR copy, 16 lanes per row
    if (!fmt && rows > 0 && 10 * (int64_t)mlen * rows > 13 * (int64_t)s_nnz && s_nnz >= 32 * rows) fmt = 2;
    if (fmt) {
        // the set as a list, sorted (at most kMaxDiag values in kPlanThreads slots)
        for (int e = t; e < kPlanTab; e += kPlanThreads) {
            const int32_t d = tab[e];
            if (d != INT_MAX) lst[atomicAdd(&s_pos, 1)] = d;
        }
        __syncthreads();
        for (int k = 2; k <= kPlanThreads; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int f = t ^ j;
                if (f > t) {
                    const int32_t x0 = lst[t], x1 = lst[f];
                    if ((x0 > x1) == ((t & k) == 0)) {
                        lst[t] = x1;
                        lst[f] = x0;
                    }
                }
                __syncthreads();
            }
        }
        if (t < ndiag) dtmp[sl * kMaxDiag + t] = lst[t];
        // an odd count gets a padding diagonal (the last offset again, zero
        // values): the values are stored in pairs of diagonals (the column
        // form likewise stores an even number of slots per row)
        if (fmt == 1 && (ndiag & 1) && t == ndiag) dtmp[sl * kMaxDiag + t] = lst[ndiag - 1];
    }
    if (t == 0) {
        slen[sl] = fmt == 2 ? 0 : 64 * (int64_t)(fmt ? ndiag + (ndiag & 1) : mlen + (mlen & 1));
        sfmt[sl] = fmt;
        cnnz[sl] = fmt == 0 ? s_nnz : (fmt == 2 ? -s_nnz : 0);   // form 2: its entries, negated
    }
}

// acc[5] += {diagonal slices, their offsets, entries of column-form slices,
// CSR-row slices, their entries}:
// a grid-stride sum per block, three atomics per block (one atomic per slice
// on three addresses serialised into hundreds of microseconds)
constexpr int kTotalsBlocks = 128;
__global__ __launch_bounds__(256) void k_sell_totals(const int64_t* __restrict__ slen, const int32_t* __restrict__ sfmt,
                                                     const int32_t* __restrict__ cnnz, int64_t ns,
                                                     unsigned long long* __restrict__ acc) {
    __shared__ unsigned long long s_a[5][256 / PR_WAVE];
    unsigned long long a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
    for (int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < ns; sl += (int64_t)gridDim.x * blockDim.x) {
        const int f = sfmt[sl];
        a0 += f == 1 ? 1ull : 0ull;
        a1 += f == 1 ? (unsigned long long)(slen[sl] / 64) : 0ull;
        a2 += f == 0 ? (unsigned long long)cnnz[sl] : 0ull;
        a3 += f == 2 ? 1ull : 0ull;
        a4 += f == 2 ? (unsigned long long)(-(int64_t)cnnz[sl]) : 0ull;
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    a3 = wave_sum(a3);
    a4 = wave_sum(a4);
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) {
        s_a[0][threadIdx.x / PR_WAVE] = a0;
        s_a[1][threadIdx.x / PR_WAVE] = a1;
        s_a[2][threadIdx.x / PR_WAVE] = a2;
        s_a[3][threadIdx.x / PR_WAVE] = a3;
        s_a[4][threadIdx.x / PR_WAVE] = a4;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long u = 0;
        for (int w = 0; w < 256 / PR_WAVE; ++w) u += s_a[threadIdx.x][w];
        atomicAdd(&acc[threadIdx.x], u);
    }
}

// Column-form slices: one thread per row.
__global__ void k_sell_fill(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, int64_t n, const int64_t* __restrict__ soff,
                            const int32_t* __restrict__ sfmt, double* __restrict__ sval,
                            int32_t* __restrict__ scol) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t sl = r / 64, lane = r % 64;
    if (sfmt[sl]) return;
    const int64_t off = soff[sl];
    const int64_t len = (soff[sl + 1] - off) / 64;
    const int64_t a = rowptr[r], l = rowptr[r + 1] - a;
    // loads unconditional from clamped addresses, in groups of 8 (a load
    // under a condition becomes a branch that waits for it)
    for (int64_t k0 = 0; k0 < len; k0 += 8) {
        double vv[8];
        int32_t cc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t k = k0 + u;
            const int64_t ks = (k < l) ? k : 0;
            vv[u] = l > 0 ? val[a + ks] : 0.0;
            cc[u] = l > 0 ? col[a + ks] : (int32_t)r;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t k = k0 + u;
            if (k < len) {
                // slots in pairs: slot k of row i at (k / 2) * 128 + 2 i + k % 2
                const bool v = k < l;
                const int64_t at = off + (k >> 1) * 128 + 2 * lane + (k & 1);
                sval[at] = v ? vv[u] : 0.0;
                scol[at] = v ? cc[u] : (int32_t)r;
            }
        }
    }
}

// Diagonal-form slices: one block per slice.  Every stored value is first
// set to 0; after the barrier each entry (four lanes per row) finds its
// offset's column by binary search and writes its value.  Values are stored
// in pairs of diagonals: diagonal k of row i at (k / 2) * 128 + 2 i + k % 2,
// so one 16-byte load gives a row its values on two diagonals.
__global__ __launch_bounds__(kPlanThreads) void k_sell_fill_diag(const int64_t* __restrict__ rowptr,
                                                                 const int32_t* __restrict__ col,
                                                                 const double* __restrict__ val, int64_t n,
                                                                 const int64_t* __restrict__ soff,
                                                                 const int32_t* __restrict__ sfmt,
                                                                 const int32_t* __restrict__ dtmp,
                                                                 double* __restrict__ sval,
                                                                 int32_t* __restrict__ sdoff) {
    __shared__ int32_t s_d[kMaxDiag];
    const int64_t sl = blockIdx.x;
    if (sfmt[sl] != 1) return;
    const int t = threadIdx.x;
    const int64_t off = soff[sl];
    const int nd = (int)((soff[sl + 1] - off) / 64);
    for (int k = t; k < nd; k += kPlanThreads) {
        const int32_t d = dtmp[sl * kMaxDiag + k];
        s_d[k] = d;
        sdoff[off / 64 + k] = d;
    }
    for (int64_t e = t; e < (int64_t)nd * 64; e += kPlanThreads) sval[off + e] = 0.0;
    __syncthreads();
    const int64_t r0 = sl * 64;
    const int rows = (int)(n - r0 < 64 ? n - r0 : 64);
    const int i = (t >> 6) * 16 + ((t & 63) >> 2), sub = t & 3;
    if (i >= rows) return;
    const int64_t a = rowptr[r0 + i], l = rowptr[r0 + i + 1] - a;
    for (int64_t k = sub; k < l; k += 4) {
        const int32_t d = (int32_t)((int64_t)col[a + k] - (r0 + i));
        int lo = 0, hi = nd - 1;          // s_d[lo] == d at the end
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_d[mid] < d) lo = mid + 1;
            else hi = mid;
        }
        sval[off + (int64_t)(lo >> 1) * 128 + 2 * i + (lo & 1)] = val[a + k];
    }
}

constexpr int kSpmvChunk = 8;   // diagonal-form entries per step (even)
static_assert(kSpmvChunk <= kSellOffsetPad, "the offset array's padding covers one step");

typedef double dpair __attribute__((ext_vector_type(2)));

// One step of the diagonal form: kSpmvChunk diagonals from k0 (kSpmvChunk / 2
// pairs).  Bit u of ADJ says that pair u's offsets are adjacent (d1 = d0 + 1),
// so one 16-byte gather brings x[c0] and x[c0 + 1]: its address is clamped
// into [0, n - 2], and at the matrix's ends the shift picks the element (a
// column outside the matrix has a zero value).  Every load of the step is
// issued before the first product; ADJ is a template argument so that the
// step has no branch between its loads (a branch per pair made the compiler
// wait for each pair's gathers at the join).
template <int ADJ>
__device__ __forceinline__ void spmv_diag_step(const dpair* __restrict__ vq, const int32_t* __restrict__ dp,
                                               const double* __restrict__ x, int64_t n, int64_t r, int k0,
                                               int len, double& acc0, double& acc1) {
    constexpr int NP = kSpmvChunk / 2;
    const int npair = len / 2;
    dpair v[NP];
    double xv[kSpmvChunk];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        const int q = k0 / 2 + u < npair ? k0 / 2 + u : npair - 1;
        v[u] = __builtin_nontemporal_load(vq + (int64_t)q * 64);
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        const int32_t d0 = dp[k0 + 2 * u], d1 = dp[k0 + 2 * u + 1];
        const int64_t c0 = r + d0;
        if (((ADJ >> u) & 1) != 0) {      // folded: the loop is unrolled
            const int64_t cp = c0 < 0 ? 0 : (c0 > n - 2 ? n - 2 : c0);
            dpair x2;
            __builtin_memcpy(&x2, x + cp, sizeof(x2));
            const int64_t sh = c0 - cp;
            xv[2 * u] = sh == 1 ? x2.y : x2.x;
            xv[2 * u + 1] = sh == -1 ? x2.x : x2.y;
        } else {
            const int64_t c1 = r + d1;
            xv[2 * u] = x[(uint64_t)c0 < (uint64_t)n ? c0 : r];
            xv[2 * u + 1] = x[(uint64_t)c1 < (uint64_t)n ? c1 : r];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        if (k0 + 2 * u < len) acc0 = fma(v[u].x, xv[2 * u], acc0);
        if (k0 + 2 * u + 1 < len) acc1 = fma(v[u].y, xv[2 * u + 1], acc1);
    }
}

// y = A x (b == nullptr) or y = b - A x; one thread per row, 64-row slices.
// The matrix values are read once per product: in the diagonal and column
// forms non-temporal loads keep them from displacing what the solve reads
// again (x, the Krylov basis, the preconditioner's data) in the caches (on
// the Nedelec 64^3 solve the apply between two products went from 30.3 to
// 25.0 us and Gram-Schmidt from 65.8 to 61.1 us per step).  The CSR-row form
// keeps ordinary loads: its 16-lane row reads ran 8 % slower with the hint.
__global__ __launch_bounds__(256) void k_spmv_sell(SellMat M, int64_t n, const double* __restrict__ x,
                                                   const double* __restrict__ b, double* __restrict__ y,
                                                   const int32_t* __restrict__ stop) {
    // the stop flag is read before the store, not here: at entry its two
    // dependent scalar loads came ahead of the slice descriptors
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // one slice per wavefront: its descriptors are wave-uniform (scalar loads)
    const int64_t sl = __builtin_amdgcn_readfirstlane((int)(r / 64));
    const int lane = (int)(r % 64);
    // the grid is rounded up to whole blocks: wavefronts past the last
    // slice hold no slice (its descriptors end at slice (n + 63) / 64 - 1)
    if (sl >= (n + 63) / 64) return;
    const int fmt = M.sfmt[sl];
    // padding lanes of the last slice hold no entries; the CSR-row form
    // needs every lane of the wavefront
    if (r >= n && fmt != 2) return;
    const int64_t off = M.soff[sl];
    const int len = (int)((M.soff[sl + 1] - off) / 64);
    double acc0 = 0.0, acc1 = 0.0;
    if (fmt == 2) {
        // rows from the CSR copy: lane group g (16 lanes) takes rows g, g + 4,
        // ...; lane t of a group takes the entry pairs a + 2 t + 32 u (u < 4)
        // of each 128-entry step, one 16-byte value load and one 8-byte
        // column load per pair (the copy is padded by kCsrPad zero entries, so
        // a pair that starts at the row's end, or is clamped there, stays
        // inside it), eight gathers of x in flight, a 16-lane sum; the 64 row
        // sums return to their lanes through LDS.  (One entry per load made
        // the address units the limit.)
        __shared__ double s_row[256];
        const int wbase = (int)(threadIdx.x & ~(PR_WAVE - 1));
        const int grp = lane >> 4, sub = lane & 15;
        const int64_t r0 = sl * 64;
        for (int rr = grp; rr < 64; rr += 4) {
            const int64_t row = r0 + rr;
            double sacc = 0.0;
            if (row < n) {
                const int64_t a = M.rowptr[row], e = M.rowptr[row + 1];
                for (int64_t q0 = a + 2 * sub; q0 < e; q0 += 128) {
                    dpair v[4];
                    int32_t cc[8];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t q = q0 + 32 * u;
                        const int64_t qc = q < e ? q : e;
                        dpair vv;
                        int2 c2;
                        __builtin_memcpy(&vv, M.val + qc, sizeof(vv));
                        __builtin_memcpy(&c2, M.col + qc, sizeof(c2));
                        v[u].x = q < e ? vv.x : 0.0;
                        v[u].y = q + 1 < e ? vv.y : 0.0;
                        cc[2 * u] = c2.x;
                        cc[2 * u + 1] = c2.y;
                    }
                    double xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) xv[u] = x[cc[u]];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        sacc = fma(v[u].x, xv[2 * u], sacc);
                        sacc = fma(v[u].y, xv[2 * u + 1], sacc);
                    }
                }
            }
            for (int o = 8; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, 16);
            if (sub == 0) s_row[wbase + rr] = sacc;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        acc0 = s_row[wbase + lane];
    } else if (fmt == 1) {
        // diagonal form, values in pairs of diagonals (an odd count padded
        // with a zero diagonal): one 16-byte load per pair.  Neither the
        // values nor the gathers depend on earlier loads, so kSpmvChunk
        // diagonals' worth of each are issued together, and the entries
        // alternate between the two accumulators by column parity.  Past
        // the slice's last column the offsets read are whatever follows (the
        // offset array is padded by kSellOffsetPad), the column is clamped
        // into range, the pair index to the last pair, and the product is
        // dropped.  (Taking the slice's offsets in one vector load and each
        // step's by readlane measured the same, 60.5 against 60.2 us on the
        // Nedelec 64^3 matrix: other wavefronts hide the scalar loads.)
        static_assert(kSpmvChunk == 8, "four pairs per step: sixteen adjacency patterns");
        const dpair* vq = reinterpret_cast<const dpair*>(M.sval + off) + lane;
        const int32_t* dp = M.sdoff + off / 64;
        for (int k0 = 0; k0 < len; k0 += kSpmvChunk) {
            int adj = 0;
#pragma unroll
            for (int u = 0; u < kSpmvChunk / 2; ++u)
                adj |= (dp[k0 + 2 * u + 1] == dp[k0 + 2 * u] + 1 && n >= 2) ? (1 << u) : 0;
            switch (adj) {
#define PR_DIAG(A) case A: spmv_diag_step<A>(vq, dp, x, n, r, k0, len, acc0, acc1); break;
                PR_DIAG(0) PR_DIAG(1) PR_DIAG(2) PR_DIAG(3) PR_DIAG(4) PR_DIAG(5) PR_DIAG(6) PR_DIAG(7)
                PR_DIAG(8) PR_DIAG(9) PR_DIAG(10) PR_DIAG(11) PR_DIAG(12) PR_DIAG(13) PR_DIAG(14) PR_DIAG(15)
#undef PR_DIAG
            }
        }
    } else {
        // column form, slots in pairs (an even count per row, padded with
        // zero values on the row's own column): one 16-byte value load and
        // one 8-byte column load per pair, two pairs per step
        const dpair* vq = reinterpret_cast<const dpair*>(M.sval + off) + lane;
        const int2* cq = reinterpret_cast<const int2*>(M.scol + off) + lane;
        const int npair = len / 2;
        int q = 0;
        for (; q + 2 <= npair; q += 2) {
            const dpair v0 = __builtin_nontemporal_load(vq + (int64_t)q * 64),
                        v1 = __builtin_nontemporal_load(vq + (int64_t)(q + 1) * 64);
            const int2 c0 = cq[(int64_t)q * 64], c1 = cq[(int64_t)(q + 1) * 64];
            acc0 = fma(v0.x, x[c0.x], acc0);
            acc1 = fma(v0.y, x[c0.y], acc1);
            acc0 = fma(v1.x, x[c1.x], acc0);
            acc1 = fma(v1.y, x[c1.y], acc1);
        }
        if (q < npair) {
            const dpair v0 = __builtin_nontemporal_load(vq + (int64_t)q * 64);
            const int2 c0 = cq[(int64_t)q * 64];
            acc0 = fma(v0.x, x[c0.x], acc0);
            acc1 = fma(v0.y, x[c0.y], acc1);
        }
    }
    const double acc = acc0 + acc1;
    if (stopped(stop)) return;
    if (r < n) y[r] = b ? b[r] - acc : acc;
}

// Selective reorthogonalisation (the test of Daniel, Gragg, Kaufman and
// Stewart, 1976): after w' = w - V (V^T w), a second projection is needed
// only when ||w'||^2 < ||w||^2 / 2, i.e. the first lost more than a factor
// sqrt(2) to cancellation.  sel[kSelIn] = ||w||^2, sel[kSelProj] = ||w'||^2;
// every kernel that depends on the decision evaluates this same predicate.
constexpr int kSelIn = 32, kSelProj = 96;
__device__ __forceinline__ bool reorth_needed(const double* sel) {
    return !(sel[kSelProj] >= 0.5 * sel[kSelIn]);
}

// ---------------------------------------------------------------------------
// Fused Gram-Schmidt passes (classical Gram-Schmidt applied twice):
//   MODE 0: out_i = V_i . w                       (i < nv)
//   MODE 1: w <- w - sum_i c_i V_i ; out_i = V_i . w   (each V_i loaded once)
//   MODE 2: w <- w - sum_i c_i V_i ; out_0 = w . w
// Each block writes its row-range partial sums; k_gs_final (modes 0 and 1)
// or k_step_end (mode 2) adds the block partials in a fixed tree.
// NC = ceil(nv / 8) is a template parameter: the NC * 8 vector loads of a
// row carry no branches between them (indices past nv repeat vector nv - 1
// and their terms are dropped), so they are all in flight at once.
// ---------------------------------------------------------------------------
template <int MODE, int NC>
__global__ __launch_bounds__(kGsThreads) void k_gs(const double* __restrict__ V, int64_t ldv, int nv,
                                                   double* __restrict__ w, int64_t n,
                                                   const double* __restrict__ c,
                                                   double* __restrict__ partial,
                                                   const int32_t* __restrict__ stop, int extra,
                                                   const double* __restrict__ sel) {
    // the dot pass (MODE 0) only writes its partials: it reads the stop flag
    // before them, not ahead of its first loads
    if (MODE != 0 && stopped(stop)) return;
    if (MODE == 2 && sel && !reorth_needed(sel)) return;
    constexpr int NV = 8 * NC;
    constexpr int NO = (MODE == 2) ? 1 : NV;
    __shared__ double s_red[kGsThreads / PR_WAVE][kMaxVec];
    const int nout = (MODE == 2) ? 1 : nv;
    double accw = 0.0;       // extra output nv: w . w (MODE 0) or the updated w . w (MODE 1)
    double cf[NV];
    if (MODE >= 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) cf[i] = (i < nv) ? c[i] : 0.0;
    }
    int64_t vo[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vo[i] = (int64_t)(i < nv ? i : (nv > 0 ? nv - 1 : 0)) * ldv;
    double acc[NO];
#pragma unroll
    for (int i = 0; i < NO; ++i) acc[i] = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    for (int64_t q = lo + threadIdx.x; q < hi; q += kGsThreads) {
        double wq = w[q];
        double v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = V[vo[i] + q];
        // keep every load of the row ahead of the arithmetic: left to itself
        // the scheduler interleaves them to save registers and keeps only
        // two loads in flight per wave
        __builtin_amdgcn_sched_barrier(0);
        if (MODE == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] = fma(v[i], wq, acc[i]);
            accw = fma(wq, wq, accw);
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) wq = fma(-cf[i], v[i], wq);    // cf = 0 past nv
            w[q] = wq;
            if (MODE == 1) {
#pragma unroll
                for (int i = 0; i < NV; ++i) acc[i] = fma(v[i], wq, acc[i]);
                accw = fma(wq, wq, accw);
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
    if (MODE != 2 && extra) {
        const double t = wave_sum(accw);
        if (lane == 0) s_red[wid][nout] = t;
    }
    __syncthreads();
    if (MODE == 0 && stopped(stop)) return;   // uniform: the whole block leaves
    const int nall = nout + ((MODE != 2 && extra) ? 1 : 0);
    if (threadIdx.x < nall) {
        double t = 0.0;
        for (int w2 = 0; w2 < kGsThreads / PR_WAVE; ++w2) t += s_red[w2][threadIdx.x];
        // output-major (output o of block b at o * gridDim.x + b): a consumer
        // reads each output's block partials as one contiguous run
        partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// Gram-Schmidt with delayed reorthogonalisation (two passes over the basis
// per Arnoldi step instead of three).  At step j the basis holds the final
// v_0 .. v_{j-1} (Q) and, in column j, u_raw = s u: the next vector after one
// projection, not normalised (s = ||u_raw||; s = 1 for v_0); w_raw = A M u_raw.
//   dot pass (k_gs MODE 0 over the j + 1 columns): b' = Q^T w_raw and
//     beta' = u_raw . w_raw;
//   update pass (k_gs_upd): v_j = (u_raw / s - Q a) / nu written over
//     column j, w_new = (w_raw / s - Q c - c_j v_j) / nu written unnormalised
//     to column j + 1, and the partials of [Q, v_j]^T w_new and
//     w_new . w_new, which are the next step's a' and s^2: the
//     reorthogonalisation coefficients of the next vector come out of this
//     pass, which loads Q anyway.
// k_dcgs_coef, one block, reduces both passes' partials (fixed trees) and
// forms the coefficients.  nv <= kMaxVec.
// ---------------------------------------------------------------------------
constexpr int kOutU = kMaxVec + 2;       // update-pass partials per block

template <int NC>
__global__ __launch_bounds__(kGsThreads) void k_gs_upd(const double* __restrict__ V, int64_t ldv, int nv,
                                                       double* __restrict__ u, const double* __restrict__ w,
                                                       double* __restrict__ wnext, int64_t n,
                                                       const double* __restrict__ coef,
                                                       double* __restrict__ partial,
                                                       const int32_t* __restrict__ stop) {
    constexpr int NV = 8 * NC;
    __shared__ double s_red[kGsThreads / PR_WAVE][kOutU];
    // coef: [0, 64) a, [64, 129) c (c[nv] multiplies v_j), [130] 1 / nu, [131] 1 / s
    double ca[NV], cw[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        ca[i] = (i < nv) ? coef[i] : 0.0;
        cw[i] = (i < nv) ? coef[64 + i] : 0.0;
    }
    const double cj = coef[64 + nv], inu = coef[130], is = coef[131];
    // the stop flag is read beside the coefficients, not ahead of them
    if (stopped(stop)) return;
    int64_t vo[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vo[i] = (int64_t)(i < nv ? i : (nv > 0 ? nv - 1 : 0)) * ldv;
    double acc[NV + 2];
#pragma unroll
    for (int i = 0; i < NV + 2; ++i) acc[i] = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    for (int64_t q = lo + threadIdx.x; q < hi; q += kGsThreads) {
        const double uq = u[q];
        const double wq = w[q];
        double v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = V[vo[i] + q];     // column 0 exists even for nv = 0
        __builtin_amdgcn_sched_barrier(0);
        double vj = uq * is, wn = wq * is;
#pragma unroll
        for (int i = 0; i < NV; ++i) {                // ca, cw = 0 past nv
            vj = fma(-ca[i], v[i], vj);
            wn = fma(-cw[i], v[i], wn);
        }
        vj *= inu;
        wn = (wn - cj * vj) * inu;
        u[q] = vj;
        wnext[q] = wn;
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = fma(v[i], wn, acc[i]);     // terms past nv are dropped
        acc[NV] = fma(vj, wn, acc[NV]);
        acc[NV + 1] = fma(wn, wn, acc[NV + 1]);
    }
    // outputs 0..nv-1 (Q . w_new), nv (v_j . w_new), nv + 1 (w_new . w_new)
    const int lane = threadIdx.x & (PR_WAVE - 1), wid = threadIdx.x / PR_WAVE;
#pragma unroll
    for (int i = 0; i < NV + 2; ++i) {
        const int k = i < NV ? i : nv + (i - NV);
        if (i >= NV || i < nv) {
            const double t = wave_sum(acc[i]);
            if (lane == 0) s_red[wid][k] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv + 2) {
        double t = 0.0;
        for (int w2 = 0; w2 < kGsThreads / PR_WAVE; ++w2) t += s_red[w2][threadIdx.x];
        partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;      // output-major
    }
}

// x of lane `src` (wave-uniform) in every lane: two v_readlane, no LDS
// round trip as a shuffle takes
__device__ __forceinline__ double lane_bcast(double x, int src) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Step j of the delayed scheme (j <= 31; j = m with `last` at the end of a
// cycle), one block of 1024 threads.  Partials: pd (dot pass of step j,
// stride kMaxVec: b'_0..b'_{j-1}, beta') and pu (update pass of step j - 1,
// stride kOutU: a'_0..a'_{j-1}, s^2), nblk blocks each; every output is
// summed by one wavefront in a fixed tree.  Then, with a = a' / s,
// b = b' / s, beta = beta' / s^2:
//   nu = sqrt(1 - |a|^2) (nu = 1, s = 1 at j = 0, where u = v_0);
//   column j-1 made final: H[0..j-1][j-1] += s a, H[j][j-1] = s nu, rotated by
//   the earlier Givens rotations, its own rotation formed, g updated and
//   the stopping test taken (as the single-projection step does);
//   unless the cycle stops or `last` is set: gv = H[0..j][0..j-1] a, the
//   provisional column j, h_Q = (b - gv_Q) / nu, h_j = ((beta - a.b) / nu -
//   gv_j) / nu, the update pass's coefficients (c = gv + nu h, 1 / nu, 1 / s)
//   and column j of T (T[i][j] = s a_i, T[j][j] = s nu: z_j = M u_raw), for
//   the flexible form's x += Z T^{-1} y.
// Hu: the unrotated Hessenberg matrix, row-major (m+1) x m; R: its rotated
// upper triangle.  gctl[1] = final columns of this cycle.
constexpr int kCoefThreads = 1024;
__global__ __launch_bounds__(kCoefThreads) void k_dcgs_coef(int j, int m, int last, const double* __restrict__ pd,
                                                            const double* __restrict__ pu, int nblk,
                                                            double* __restrict__ Hu, double* __restrict__ R,
                                                            double* __restrict__ cs, double* __restrict__ sn,
                                                            double* __restrict__ g, double* __restrict__ est,
                                                            double* __restrict__ T, double* __restrict__ coef,
                                                            int32_t* __restrict__ gctl,
                                                            const double* __restrict__ tolp,
                                                            const int64_t* __restrict__ itb, int64_t max_iters) {
    __shared__ double sa[64], sb[64], col[65], scs[64], ssn[64], s_ak[64];
    __shared__ double sH[33][32];             // band of H[0..j][0..j-1]
    __shared__ double s_part[64][65];         // lane sums per live output (padded rows)
    __shared__ double s_s, s_beta, s_g, s_tol;
    __shared__ int64_t s_itb;
    __shared__ int s_stop;
    const int t = threadIdx.x, lane = t & (PR_WAVE - 1), wv = t / PR_WAVE;
    constexpr int NW = kCoefThreads / PR_WAVE;
    const int c = j - 1;
    // every input, loaded by all threads in one round: the scalars, the
    // Hessenberg band, the rotations, then each wavefront's sums
    if (t == 0) s_stop = gctl[0];
    if (t == 1 && j > 0) s_g = g[c];
    if (t == 2) s_tol = *tolp;
    if (t == 3) s_itb = *itb;
    {
        const int i = t >> 5, k = t & 31;     // row i, column k of the band
        // zero outside the band, so the product with a below needs no test
        sH[i][k] = (i <= j && k < j && k + 1 >= i) ? Hu[(int64_t)i * m + k] : 0.0;
    }
    if (t < c) {
        scs[t] = cs[t];
        ssn[t] = sn[t];
    }
    const int nd = last ? 0 : j + 1;         // dot-pass outputs
    const int nu_out = j > 0 ? j + 1 : 0;     // update-pass outputs
    // block partials (output-major: a contiguous run of nblk, even, per
    // output).  Live output q < nd is dot output q, q >= nd update output
    // q - nd.  Wavefront w takes outputs w, w + NW, w + 2 NW, w + 3 NW; lane l
    // adds the 16-byte pairs l, l + 64, ... of each (every load in flight at
    // once), the lane sums go to LDS, and thread q adds its output's 64 lane
    // sums in lane order: a fixed tree.
    {
        static_assert(4 * (kCoefThreads / PR_WAVE) >= 64 && 4 * 2 * PR_WAVE >= 512,
                      "four outputs per wavefront and four pairs per lane cover 64 outputs of 512 blocks");
        const int L = nd + nu_out;
        const int npair = nblk / 2;
        double2 v[4][4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int q = wv + NW * qq;
            const double* P = q < nd ? pd + (int64_t)q * nblk : pu + (int64_t)(q - nd) * nblk;
            const double2* P2 = reinterpret_cast<const double2*>(q < L ? P : pd);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = lane + PR_WAVE * u;
                const bool ok = q < L && k < npair;
                const double2 x = P2[ok ? k : 0];
                v[qq][u].x = ok ? x.x : 0.0;
                v[qq][u].y = ok ? x.y : 0.0;
            }
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int q = wv + NW * qq;
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += v[qq][u].x + v[qq][u].y;
            if (q < L) s_part[q][lane] = acc;
        }
        __syncthreads();
        if (t < L) {
            double acc = 0.0;
            for (int l = 0; l < PR_WAVE; ++l) acc += s_part[t][l];
            if (t < nd) {
                if (t < j) sb[t] = acc; else s_beta = acc;
            } else {
                const int o = t - nd;
                if (o < j) sa[o] = acc; else s_s = acc;
            }
        }
    }
    __syncthreads();
    if (s_stop || wv != 0) return;
    // the rest by one wavefront, lane i holding row i (j <= 31).  Every
    // global store comes at the end: a store still reading its registers
    // would make the loops below wait for all memory operations.
    const int i = lane;
    double sc = 1.0, nu = 1.0;
    double ai = 0.0, bi = 0.0;
    double beta = last ? 0.0 : s_beta;        // beta' / s^2 (s = 1 at j = 0)
    bool stop = false;
    double hcol = 0.0, rcol = 0.0, cc = 1.0, ss = 0.0, gj = 0.0;
    if (j > 0) {
        sc = sqrt(fmax(s_s, 0.0));
        const double isc = sc > 0.0 ? 1.0 / sc : 0.0;
        ai = i < j ? sa[i] * isc : 0.0;
        const double s2 = wave_sum(ai * ai);
        nu = (s2 < 1.0 && sc > 0.0) ? sqrt(1.0 - s2) : 0.0;
        if (!last) {
            bi = i < j ? sb[i] * isc : 0.0;
            beta *= isc * isc;
        }
        // column j-1 final (Hu and the band), then rotated
        double cl = 0.0;
        if (i < j) cl = sH[i][c] + sc * ai;
        if (i == j) cl = sc * nu;
        hcol = cl;
        if (i <= j) {
            sH[i][c] = cl;
            col[i] = cl;
        }
        // the earlier rotations, in order, by one lane: rotation r maps the
        // pair (x_r, x_{r+1}) with x_r already rotated by rotation r - 1, so
        // only that carried value is a dependency; the column is read from
        // LDS ahead of it
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");    // one wavefront: LDS in order
        __builtin_amdgcn_wave_barrier();
        if (i == 0) {
            double carry = col[0];
#pragma unroll 4
            for (int r = 0; r < c; ++r) {
                const double x1 = col[r + 1], cr = scs[r], sr = ssn[r];
                col[r] = cr * carry + sr * x1;
                carry = -sr * carry + cr * x1;
            }
            col[c] = carry;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const double a0 = col[c], hn = lane_bcast(cl, j);
        const double den = hypot(a0, hn);
        cc = den > 0.0 ? a0 / den : 1.0;
        ss = den > 0.0 ? hn / den : 0.0;
        rcol = i < c ? col[i] : den;
        gj = -ss * s_g;
        stop = !(fabs(gj) > s_tol) || s_itb + j >= max_iters || j >= m || !(nu > 0.0);
    }
    // provisional column j and the update coefficients: lane i forms
    // gv_i = sum_k H[i][k] a_k over the Hessenberg band (H[i][k] = 0 for
    // i > k + 1, stored as zeros)
    double hq = 0.0, cq = 0.0;
    const double inu = 1.0 / nu;
    if (!stop && !last) {
        const double ab = wave_sum(ai * bi);
        double gvt = 0.0;
        // a from LDS (a loop with lane reads is not unrolled, its loads
        // would wait one by one)
        s_ak[i] = ai;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int ir = i <= j ? i : 0;        // rows past j: any row, result unused
#pragma unroll 4
        for (int k = 0; k < j; ++k) gvt += sH[ir][k] * s_ak[k];
        hq = i < j ? (bi - gvt) * inu : ((beta - ab) * inu - gvt) * inu;
        cq = gvt + nu * hq;
    }
    if (j > 0) {
        if (i <= j) Hu[(int64_t)i * m + c] = hcol;
        if (i <= c) R[(int64_t)i * m + c] = rcol;
        if (i == 0) {
            cs[c] = cc;
            sn[c] = ss;
            g[j] = gj;
            g[c] = cc * s_g;
            gctl[1] = j;
            gctl[2] = j;
            est[0] = fabs(gj);
            if (stop) gctl[0] = 1;
        }
    }
    if (stop || last) return;
    if (i < j) {
        Hu[(int64_t)i * m + j] = hq;
        coef[i] = ai;
        coef[64 + i] = cq;
        T[(int64_t)i * m + j] = sc * ai;
    } else if (i == j) {
        Hu[(int64_t)j * m + j] = hq;
        coef[64 + j] = cq;
        coef[130] = inu;
        coef[131] = 1.0 / sc;
        T[(int64_t)j * m + j] = sc * nu;
    }
}

// x = U^{-1} b for the leading mm x mm block of an upper triangular U
// (row-major, leading dimension m <= 64), one wavefront: U's triangle is
// staged in LDS in one round, lane l holds b_l, and column i is eliminated
// once x_i is known (x_i broadcast from lane i), so every step is one
// division and one fused multiply-add per lane.  b and x may alias.
__device__ __forceinline__ void tri_upper_solve(int m, int mm, const double* __restrict__ U, const double* b,
                                                double* x) {
    __shared__ double sU[64][65];
    const int l = threadIdx.x;
    for (int e = l; e < mm * mm; e += PR_WAVE) {
        const int i = e / mm, k = e % mm;
        if (k >= i) sU[i][k] = U[(int64_t)i * m + k];
    }
    double t = l < mm ? b[l] : 0.0;
    __syncthreads();
    for (int i = mm - 1; i >= 0; --i) {
        const double xi = lane_bcast(t / sU[i][i], i);
        if (l == i) t = xi;
        if (l < i) t = fma(-sU[l][i], xi, t);
    }
    if (l < mm) x[l] = t;
}

// y <- T^{-1} y over the final columns (T upper triangular, row-major m x m)
__global__ __launch_bounds__(PR_WAVE) void k_trisolve_T(int m, const double* __restrict__ T, double* y,
                                                        const int32_t* __restrict__ gctl) {
    tri_upper_solve(m, gctl[1], T, y, y);
}

// out[i] = sum over blocks of partial[i][b]; one block per output (a fixed
// tree).  (A last-block-reduces variant inside k_gs needs a device-scope
// release per block, an L2 write-back on this GPU; it measured twice as
// slow as this separate launch.)
__global__ __launch_bounds__(256) void k_gs_final(const double* __restrict__ partial, int nblk, int nreg,
                                                  double* __restrict__ out,
                                                  const int32_t* __restrict__ stop) {
    if (stopped(stop)) return;
    __shared__ double s_w[256 / PR_WAVE];
    const int i = blockIdx.x;
    double t = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) t += partial[(int64_t)i * nblk + b];
    t = wave_sum(t);
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) s_w[threadIdx.x / PR_WAVE] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = 0.0;
        for (int w2 = 0; w2 < 256 / PR_WAVE; ++w2) u += s_w[w2];
        out[i < nreg ? i : kMaxVec] = u;      // the extra norm output goes to out[32]
    }
}

// dst = src / sqrt(denom[0])   (denom holds a squared norm)
__global__ void k_scale(const double* __restrict__ src, double* __restrict__ dst,
                        const double* __restrict__ denom, int64_t n, const int32_t* __restrict__ stop) {
    if (stopped(stop)) return;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double d = sqrt(denom[0]);
    dst[q] = d > 0.0 ? src[q] / d : 0.0;
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = fma(a, x[q], y[q]);
}

// out = sum_{i < nv} c_i V_i with nv read from the device
__global__ void k_gemv_small(const double* __restrict__ V, int64_t ldv, const int32_t* __restrict__ nvp,
                             const double* __restrict__ c, int64_t n, double* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int nv = *nvp;
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc = fma(c[i], V[(int64_t)i * ldv + q], acc);
    out[q] = acc;
}

__global__ void k_zero(double* x, int64_t n, const int32_t* __restrict__ stop) {
    if (stopped(stop)) return;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) x[q] = 0.0;
}

// dst = src (graph-safe copy)
__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = src[q];
}

// Restart cycle start: g = (||r||, 0, ..., 0) from the squared norm in hd[0],
// stop flag and column count cleared (a kernel, so the cycle can be replayed
// from a graph)
__global__ void k_cycle_init(double* __restrict__ g, int m, const double* __restrict__ hd,
                             int32_t* __restrict__ gctl) {
    for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = (i == 0) ? sqrt(hd[0]) : 0.0;
    if (threadIdx.x == 0) {
        gctl[0] = 0;
        gctl[1] = 0;
        gctl[2] = 0;      // steps of this cycle that took the second projection
    }
}

// End of Arnoldi step j, one launch:
//   ||w||^2 from the last Gram-Schmidt pass's block partials (every block adds
//   them in the same fixed tree, so all blocks agree to the bit; in selective
//   mode a skipped third pass leaves the norm in sel[96]);
//   v_{j+1} = w / ||w|| over a grid-stride range;
//   block 0: column j of the Hessenberg matrix, h = h1 + h2 and
//   h_{j+1} = ||w||, the previous rotations applied, the new one formed, the
//   residual vector g updated; stop when |g_{j+1}| <= tol_abs (or not finite)
//   or the iteration limit is reached (tolp: device absolute tolerance; itb:
//   device count of the iterations of earlier cycles).  j < 64.
// gctl: [0] stop  [1] columns done this cycle  [2] steps with a third pass.
// The stop flag is read once per block; a block that starts after block 0 has
// set it skips its part of v_{j+1}, which a stopped cycle never reads.
constexpr int kEndUnroll = 4;
__global__ __launch_bounds__(kEndThreads) void k_step_end(
        const double* __restrict__ partial, int nblk, const double* sel, const double* __restrict__ w,
        double* __restrict__ vnext, int64_t n, int j, int m, double* hd, double* __restrict__ R,
        double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g, double* __restrict__ est,
        int32_t* __restrict__ gctl, const double* __restrict__ tolp, const int64_t* __restrict__ itb,
        int64_t max_iters) {
    __shared__ int s_stop;
    __shared__ double s_w[kEndThreads / PR_WAVE];
    __shared__ double col[65], c_s[64], s_s[64];
    const int t = threadIdx.x;
    const bool first = blockIdx.x == 0;
    // every load is issued before the first wait: the stop flag, the block
    // partials (read even when the selective test skipped the pass; their
    // sum is then not used), this thread's first rows of w and, in block 0,
    // the Hessenberg column and the previous rotations
    if (t == 0) s_stop = gctl[0];
    double a = 0.0;
    for (int b = t; b < nblk; b += kEndThreads) a += partial[b];
    const int64_t stride = (int64_t)gridDim.x * kEndThreads;
    const int64_t base0 = (int64_t)blockIdx.x * kEndThreads + t;
    double v[kEndUnroll];
#pragma unroll
    for (int u = 0; u < kEndUnroll; ++u) {
        const int64_t q = base0 + u * stride;
        v[u] = w[q < n ? q : n - 1];
    }
    // selective mode: the second projection's coefficients count only when
    // it ran
    const bool skip3 = sel && !reorth_needed(sel);
    const bool h2 = !skip3;
    if (first) {
        if (t <= j) col[t] = hd[t] + (h2 ? hd[64 + t] : 0.0);
        if (t < j) {
            c_s[t] = cs[t];
            s_s[t] = sn[t];
        }
    }
    a = wave_sum(a);
    if ((t & (PR_WAVE - 1)) == 0) s_w[t / PR_WAVE] = a;
    __syncthreads();
    if (s_stop) return;
    double nrm2;
    if (skip3) {
        nrm2 = sel[kSelProj];
    } else {
        double u = 0.0;
        for (int w2 = 0; w2 < kEndThreads / PR_WAVE; ++w2) u += s_w[w2];
        nrm2 = u;
    }
    if (first) {
        // Givens update of column j, ahead of this block's share of v_{j+1}
        if (t == 0) {
            hd[128] = nrm2;
            const int64_t iters_base = *itb;
            const double tol_abs = *tolp;
            const double hn = sqrt(fmax(nrm2, 0.0));
            for (int i = 0; i < j; ++i) {
                const double a0 = col[i], b0 = col[i + 1];
                col[i] = c_s[i] * a0 + s_s[i] * b0;
                col[i + 1] = -s_s[i] * a0 + c_s[i] * b0;
            }
            const double a0 = col[j];
            const double den = hypot(a0, hn);
            const double cj = den > 0.0 ? a0 / den : 1.0;
            const double sj = den > 0.0 ? hn / den : 0.0;
            cs[j] = cj;
            sn[j] = sj;
            col[j] = den;
            const double gj = g[j];
            g[j + 1] = -sj * gj;
            g[j] = cj * gj;
            gctl[1] = j + 1;
            if (h2) gctl[2] += 1;
            est[0] = fabs(g[j + 1]);
            if (!(fabs(g[j + 1]) > tol_abs) || iters_base + j + 1 >= max_iters || j + 1 >= m) gctl[0] = 1;
        }
        __syncthreads();
        if (t <= j) R[(int64_t)t * m + j] = col[t];
    }
    const double d = sqrt(nrm2);
#pragma unroll
    for (int u = 0; u < kEndUnroll; ++u) {
        const int64_t q = base0 + u * stride;
        if (q < n) vnext[q] = d > 0.0 ? v[u] / d : 0.0;
    }
    for (int64_t base = base0 + kEndUnroll * stride; base < n; base += kEndUnroll * stride) {
        double v2[kEndUnroll];
#pragma unroll
        for (int u = 0; u < kEndUnroll; ++u) {
            const int64_t q = base + u * stride;
            v2[u] = w[q < n ? q : n - 1];
        }
#pragma unroll
        for (int u = 0; u < kEndUnroll; ++u) {
            const int64_t q = base + u * stride;
            if (q < n) vnext[q] = d > 0.0 ? v2[u] / d : 0.0;
        }
    }
}

// y = R^{-1} g over the columns done (upper triangular back substitution)
__global__ __launch_bounds__(PR_WAVE) void k_trisolve(int m, const double* __restrict__ R,
                                                      const double* __restrict__ g, double* __restrict__ y,
                                                      const int32_t* __restrict__ gctl) {
    tri_upper_solve(m, gctl[1], R, g, y);
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_sell_plan(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t* slen, int32_t* sfmt,
                      int32_t* dtmp, unsigned long long* acc, hipStream_t s) {
    const int64_t ns = (n + 63) / 64;
    // per-slice entry counts of column-form slices in the tail of dtmp's space
    int32_t* cnnz = dtmp + ns * kMaxDiag;
    k_sell_plan<<<(unsigned)(ns + 1), kPlanThreads, 0, s>>>(rowptr, col, n, slen, sfmt, dtmp, cnnz);
    const unsigned tb = nb(ns, 256);
    k_sell_totals<<<tb < kTotalsBlocks ? tb : kTotalsBlocks, 256, 0, s>>>(slen, sfmt, cnnz, ns, acc);
}

void launch_sell_fill(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n, const int64_t* soff,
                      const int32_t* sfmt, const int32_t* dtmp, double* sval, int32_t* scol, int32_t* sdoff,
                      hipStream_t s) {
    const int64_t ns = (n + 63) / 64;
    k_sell_fill<<<nb(n, 256), 256, 0, s>>>(rowptr, col, val, n, soff, sfmt, sval, scol);
    k_sell_fill_diag<<<(unsigned)ns, kPlanThreads, 0, s>>>(rowptr, col, val, n, soff, sfmt, dtmp, sval, sdoff);
}

void launch_spmv_sell(const SellMat& M, int64_t n, const double* x, const double* b, double* y, hipStream_t s,
                      const int32_t* stop) {
    const int64_t ns = (n + 63) / 64;
    k_spmv_sell<<<nb(ns * 64, 256), 256, 0, s>>>(M, n, x, b, y, stop);
}

int gs_blocks(int64_t n) {
    int64_t b = (n + 1023) / 1024;        // several rows per thread: the loads of
    if (b > 512) b = 512;                 // consecutive rows overlap (measured best)
    if (b < 1) b = 1;
    return (int)(b + (b & 1));            // even: each output's run of block partials
                                          // is read in 16-byte pairs
}

// mode 0: out = V^T w ; mode 1: w -= V c, out = V^T w ; mode 2: w -= V c and
// the block partials of w.w in partial[0..gs_blocks(n)) (out unused).
// partial: gs_blocks(n) * 32 doubles.
void launch_gs(int mode, const double* V, int64_t ldv, int nv, double* w, int64_t n, const double* c,
               double* partial, double* out, hipStream_t s, const int32_t* stop, bool extra,
               const double* sel) {
    const int nbk = gs_blocks(n);
    // the extra norm output (at out[32]) needs one chunk with a free slot
    const int ex = (extra && mode != 2 && nv < kMaxVec) ? 1 : 0;
    for (int base = 0; base < nv || (nv == 0 && base == 0); base += kMaxVec) {
        const int cnt = nv - base < kMaxVec ? nv - base : kMaxVec;
        const double* Vb = V + (int64_t)base * ldv;
        const int nc = cnt <= 0 ? 1 : (cnt + 7) / 8;
#define PR_GS(M, CC)                                                                                 \
    k_gs<M, CC><<<nbk, kGsThreads, 0, s>>>(Vb, ldv, cnt, w, n, (M) == 0 ? c : c + base, partial, stop, ex, sel)
#define PR_GS_NC(M)                 \
    if (nc == 1) PR_GS(M, 1);       \
    else if (nc == 2) PR_GS(M, 2);  \
    else if (nc == 3) PR_GS(M, 3);  \
    else PR_GS(M, 4)
        if (mode == 0) {
            PR_GS_NC(0);
            k_gs_final<<<cnt + ex, 256, 0, s>>>(partial, nbk, cnt, out + base, stop);
        } else if (mode == 1) {
            PR_GS_NC(1);
            k_gs_final<<<cnt + ex, 256, 0, s>>>(partial, nbk, cnt, out + base, stop);
        } else {
            PR_GS_NC(2);       // partial[0..nbk): launch_step_end adds them
        }
#undef PR_GS_NC
#undef PR_GS
        if (nv == 0) break;
    }
}

void launch_gs_partials(const double* V, int64_t ldv, int nv, double* w, int64_t n, double* partial, hipStream_t s,
                        const int32_t* stop) {
    const int nbk = gs_blocks(n);
    const int nc = (nv + 7) / 8;
#define PR_GS0(CC) k_gs<0, CC><<<nbk, kGsThreads, 0, s>>>(V, ldv, nv, w, n, nullptr, partial, stop, 0, nullptr)
    if (nc <= 1) PR_GS0(1);
    else if (nc == 2) PR_GS0(2);
    else if (nc == 3) PR_GS0(3);
    else PR_GS0(4);
#undef PR_GS0
}

void launch_gs_upd(const double* V, int64_t ldv, int nv, double* u, const double* w, double* wnext, int64_t n,
                   const double* coef, double* partial, hipStream_t s, const int32_t* stop) {
    const int nbk = gs_blocks(n);
    const int nc = nv <= 8 ? 1 : (nv + 7) / 8;
#define PR_GSU(CC) k_gs_upd<CC><<<nbk, kGsThreads, 0, s>>>(V, ldv, nv, u, w, wnext, n, coef, partial, stop)
    if (nc == 1) PR_GSU(1);
    else if (nc == 2) PR_GSU(2);
    else if (nc == 3) PR_GSU(3);
    else PR_GSU(4);
#undef PR_GSU
}

void launch_dcgs_coef(int j, int m, bool last, const double* pd, const double* pu, int64_t n, double* Hu, double* R,
                      double* cs, double* sn, double* g, double* est, double* T, double* coef, int32_t* gctl,
                      const double* tolp, const int64_t* itb, int64_t max_iters, hipStream_t s) {
    k_dcgs_coef<<<1, kCoefThreads, 0, s>>>(j, m, last ? 1 : 0, pd, pu, gs_blocks(n), Hu, R, cs, sn, g, est, T, coef,
                                           gctl, tolp, itb, max_iters);
}

void launch_trisolve_T(int m, const double* T, double* y, const int32_t* gctl, hipStream_t s) {
    k_trisolve_T<<<1, 64, 0, s>>>(m, T, y, gctl);
}

void launch_scale(const double* src, double* dst, const double* denom, int64_t n, hipStream_t s,
                  const int32_t* stop) {
    if (n > 0) k_scale<<<nb(n, 256), 256, 0, s>>>(src, dst, denom, n, stop);
}

void launch_axpy_dev(double* y, const double* x, double a, int64_t n, hipStream_t s) {
    if (n > 0) k_axpy<<<nb(n, 256), 256, 0, s>>>(y, x, a, n);
}

void launch_gemv_small(const double* V, int64_t ldv, const int32_t* nvp, const double* coef, int64_t n,
                       double* out, hipStream_t s) {
    if (n > 0) k_gemv_small<<<nb(n, 256), 256, 0, s>>>(V, ldv, nvp, coef, n, out);
}

void launch_zero(double* x, int64_t n, hipStream_t s, const int32_t* stop) {
    if (n > 0) k_zero<<<nb(n, 256), 256, 0, s>>>(x, n, stop);
}

void launch_step_end(const double* partial, const double* sel, const double* w, double* vnext, int64_t n,
                     int j, int m, double* hd, double* R, double* cs, double* sn, double* g, double* est,
                     int32_t* gctl, const double* tolp, const int64_t* itb, int64_t max_iters, hipStream_t s) {
    const int64_t want = (n + kEndThreads - 1) / kEndThreads;
    const unsigned grid = (unsigned)(want < kEndBlocks ? (want > 0 ? want : 1) : kEndBlocks);
    k_step_end<<<grid, kEndThreads, 0, s>>>(partial, gs_blocks(n), sel, w, vnext, n, j, m, hd, R, cs, sn, g, est,
                                            gctl, tolp, itb, max_iters);
}

void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
    if (n > 0) k_copy<<<nb(n, 256), 256, 0, s>>>(dst, src, n);
}

void launch_cycle_init(double* g, int m, const double* hd, int32_t* gctl, hipStream_t s) {
    k_cycle_init<<<1, 64, 0, s>>>(g, m, hd, gctl);
}

void launch_trisolve(int m, const double* R, const double* g, double* y, const int32_t* gctl,
                     hipStream_t s) {
    k_trisolve<<<1, 64, 0, s>>>(m, R, g, y, gctl);
}
