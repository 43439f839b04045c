// Setup kernels: validation, cover counts and W (Section 2), dense patch
// extraction A_k = V_k A V_k^T with the boundary key of Section 3.2, and the
// generic device primitives (exclusive scan, bitonic key/value sort) used to
// order patches.
#include "pr_internal.h"

#include <climits>

namespace {

constexpr int kMaxPs = 32;

// flags layout (int32[8], initialised by the host):
//  [0] bad CSR (0/1)      [1] bad patch ptr (0/1)   [2] min patch with dof out of range
//  [3] min patch with dup [4] min uncovered dof     [5] min patch with non-finite tile
//  [6] patch too large    [7] unused

__global__ void k_validate_csr(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               int64_t n, int64_t nnz, int32_t* flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rowptr[0] != 0 || rowptr[n] != nnz)) flags[0] = 1;
    if (i >= n) return;
    int64_t s = rowptr[i], e = rowptr[i + 1];
    if (s > e || s < 0 || e > nnz) {
        flags[0] = 1;
        return;
    }
    // columns in groups of 8, loaded before they are checked (clamped
    // addresses inside the row, so no load waits behind a branch)
    int32_t prev = -1;
    bool bad = false;
    for (int64_t q0 = s; q0 < e && !bad; q0 += 8) {
        int32_t cc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) cc[u] = col[q0 + u < e ? q0 + u : s];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (q0 + u < e) {
                const int32_t c = cc[u];
                if (c < 0 || c >= n || c <= prev) bad = true;
                prev = c;
            }
        }
    }
    if (bad) flags[0] = 1;
}

// Grid-stride over the patches; a patch's dofs are loaded together (clamped
// addresses), checked against [0, n) and pairwise for duplicates; the
// smallest and largest patch size go out with one atomic per block.
constexpr int kValidateBlocks = 1024;
__global__ __launch_bounds__(256) void k_validate_patches(const int64_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ dofs, int64_t n_p,
                                                          int64_t n, int64_t total, int32_t* flags,
                                                          int32_t* minmax) {
    __shared__ int32_t s_mn[256 / PR_WAVE], s_mx[256 / PR_WAVE];
    const int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k0 == 0 && (ptr[0] != 0 || ptr[n_p] != total)) flags[1] = 1;
    int32_t mn = INT_MAX, mx = 0;
    for (int64_t k = k0; k < n_p; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = ptr[k], e = ptr[k + 1];
        if (s < 0 || e <= s || e > total) {
            flags[1] = 1;
            continue;
        }
        const int64_t p = e - s;
        const int32_t pc = (int32_t)(p > INT_MAX ? INT_MAX : p);
        mn = pc < mn ? pc : mn;
        mx = pc > mx ? pc : mx;
        if (p > kMaxPs) {
            flags[6] = 1;
            continue;
        }
        int32_t loc[kMaxPs];
#pragma unroll
        for (int a = 0; a < kMaxPs; ++a) loc[a] = dofs[s + (a < p ? a : 0)];
        bool bad = false, dup = false;
#pragma unroll
        for (int a = 0; a < kMaxPs; ++a)
            if (a < p && (loc[a] < 0 || loc[a] >= n)) bad = true;
        if (bad) {
            atomicMin(&flags[2], (int32_t)k);
            continue;
        }
#pragma unroll
        for (int a = 0; a < kMaxPs; ++a)
#pragma unroll
            for (int b = a + 1; b < kMaxPs; ++b)
                if (b < p && loc[a] == loc[b]) dup = true;
        if (dup) atomicMin(&flags[3], (int32_t)k);
    }
    for (int o = PR_WAVE >> 1; o > 0; o >>= 1) {
        const int32_t a = __shfl_xor(mn, o), b = __shfl_xor(mx, o);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) {
        s_mn[threadIdx.x / PR_WAVE] = mn;
        s_mx[threadIdx.x / PR_WAVE] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / PR_WAVE; ++w) {
            mn = s_mn[w] < mn ? s_mn[w] : mn;
            mx = s_mx[w] > mx ? s_mx[w] : mx;
        }
        if (mn != INT_MAX) atomicMin(&minmax[0], mn);
        atomicMax(&minmax[1], mx);
    }
}

__global__ void k_cover(const int32_t* __restrict__ dofs, int64_t total, int32_t* cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) atomicAdd(&cnt[dofs[i]], 1);
}

__global__ void k_weights(const int32_t* __restrict__ cnt, int64_t n, double* W, int32_t* flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = cnt[i];
    if (c == 0) {
        atomicMin(&flags[4], (int32_t)i);
        W[i] = 0.0;
    } else {
        W[i] = 1.0 / (double)c;   // W = (sum_l V_l^T V_l)^{-1}, Section 2
    }
}

__global__ void k_square_sizes(const int64_t* __restrict__ ptr, int64_t n_p, int64_t* out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_p) {
        int64_t p = ptr[k + 1] - ptr[k];
        out[k] = p * p;
    }
}

// One wavefront (one block of 64 threads) per patch, grid-stride.
// A_k[a][b] = A[g_a][g_b]: the wave walks the CSR rows of the patch's dofs as
// one flattened, coalesced sequence of nonzeros; each nonzero's column is
// looked up among the patch dofs (sorted in LDS) by binary search.  The tile
// buffer is dynamic LDS of max_ps^2 doubles, so small patches leave room
// for more resident blocks.
__global__ __launch_bounds__(64) void k_extract(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int64_t* __restrict__ ptr,
    const int32_t* __restrict__ dofs, int64_t n_p, const int64_t* __restrict__ toff,
    int uniform_ps, double* __restrict__ tiles, uint32_t* __restrict__ keys,
    double* __restrict__ fnorm, double* __restrict__ l1norm, int32_t* flags) {
    extern __shared__ double s_tile[];
    __shared__ int32_t s_sorted[kMaxPs];
    __shared__ int32_t s_loc[kMaxPs];
    __shared__ int64_t s_rs[kMaxPs];
    __shared__ int32_t s_off[kMaxPs + 1];
    const int lane = threadIdx.x;

    for (int64_t k = blockIdx.x; k < n_p; k += gridDim.x) {
        const int64_t s0 = ptr[k];
        const int p = (int)(ptr[k + 1] - s0);
        const int64_t t0 = uniform_ps ? k * (int64_t)uniform_ps * uniform_ps : toff[k];

        int32_t g = lane < p ? dofs[s0 + lane] : INT_MAX;
        int64_t rs = 0, re = 0;
        if (lane < p) {
            rs = rowptr[g];
            re = rowptr[g + 1];
        }
        // rank of my dof among the patch dofs (distinct) -> sorted order
        int rank = 0;
        for (int b = 0; b < p; ++b) {
            int32_t gb = __shfl(g, b);
            rank += (gb < g) ? 1 : 0;
        }
        if (lane < p) {
            s_sorted[rank] = g;
            s_loc[rank] = lane;
            s_rs[lane] = rs;
        }
        // exclusive prefix of row lengths over the p lanes
        int len = lane < p ? (int)(re - rs) : 0;
        int incl = len;
        for (int o = 1; o < PR_WAVE; o <<= 1) {
            int u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane < p) s_off[lane] = incl - len;
        const int T = __shfl(incl, p - 1);
        for (int e = lane; e < p * p; e += PR_WAVE) s_tile[e] = 0.0;
        __syncthreads();

        for (int e = lane; e < T; e += PR_WAVE) {
            // row a: last a with s_off[a] <= e
            int lo = 0, hi = p - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
            }
            const int a = lo;
            const int64_t q = s_rs[a] + (e - s_off[a]);
            const int32_t c = col[q];
            const double v = val[q];
            int l2 = 0, h2 = p - 1;
            while (l2 < h2) {
                int mid = (l2 + h2) >> 1;
                if (s_sorted[mid] < c) l2 = mid + 1; else h2 = mid;
            }
            if (s_sorted[l2] == c) s_tile[a * p + s_loc[l2]] = v;
        }
        __syncthreads();

        double sq = 0.0, ab = 0.0;
        bool finite = true;
        for (int e = lane; e < p * p; e += PR_WAVE) {
            const double v = s_tile[e];
            tiles[t0 + e] = v;
            sq += v * v;
            ab += fabs(v);
            finite = finite && isfinite(v);
        }
        int nz = 0;
        if (lane < p)
            for (int b = 0; b < p; ++b) nz += (s_tile[lane * p + b] != 0.0) ? 1 : 0;
        const unsigned long long bal = __ballot(lane < p && nz == 1);
        sq = wave_sum(sq);
        ab = wave_sum(ab);
        const bool allfin = __all(finite);
        if (lane == 0) {
            keys[k] = (uint32_t)bal;
            fnorm[k] = sqrt(sq);
            l1norm[k] = ab;
            if (!allfin) atomicMin(&flags[5], (int32_t)k);
        }
        __syncthreads();
    }
}

__global__ void k_iota(int32_t* a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (int32_t)i;
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// ---- exclusive scan (int64) ------------------------------------------------

constexpr int kScanThreads = 512;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int64_t* __restrict__ in,
                                                            int64_t* __restrict__ out, int64_t n,
                                                            int64_t* __restrict__ block_sums) {
    __shared__ int64_t s_warp[kScanThreads / PR_WAVE];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t tsum = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        v[t] = (base + t < n) ? in[base + t] : 0;
        tsum += v[t];
    }
    const int lane = threadIdx.x & (PR_WAVE - 1), wid = threadIdx.x / PR_WAVE;
    int64_t incl = tsum;
    for (int o = 1; o < PR_WAVE; o <<= 1) {
        int64_t u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == PR_WAVE - 1) s_warp[wid] = incl;
    __syncthreads();
    int64_t woff = 0;
    for (int w = 0; w < wid; ++w) woff += s_warp[w];
    int64_t run = woff + incl - tsum;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        if (base + t < n) out[base + t] = run;
        run += v[t];
    }
    if (threadIdx.x == kScanThreads - 1) block_sums[blockIdx.x] = woff + incl;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ offs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += offs[i / kScanTile];
}

// ---- bitonic sort of (uint64 key, int32 value) pairs -----------------------

constexpr int kSortThreads = 512;
constexpr int kSortLocal = 2 * kSortThreads;  // elements sorted inside one block

__device__ __forceinline__ void cswap(uint64_t& ka, int32_t& va, uint64_t& kb, int32_t& vb, bool up) {
    const bool gt = (ka > kb) || (ka == kb && va > vb);
    if (gt == up) {
        uint64_t tk = ka; ka = kb; kb = tk;
        int32_t tv = va; va = vb; vb = tv;
    }
}

// Sort-in-LDS phases: for every stage k <= kmax, or (when kfix > 0) only the
// j < kSortLocal steps of stage kfix.
__global__ __launch_bounds__(kSortThreads) void k_bitonic_local(uint64_t* keys, int32_t* vals,
                                                                int64_t N, int64_t kfix) {
    __shared__ uint64_t sk[kSortLocal];
    __shared__ int32_t sv[kSortLocal];
    const int64_t base = (int64_t)blockIdx.x * kSortLocal;
    for (int t = threadIdx.x; t < kSortLocal; t += kSortThreads) {
        sk[t] = keys[base + t];
        sv[t] = vals[base + t];
    }
    __syncthreads();
    const int64_t kbeg = kfix > 0 ? kfix : 2;
    const int64_t kend = kfix > 0 ? kfix : (int64_t)kSortLocal;
    for (int64_t k = kbeg; k <= kend; k <<= 1) {
        for (int64_t j = (kfix > 0 ? kSortLocal / 2 : k / 2); j > 0; j >>= 1) {
            const int t = threadIdx.x;
            const int i = (int)(2 * j * (t / j) + (t % j));
            const int l = i + (int)j;
            const bool up = ((base + i) & k) == 0;
            cswap(sk[i], sv[i], sk[l], sv[l], up);
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < kSortLocal; t += kSortThreads) {
        keys[base + t] = sk[t];
        vals[base + t] = sv[t];
    }
}

__global__ void k_bitonic_global(uint64_t* keys, int32_t* vals, int64_t N, int64_t k, int64_t j) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N / 2) return;
    const int64_t i = 2 * j * (t / j) + (t % j);
    const int64_t l = i + j;
    const bool up = (i & k) == 0;
    uint64_t ka = keys[i], kb = keys[l];
    int32_t va = vals[i], vb = vals[l];
    cswap(ka, va, kb, vb, up);
    keys[i] = ka; keys[l] = kb;
    vals[i] = va; vals[l] = vb;
}

__global__ void k_pad_copy(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                           int64_t n, uint64_t* kout, int32_t* vout, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    kout[i] = i < n ? kin[i] : ~0ull;
    vout[i] = i < n ? vin[i] : INT_MAX;
}

__global__ void k_unpad_copy(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                             int64_t n, uint64_t* kout, int32_t* vout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        kout[i] = kin[i];
        vout[i] = vin[i];
    }
}

// ---- grouped order ------------------------------------------------------------

__global__ void k_group_sizes(const int32_t* __restrict__ order, int64_t n_p,
                              const int64_t* __restrict__ ptr, int64_t* __restrict__ sizes) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_p) {
        const int32_t k = order[s];
        sizes[s] = ptr[k + 1] - ptr[k];
    } else if (s == n_p) {
        sizes[s] = 0;
    }
}

__global__ void k_group_gather(const int32_t* __restrict__ order, int64_t n_p,
                               const int64_t* __restrict__ ptr, const int32_t* __restrict__ dofs,
                               const int64_t* __restrict__ goff, int pst, int32_t* __restrict__ gdofs,
                               int32_t* __restrict__ gphi, const int32_t* __restrict__ phi) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_p) return;
    const int32_t k = order[s];
    const int64_t a0 = ptr[k], a1 = ptr[k + 1];
    const int64_t o = goff ? goff[s] : s * (int64_t)pst;
    for (int64_t q = a0; q < a1; ++q) gdofs[o + (q - a0)] = dofs[q];
    gphi[s] = phi[k];
}

// slot of local row a of grouped patch s: tiles of 16 patches, row-planes
// inside a tile, ((s / 16) * pmax + a) * 16 + s % 16 (the apply's layout)
__global__ void k_transpose_fill(const int32_t* __restrict__ gdofs, const int64_t* __restrict__ goff, int pst,
                                 int64_t n_p, int pmax, const int64_t* __restrict__ dof_ptr,
                                 int32_t* __restrict__ fill, int32_t* __restrict__ dof_slots) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_p * pmax) return;
    const int64_t s = t / pmax;
    const int a = (int)(t % pmax);
    const int64_t o = goff ? goff[s] : s * pst;
    const int p = goff ? (int)(goff[s + 1] - o) : pst;
    if (a >= p) return;
    const int32_t g = gdofs[o + a];
    const int32_t pos = atomicAdd(&fill[g], 1);
    dof_slots[dof_ptr[g] + pos] = (int32_t)((((s >> 4) * pmax + a) << 4) + (s & 15));
}

// each dof's slot list in ascending slot order (fixed summation order)
__global__ void k_transpose_sort(int64_t n, const int64_t* __restrict__ dof_ptr,
                                 int32_t* __restrict__ dof_slots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = dof_ptr[i], b = dof_ptr[i + 1];
    for (int64_t x = a + 1; x < b; ++x) {
        const int32_t v = dof_slots[x];
        int64_t y = x - 1;
        while (y >= a && dof_slots[y] > v) {
            dof_slots[y + 1] = dof_slots[y];
            --y;
        }
        dof_slots[y + 1] = v;
    }
}

// largest count: a grid-stride maximum per block, one atomic per block (one
// per wavefront on a single address serialised at about 11 ns each)
constexpr int kMaxBlocks = 512;
__global__ __launch_bounds__(256) void k_max_i32(const int32_t* __restrict__ a, int64_t n,
                                                 int32_t* __restrict__ out) {
    __shared__ int32_t s_m[256 / PR_WAVE];
    int32_t v = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v = a[i] > v ? a[i] : v;
    v = wave_max(v);
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) s_m[threadIdx.x / PR_WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = s_m[0];
        for (int w = 1; w < 256 / PR_WAVE; ++w) m = s_m[w] > m ? s_m[w] : m;
        atomicMax(out, m);
    }
}

// padded copy of the dof -> slot lists: C entries per dof, -1 after the last
__global__ void k_build_ell(int64_t n, const int64_t* __restrict__ dof_ptr,
                            const int32_t* __restrict__ dof_slots, int C, int32_t* __restrict__ ell) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = dof_ptr[i], c = dof_ptr[i + 1] - a;
    for (int u = 0; u < C; ++u) ell[i * C + u] = u < c ? dof_slots[a + u] : -1;
}

__global__ void k_i32_to_i64(const int32_t* __restrict__ in, int64_t* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
    else if (i == n) out[i] = 0;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_validate_csr(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                         int32_t* flags, hipStream_t s) {
    k_validate_csr<<<nblk(n > 0 ? n : 1, 256), 256, 0, s>>>(rowptr, col, n, nnz, flags);
}

void launch_validate_patches(const int64_t* ptr, const int32_t* dofs, int64_t n_p, int64_t n,
                             int64_t total, int32_t* flags, int32_t* minmax_ps, hipStream_t s) {
    const unsigned b = nblk(n_p > 0 ? n_p : 1, 256);
    k_validate_patches<<<b < kValidateBlocks ? b : kValidateBlocks, 256, 0, s>>>(ptr, dofs, n_p, n, total, flags,
                                                                                minmax_ps);
}

void launch_cover(const int32_t* dofs, int64_t total, int32_t* cnt, hipStream_t s) {
    if (total > 0) k_cover<<<nblk(total, 256), 256, 0, s>>>(dofs, total, cnt);
}

void launch_weights(const int32_t* cnt, int64_t n, double* W, int32_t* flags, hipStream_t s) {
    k_weights<<<nblk(n, 256), 256, 0, s>>>(cnt, n, W, flags);
}

int64_t scan_scratch_elems(int64_t n) {
    int64_t tot = 0;
    while (n > 1) {
        n = (n + kScanTile - 1) / kScanTile;
        tot += 2 * n + 1;
    }
    return tot + 2;
}

void launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch,
                               hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    int64_t* sums = scratch;
    k_scan_tile<<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, sums);
    if (nb == 1) return;
    int64_t* offs = scratch + nb;
    launch_exclusive_scan_i64(sums, offs, nb, scratch + 2 * nb + 1, s);
    k_scan_add<<<nblk(n, 256), 256, 0, s>>>(out, n, offs);
}

void launch_tile_offsets(const int64_t* ptr, int64_t n_p, int64_t* toff, int64_t* scratch,
                         hipStream_t s) {
    // toff[k] = sum_{l<k} p_l^2 ; toff has n_p+1 entries (sizes written to toff+... via scratch)
    int64_t* sq = scratch;
    k_square_sizes<<<nblk(n_p + 1, 256), 256, 0, s>>>(ptr, n_p, sq);
    hipMemsetAsync(sq + n_p, 0, sizeof(int64_t), s);
    launch_exclusive_scan_i64(sq, toff, n_p + 1, scratch + n_p + 1, s);
}

void launch_extract(const int64_t* rowptr, const int32_t* col, const double* val,
                    const int64_t* ptr, const int32_t* dofs, int64_t n_p, const int64_t* toff,
                    int uniform_ps, int max_ps, double* tiles, uint32_t* keys, double* fnorm, double* l1norm,
                    int32_t* flags, hipStream_t s) {
    if (n_p <= 0) return;
    const int64_t grid = n_p < 65536 * 4 ? n_p : 65536 * 4;
    const int pm = max_ps > 0 && max_ps <= kMaxPs ? max_ps : kMaxPs;
    k_extract<<<(unsigned)grid, 64, (size_t)pm * pm * sizeof(double), s>>>(
        rowptr, col, val, ptr, dofs, n_p, toff, uniform_ps, tiles, keys, fnorm, l1norm, flags);
}

void launch_iota(int32_t* a, int64_t n, hipStream_t s) {
    if (n > 0) k_iota<<<nblk(n, 256), 256, 0, s>>>(a, n);
}

// ---- distinct boundary keys (an open-addressing set) ------------------------
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

__global__ void k_set_clear(uint32_t* table, int64_t T, unsigned* count) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < T) table[i] = 0xFFFFFFFFu;
    if (i < 2) count[i] = 0u;
}

// count[0]: keys other than 0xFFFFFFFF inserted first; count[1]: 1 if that
// key occurs.  Patches with one boundary key come in long runs, so each
// wavefront walks its chunks of 64 keys reducing each to one lane per
// distinct value (one pass per distinct value), skips the value it inserted
// last, and reads the slot before it tries the atomic (a key already present
// costs a load, not a serialised atomic).  The table has at least 2n slots,
// so every probe sequence meets a free slot; the loop bound is the table size.
__global__ void k_set_insert(const uint32_t* keys, int64_t n, uint32_t* table, uint32_t mask, unsigned* count) {
    const int lane = threadIdx.x & (PR_WAVE - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / PR_WAVE);
    const int64_t wv = (int64_t)blockIdx.x * (blockDim.x / PR_WAVE) + threadIdx.x / PR_WAVE;
    uint32_t last = 0xFFFFFFFFu;
    for (int64_t c0 = wv * PR_WAVE; c0 < n; c0 += waves * PR_WAVE) {
        const int64_t i = c0 + lane;
        const uint32_t k = keys[i < n ? i : n - 1];
        bool pending = i < n;
        if (pending && k == 0xFFFFFFFFu) {
            atomicOr(&count[1], 1u);
            pending = false;
        }
        for (;;) {
            const uint64_t m = __ballot(pending);
            if (m == 0) break;
            const int leader = __ffsll((unsigned long long)m) - 1;
            const uint32_t kl = __shfl(k, leader);
            if (pending && k == kl) pending = false;
            if (kl == last) continue;
            last = kl;
            if (lane == leader) {
                uint32_t slot = mix32(kl) & mask;
                for (uint32_t probe = 0; probe <= mask; ++probe) {
                    const uint32_t seen = table[slot];
                    if (seen == kl) break;
                    if (seen == 0xFFFFFFFFu) {
                        const uint32_t prev = atomicCAS(&table[slot], 0xFFFFFFFFu, kl);
                        if (prev == 0xFFFFFFFFu) {
                            atomicAdd(&count[0], 1u);
                            break;
                        }
                        if (prev == kl) break;
                    }
                    slot = (slot + 1) & mask;
                }
            }
        }
    }
}

void launch_count_distinct_u32(const uint32_t* keys, int64_t n, uint32_t* table, int64_t T, unsigned* count,
                               hipStream_t s) {
    k_set_clear<<<nblk(T, 256), 256, 0, s>>>(table, T, count);
    if (n > 0) {
        const unsigned b = nblk(n, 256 * 8);        // about 8 chunks of 64 keys per wavefront
        k_set_insert<<<b < 1 ? 1 : b, 256, 0, s>>>(keys, n, table, (uint32_t)(T - 1), count);
    }
}

void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t s) {
    if (n > 0) k_fill_i32<<<nblk(n, 256), 256, 0, s>>>(a, n, v);
}

void launch_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, uint64_t* kscr, int32_t* vscr,
                       hipStream_t s) {
    if (n <= 1) return;
    int64_t N = kSortLocal;
    while (N < n) N <<= 1;
    k_pad_copy<<<nblk(N, 256), 256, 0, s>>>(keys, vals, n, kscr, vscr, N);
    const unsigned lblocks = (unsigned)(N / kSortLocal);
    k_bitonic_local<<<lblocks, kSortThreads, 0, s>>>(kscr, vscr, N, 0);
    for (int64_t k = 2 * kSortLocal; k <= N; k <<= 1) {
        for (int64_t j = k / 2; j >= kSortLocal; j >>= 1)
            k_bitonic_global<<<nblk(N / 2, 256), 256, 0, s>>>(kscr, vscr, N, k, j);
        k_bitonic_local<<<lblocks, kSortThreads, 0, s>>>(kscr, vscr, N, k);
    }
    k_unpad_copy<<<nblk(n, 256), 256, 0, s>>>(kscr, vscr, n, keys, vals);
}

void launch_group_sizes(const int32_t* order, int64_t n_p, const int64_t* ptr, int64_t* sizes,
                        hipStream_t s) {
    k_group_sizes<<<nblk(n_p + 1, 256), 256, 0, s>>>(order, n_p, ptr, sizes);
}

// ---- grouping and Algorithm 1 statistics on the device -----------------------
namespace {

// keys[k] = phi[k] << 32 | k and order[k] = k; bad[0] = 1 if some phi[k] lies
// outside [0, m)
__global__ void k_group_keys(const int32_t* __restrict__ phi, int64_t n_p, int64_t m, uint64_t* __restrict__ keys,
                             int32_t* __restrict__ order, int32_t* __restrict__ bad) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_p) return;
    const int32_t j = phi[k];
    if (j < 0 || j >= m) bad[0] = 1;
    keys[k] = ((uint64_t)(uint32_t)j << 32) | (uint32_t)k;
    order[k] = (int32_t)k;
}

// estart[j] = first grouped position of entry j (gphi ascending); entries
// without patches keep the -1 the caller filled in
__global__ void k_entry_starts(const int32_t* __restrict__ gphi, int64_t n_p, int64_t m, int32_t* __restrict__ estart) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_p) return;
    const int32_t j = gphi[s];
    if (j < 0 || j >= m) return;        // reported through k_group_keys' flag
    if (s == 0 || gphi[s - 1] != j) estart[j] = (int32_t)s;
}

// sizes[j] = size of patch reps[j]
__global__ void k_rep_sizes(const int32_t* __restrict__ reps, const int64_t* __restrict__ ptr, int64_t m,
                            int32_t* __restrict__ sizes) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) sizes[j] = (int32_t)(ptr[reps[j] + 1] - ptr[reps[j]]);
}

// out += sum over patches i of before[phi[i]] + (reps[phi[i]] != i): the
// comparisons the sequential Algorithm 1 makes (grid-stride, one atomic per
// block)
__global__ __launch_bounds__(256) void k_naive_pairs(const int32_t* __restrict__ phi, const int32_t* __restrict__ reps,
                                                     const int32_t* __restrict__ before, int64_t n_p, int64_t m,
                                                     unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s_a[256 / PR_WAVE];
    unsigned long long a = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_p; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = phi[i];
        if (j < 0 || j >= m) continue;      // the grouping step reports a map out of range
        a += (unsigned long long)before[j] + (reps[j] == (int32_t)i ? 0ull : 1ull);
    }
    a = wave_sum(a);
    if ((threadIdx.x & (PR_WAVE - 1)) == 0) s_a[threadIdx.x / PR_WAVE] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long u = 0;
        for (int w = 0; w < 256 / PR_WAVE; ++w) u += s_a[w];
        atomicAdd(out, u);
    }
}

}  // namespace

void launch_group_keys(const int32_t* phi, int64_t n_p, int64_t m, uint64_t* keys, int32_t* order, int32_t* bad,
                       hipStream_t s) {
    if (n_p > 0) k_group_keys<<<nblk(n_p, 256), 256, 0, s>>>(phi, n_p, m, keys, order, bad);
}

void launch_entry_starts(const int32_t* gphi, int64_t n_p, int64_t m, int32_t* estart, hipStream_t s) {
    if (n_p > 0) k_entry_starts<<<nblk(n_p, 256), 256, 0, s>>>(gphi, n_p, m, estart);
}

void launch_rep_sizes(const int32_t* reps, const int64_t* ptr, int64_t m, int32_t* sizes, hipStream_t s) {
    if (m > 0) k_rep_sizes<<<nblk(m, 256), 256, 0, s>>>(reps, ptr, m, sizes);
}

void launch_naive_pairs(const int32_t* phi, const int32_t* reps, const int32_t* before, int64_t n_p, int64_t m,
                        unsigned long long* out, hipStream_t s) {
    if (n_p <= 0) return;
    const unsigned b = nblk(n_p, 256);
    k_naive_pairs<<<b < 512 ? b : 512, 256, 0, s>>>(phi, reps, before, n_p, m, out);
}

void launch_group_gather(const int32_t* order, int64_t n_p, const int64_t* ptr, const int32_t* dofs,
                         const int64_t* goff, int pst, int32_t* gdofs, int32_t* gphi,
                         const int32_t* phi, hipStream_t s) {
    if (n_p > 0)
        k_group_gather<<<nblk(n_p, 256), 256, 0, s>>>(order, n_p, ptr, dofs, goff, pst, gdofs, gphi, phi);
}

void launch_transpose_fill(const int32_t* gdofs, const int64_t* goff, int pst, int64_t n_p, int pmax,
                           const int64_t* dof_ptr, int32_t* fill, int32_t* dof_slots, hipStream_t s) {
    const int64_t total = n_p * pmax;
    if (total > 0)
        k_transpose_fill<<<nblk(total, 256), 256, 0, s>>>(gdofs, goff, pst, n_p, pmax, dof_ptr, fill, dof_slots);
}

void launch_transpose_sort(int64_t n, const int64_t* dof_ptr, int32_t* dof_slots, hipStream_t s) {
    if (n > 0) k_transpose_sort<<<nblk(n, 256), 256, 0, s>>>(n, dof_ptr, dof_slots);
}

void launch_max_i32(const int32_t* a, int64_t n, int32_t* out, hipStream_t s) {
    if (n > 0) {
        const unsigned b = nblk(n, 256);
        k_max_i32<<<b < kMaxBlocks ? b : kMaxBlocks, 256, 0, s>>>(a, n, out);
    }
}

void launch_build_ell(int64_t n, const int64_t* dof_ptr, const int32_t* dof_slots, int C, int32_t* ell,
                      hipStream_t s) {
    if (n > 0) k_build_ell<<<nblk(n, 256), 256, 0, s>>>(n, dof_ptr, dof_slots, C, ell);
}

void launch_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
    k_i32_to_i64<<<nblk(n + 1, 256), 256, 0, s>>>(in, out, n);
}
