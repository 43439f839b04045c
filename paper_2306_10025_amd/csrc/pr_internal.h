// Internal declarations shared by the translation units of libpatchrelax.so.
// gfx950 only: 64-lane wavefronts, FP64 hardware atomics, MFMA.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/patchrelax.h"

#define PR_WAVE 64
// largest patch (dofs) the library accepts; patches above 32 dofs take the
// block-per-patch kernels of k_wide.hip
constexpr int kWideMaxPs = 512;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T v, int width = PR_WAVE) {
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v, int width = PR_WAVE) {
    for (int o = width >> 1; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, width);
        v = u > v ? u : v;
    }
    return v;
}

// FP32 -> BF16 round-to-nearest-even (finite inputs), returned as raw bits.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
    _Float16 h = (_Float16)f;   // v_cvt_f16_f32: round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}

// Exponent e with m * 2^-e in [2^13, 2^14) for a float magnitude m > 0.
__device__ __forceinline__ int fp16_scale_exp(float m) {
    if (m == 0.0f) return 0;
    int E;
    frexpf(m, &E);              // m = f 2^E, f in [0.5, 1)
    return E - 14;
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------

// Hybrid sliced-ELL copy of A (k_krylov.hip): per 64-row slice either the
// diagonal form (sfmt 1: offsets sdoff[soff/64 + k], values) or the column
// form (sfmt 0: values and column indices scol), both column-major in the
// slice from sval[soff[slice]].
struct SellMat {
    const int64_t* soff = nullptr;
    const double* sval = nullptr;
    const int32_t* scol = nullptr;
    const int32_t* sdoff = nullptr;
    const int32_t* sfmt = nullptr;      // 0 column form, 1 diagonal form, 2 rows read from the CSR copy
    const int64_t* rowptr = nullptr;    // the CSR copy (form 2)
    const int32_t* col = nullptr;
    const double* val = nullptr;
};
constexpr int kSellMaxDiag = 192;   // distinct offsets a diagonal-form slice may hold
constexpr int kSellOffsetPad = 16;  // entries allocated past the last slice's offsets
constexpr int kCsrPad = 2;          // zero entries (column 0, value 0) past the CSR copy's last

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct pr_handle_s {
    pr_params prm;
    hipStream_t stream = nullptr;
    int device = 0;

    int64_t n = 0, nnz = 0, n_p = 0, total_dofs = 0, total_tile = 0;
    int max_ps = 0, min_ps = 0;
    bool uniform = true;

    // copies of the inputs
    int64_t* rowptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    int64_t* pptr = nullptr;
    int32_t* pdofs = nullptr;

    // sliced-ELL copy of A for the solve's SpMV (64-row slices)
    int64_t* soff = nullptr;
    double* sval = nullptr;
    int32_t* scol = nullptr;
    int32_t* sdoff = nullptr;
    int32_t* sfmt = nullptr;
    SellMat sell() const { return SellMat{soff, sval, scol, sdoff, sfmt, rowptr, col, val}; }

    // Section 2 objects
    int32_t* cnt = nullptr;
    double* W = nullptr;
    int64_t* toff = nullptr;      // tile offsets (int64[n_p+1]); null when uniform
    double* tiles = nullptr;
    uint32_t* keys = nullptr;     // boundary keys
    double* fnorm = nullptr;      // ||A_k||_F
    double* l1norm = nullptr;     // sum |A_k|

    // database
    int64_t m_p = 0;
    int32_t* phi = nullptr;
    int32_t* reps = nullptr;      // patch id of entry j (or -1)
    std::vector<int32_t> reps_host;
    double* db = nullptr;         // FP64 inverses of the entries
    double* db_mat = nullptr;     // entry matrices B_j (cluster means); null for patch reps
    int64_t* dboff = nullptr;     // int64[m_p+1] offsets in doubles (null when uniform)
    std::vector<int64_t> dboff_host;
    std::vector<int32_t> dbps_host;  // p of entry j

    // grouped apply
    int32_t* order = nullptr;     // patches grouped by entry, ascending id within
    int32_t* items = nullptr;     // int32[4*n_items]: entry, start, count, p
    int64_t n_items = 0;
    void* db_lp = nullptr;        // lane-ready low-precision database
    int64_t* dblp_off = nullptr;  // element offsets into db_lp per entry
    int32_t* db_exp = nullptr;    // FP16 scale exponents
    float* db_f32 = nullptr;      // FP32 database (row-major per entry; column-major when wide)
    bool wide = false;            // some patch has more than 32 dofs (k_wide.hip kernels)
    double* db_t = nullptr;       // wide FP64 apply: inverses column-major per entry
    int wide_form = 0;            // wide apply: 1 grouped matrix-core kernel, 2 one patch per block
    int apply_prec = PR_FP64;
    int32_t* gdofs = nullptr;     // dof lists in grouped order
    int64_t* goff = nullptr;      // grouped offsets (uneven sizes only)
    int32_t* gphi = nullptr;      // entry of each grouped position
    int64_t* dof_ptr = nullptr;   // dof -> grouped slots (deterministic scatter)
    int32_t* dof_slots = nullptr;
    int32_t* dof_ell = nullptr;   // padded dof -> slots table (ell_c per dof) or null
    int ell_c = 0;
    int tile_p = 0;               // > 0: MFMA apply over fixed tiles of patches with tile_p dofs
    void* Ybuf = nullptr;         // slot values of the deterministic scatter
    int tune_threads = 0;         // apply launch shape (autotuned or defaults)
    int64_t tune_cap = 0;
    int tune_slot = 0;
    int tune_tpw = 0;             // tiles per wave of the fixed-tile kernel (0: default)
    int tune_remap = 1;           // XCD-contiguous block order (fixed tiles, padded slot sum; default
                                  // on: same time as launch order, a quarter less HBM traffic)

    // solve workspace
    double* V = nullptr;
    double* Zb = nullptr;         // preconditioned basis of flexible GMRES (restart columns)
    int64_t zb_restart = -1;
    double* w = nullptr;
    double* t1 = nullptr;
    double* t2 = nullptr;
    double* red = nullptr;        // reduction partials
    double* gm = nullptr;         // device GMRES state: R, cs, sn, g, y, estimate
    int32_t* gctl = nullptr;      // device GMRES control: stop flag, columns done
    int64_t ldv = 0;              // leading dimension of the Krylov basis
    double* hd = nullptr;         // device scalars
    double* hh = nullptr;         // pinned host mirror
    size_t hh_got = 0;            // its cached block size
    int64_t ws_restart = -1;
    std::vector<hipEvent_t> evpool;   // reusable events for per-kernel timing
    // graph replay of a restart cycle: own capture stream, handle-owned b
    // and x, device tolerance and iteration base
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_m = -1;
    hipGraphExec_t bgexec = nullptr;   // one restart cycle of the batch solve
    int bgraph_m = -1;
    double* gb = nullptr;
    double* gx = nullptr;
    double* gtol = nullptr;
    int64_t* gitb = nullptr;

    // block-diagonal batch of independent systems (pr_set_systems)
    int nsys = 0;
    std::vector<int64_t> sys_ptr_host;
    int64_t nch = 0;
    int32_t* ch_sys = nullptr;
    int64_t* ch_lo = nullptr;
    int32_t* ch_len = nullptr;
    int32_t* sys_ch0 = nullptr;
    int32_t* sys_nch = nullptr;
    double* bpart = nullptr;      // per-chunk partials
    double* bscal = nullptr;      // per-system scalars: h1, h2, hn, norms (kBStride each)
    double* bgm = nullptr;        // per-system R, cs, sn, g, y, est
    int32_t* bctl = nullptr;      // per-system stop, columns, active; global stop
    int64_t* bbase = nullptr;     // per-system iterations of earlier cycles
    double* btol = nullptr;       // per-system absolute tolerance
    std::vector<int64_t> sys_iters;
    std::vector<double> sys_relres;

    // learned predictor (Algorithm 1 with predictions): training patches,
    // the other patches and their top-k candidate entries
    float* mlp_X = nullptr;       // raw features, float[n_p][mlp_F]
    int mlp_F = 0;
    int32_t* mlp_train = nullptr;
    int64_t mlp_ns = 0;
    int32_t* mlp_q = nullptr;
    int64_t mlp_nq = 0;
    int32_t* mlp_cand = nullptr;
    int mlp_k = 0;

    // two-level combination of Eq.(2) (pr_set_coarse): P0 (n x n0), R0 = P0^T,
    // A0 = R0 A P0 and its transpose (CSR), and the direct solver's data:
    // the dense inverse (c_dense) or the inverses of the block LU's Schur
    // complements (c_nb blocks of c_s rows); c_r0, c_w, c_x are padded vectors
    int64_t n0 = 0, a0_nnz = 0;
    int64_t *p0_rp = nullptr, *r0_rp = nullptr, *a0_rp = nullptr, *a0t_rp = nullptr;
    int32_t *p0_ci = nullptr, *r0_ci = nullptr, *a0_ci = nullptr, *a0t_ci = nullptr;
    double *p0_v = nullptr, *r0_v = nullptr, *a0_v = nullptr, *a0t_v = nullptr;
    int c_dense = 0, c_s = 0, c_nb = 0;
    int64_t c_np = 0;
    double* c_X = nullptr;
    double *c_G = nullptr, *c_H = nullptr;   // S_i^{-1} L_i and S_i^{-1} U_i (banded form)
    double *c_r0 = nullptr, *c_u = nullptr, *c_w = nullptr, *c_x = nullptr;

    // database of the previous system of a sequence (pr_setup_reuse)
    bool has_reuse = false;
    std::vector<int32_t> reuse_phi, reuse_reps;

    pr_solve_info sinfo{};
    pr_stats stats{};
    std::string last_error;
    std::vector<DevBuf> owned;
};

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------

void pr_set_global_error(const std::string& s);
int pr_fail(pr_handle h, int code, const std::string& msg);

#define PR_HIP(h, expr)                                                               \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess)                                                         \
            return pr_fail((h), _e == hipErrorOutOfMemory ? PR_ERR_OOM : PR_ERR_HIP,   \
                           std::string(#expr) + ": " + hipGetErrorString(_e));        \
    } while (0)

#define PR_TRY(expr)                 \
    do {                             \
        int _s = (expr);             \
        if (_s < 0) return _s;       \
    } while (0)

// per-device cache of idle device blocks (pr_pool.hip): *got receives the
// block's size, which pool_release takes back
hipError_t pool_alloc(int device, size_t bytes, void** p, size_t* got);
void pool_release(int device, void* p, size_t got);
hipError_t pool_host_alloc(size_t bytes, void** p, size_t* got);
void pool_host_release(void* p, size_t got);

// device allocation owned by the handle (returned to the cache by pr_destroy)
template <typename T>
int dalloc(pr_handle h, T** p, size_t count) {
    if (count == 0) count = 1;
    size_t got = 0;
    hipError_t e = pool_alloc(h->device, count * sizeof(T), (void**)p, &got);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return pr_fail(h, PR_ERR_OOM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                          " bytes failed: " + hipGetErrorString(e));
    }
    h->owned.push_back({(void*)*p, got});
    return PR_OK;
}

// returns an owned allocation to the cache before pr_destroy; every stream
// that used it must have been synchronised
template <typename T>
void dfree(pr_handle h, T* p) {
    for (size_t k = 0; k < h->owned.size(); ++k)
        if (h->owned[k].p == (void*)p) {
            pool_release(h->device, h->owned[k].p, h->owned[k].bytes);
            h->owned.erase(h->owned.begin() + (std::ptrdiff_t)k);
            return;
        }
}

// Algorithm 1 rounds after which the unresolved patches are inverted in one
// batch (2 + 4 + 8 rounds have run by then)
constexpr int64_t kA1BatchInvertAfter = 14;
// entries a component may open per round after the batched inversion, and
// the positions scanned for them
constexpr int kA1Spec = 16;
constexpr int kA1SpecWindow = 256;

inline int64_t next_pow2(int64_t n) {
    int64_t N = 1024;
    while (N < n) N <<= 1;
    return N;
}

// Algorithm 1 on a subset of the patches (pr_api.hip).  subset: device
// int32[ns] of patch ids in ascending order, or null for all patches.
struct A1Run {
    int64_t m = 0;                     // entries found
    int32_t* repof = nullptr;          // int32[n_p]: entry patch of each subset patch
    int32_t* slot_of_patch = nullptr;  // int32[n_p]: slot of an entry's inverse in dbt
    double* dbt = nullptr;             // FP64 inverses by slot
    int64_t* flag = nullptr;           // int64[ns+1] scratch
    int64_t* excl = nullptr;           // int64[ns+1] scratch
    int64_t* scr = nullptr;            // scan scratch
    unsigned long long cnt[4] = {0, 0, 0, 0};   // evaluations, exact singular values
    int rounds = 0;
};
int alg1_core(pr_handle h, const int32_t* subset, int64_t ns, A1Run& R);

// ---------------------------------------------------------------------------
// launchers (one translation unit each)
// ---------------------------------------------------------------------------

// k_setup.hip
void launch_validate_csr(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                         int32_t* flags, hipStream_t s);
void launch_validate_patches(const int64_t* ptr, const int32_t* dofs, int64_t n_p, int64_t n,
                             int64_t total, int32_t* flags, int32_t* minmax_ps, hipStream_t s);
void launch_cover(const int32_t* dofs, int64_t total, int32_t* cnt, hipStream_t s);
void launch_weights(const int32_t* cnt, int64_t n, double* W, int32_t* flags, hipStream_t s);
void launch_tile_offsets(const int64_t* ptr, int64_t n_p, int64_t* toff, int64_t* scratch,
                         hipStream_t s);
void launch_extract(const int64_t* rowptr, const int32_t* col, const double* val,
                    const int64_t* ptr, const int32_t* dofs, int64_t n_p, const int64_t* toff,
                    int uniform_ps, int max_ps, double* tiles, uint32_t* keys, double* fnorm, double* l1norm,
                    int32_t* flags, hipStream_t s);
void launch_iota(int32_t* a, int64_t n, hipStream_t s);
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t s);
// number of distinct keys: count[0] + count[1] after the launch; table is
// scratch of T >= 2n slots, T a power of two at most 2^32
void launch_count_distinct_u32(const uint32_t* keys, int64_t n, uint32_t* table, int64_t T, unsigned* count,
                               hipStream_t s);
// sort (key, value) pairs by key, ascending; keys/vals have length n (any n).
// scratch must hold next_pow2(n) keys and values.
void launch_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, uint64_t* kscr, int32_t* vscr,
                       hipStream_t s);
void launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* scratch,
                               hipStream_t s);
int64_t scan_scratch_elems(int64_t n);

// k_dense.hip
// Inverse of matrices m = sel ? sel[i] : i, i < count.  Matrix m has size
// pptr ? pptr[m+1]-pptr[m] : p (p is then the maximum size) and lives at
// A + (aoff ? aoff[m] : m*p*p); its inverse goes to X + (xoff ? xoff[m] : m*p*p).
void launch_batch_inverse(int p, int64_t count, const double* A, const int64_t* aoff,
                          const int32_t* sel, const int64_t* pptr, double* X,
                          const int64_t* xoff, int32_t* info, hipStream_t s);
void launch_batch_criterion(int p, int64_t count, int crit, const double* A, const double* B,
                            const double* X, double* d, hipStream_t s);

// k_alg1.hip: Algorithm 1 by independent components (see that file)
struct A1Dev {
    int64_t n_p, n_comp;
    const int64_t* ptr;
    const double* tiles;
    const int64_t* toff;      // null when uniform
    int uniform_ps;
    int32_t* ctl;             // int32[8]
    unsigned long long* counters;  // [0] evaluations [1] exact singular values
    const int32_t* cstart;    // int32[n_comp+1] first sorted position of each component
    int32_t* next;            // int32[n_comp] lowest unresolved position
    const int32_t* mem;       // patch at each sorted position (component, then id)
    const int32_t* pos_comp;  // component of each sorted position
    int32_t* status;          // int32[n_p] per sorted position
    int32_t* rep_slot;        // int32[n_comp] temporary slot of the current entry
    int32_t* rep_patch;       // int32[n_p] patch of each slot
    int32_t* slot_of_patch;   // int32[n_p]
    int32_t* repof;           // int32[n_p] entry patch of each patch
    int32_t* active;          // int32[n_comp]
    int32_t* cand;            // int32[n_p]
    int4* cinfo;              // per candidate {patch, component, slot, entry patch}
    double* dbt;              // inverses by slot, stride doubles each
    int64_t stride;
    double* inv;              // null, or inverses by sorted position after the batched inversion
    int32_t* inv_info;        // int32[n_p] zero-pivot report of each batched inverse
    // rounds of several entries (after the batched inversion), kA1Spec per component:
    int32_t* spec;            // int32[n_comp * kA1Spec] speculative members (positions)
    int32_t* spec_n;          // int32[n_comp]
    int32_t* pairm;           // int32[n_comp * kA1Spec] bit i of [c][j]: u_i matches u_j
    int32_t* ent;             // int32[n_comp * kA1Spec] the round's entries (positions)
    int32_t* ent_n;           // int32[n_comp]
    int32_t* ent_slot;        // int32[n_comp * kA1Spec]
};
void launch_a1_keys(int64_t n_p, const int32_t* subset, const int64_t* ptr, const double* keynorm,
                    uint64_t* keys, int32_t* vals, hipStream_t s);
// entries of a subset run in ascending patch id: entries[r] and
// rank_of_patch[entry] = base + r
void launch_a1_subset_entries(int64_t ns, const int32_t* subset, const int32_t* repof, int64_t* flags,
                              int64_t* rank, int64_t* scr, int32_t base, int32_t* entries,
                              int32_t* rank_of_patch, hipStream_t s);
void launch_a1_comp_flags(int64_t n_p, const int32_t* sidx, const int64_t* ptr, const double* keynorm,
                          int crit, double eps, int prune, int64_t* flag, hipStream_t s);
void launch_a1_key2(int64_t n_p, const int64_t* flag, const int64_t* excl, const int32_t* sidx,
                    uint64_t* key2, int32_t* val2, hipStream_t s);
void launch_a1_cstart(int64_t n_p, int64_t n_comp, const uint64_t* key2, int32_t* pos_comp,
                      int32_t* cstart, int32_t* next, hipStream_t s);
void launch_a1_rounds(int rounds, const A1Dev& d, int crit, double eps, int max_ps, hipStream_t s);
// inverts every unresolved patch into d.inv (by sorted position); the
// multi-entry rounds then copy from there instead of inverting
void launch_a1_preinvert(const A1Dev& d, int max_ps, hipStream_t s);
// rounds of up to kA1Spec entries per component; needs d.inv and the
// speculation arrays
void launch_a1_spec_rounds(int rounds, const A1Dev& d, int crit, double eps, int max_ps, hipStream_t s);
void launch_a1_finish(int64_t n_p, const int32_t* repof, int64_t* flags, int64_t* rank, int64_t* scr,
                      int32_t* phi, int32_t* reps, hipStream_t s);
void launch_a1_closest(int64_t n_p, const int64_t* ptr, const double* tiles, const int64_t* toff, int ups,
                       const int32_t* reps, int64_t m_p, const int64_t* rank, const double* keynorm,
                       double* ekey, int32_t* esz, const double* db, int64_t stride, int crit, double eps,
                       double tie, int32_t* phi, double* lbscr, int64_t grid, unsigned long long* counters,
                       hipStream_t s);
void launch_a1_copy_db(int64_t m_p, const int32_t* reps, const int32_t* slot_of_patch, const int64_t* ptr,
                       const double* dbt, double* db, int64_t stride, hipStream_t s);

// k_kmeans.hip: Algorithm 2 and its variants (see that file)
int64_t km_assign_grid(int64_t n_p, int64_t lbld);
void launch_km_assign(int64_t grid, int64_t n_p, const int64_t* ptr, const double* tiles, const int64_t* toff,
                      int uniform_ps, const int32_t* pg, const int32_t* gc0, const int32_t* gc1,
                      const int32_t* gactive, int crit, const double* l1n, const double* cen, int64_t stride,
                      double tie, int32_t* phi, int32_t* gchanged, double* lbscr, int64_t lbld,
                      unsigned long long* counters, hipStream_t s);
void launch_km_update(int64_t m_p, const int32_t* cgroup, const int32_t* gupd, const int64_t* cptr,
                      const int32_t* mem, const int32_t* cps, int medoid, const double* tiles,
                      const int64_t* toff, int uniform_ps, double* B, int64_t stride, int32_t* rep_patch,
                      double tie, unsigned long long* counters, hipStream_t s);
void launch_km_init(int64_t m_p, const int32_t* rep, const int64_t* ptr, const double* tiles,
                    const int64_t* toff, int uniform_ps, double* B, int64_t stride, hipStream_t s);
void launch_km_keys(int64_t n_p, const int32_t* phi, const int32_t* pg, const int32_t* gupd, uint64_t* keys,
                    int32_t* vals, unsigned long long* ccount, hipStream_t s);
void launch_km_key1(int64_t n_p, const int64_t* ptr, const uint32_t* bkeys, int partition, uint64_t* keys,
                    int32_t* vals, hipStream_t s);
void launch_km_flags(int64_t n, const uint64_t* keys, int64_t* flag, hipStream_t s);
void launch_km_gid(int64_t n, const uint64_t* keys, const int32_t* vals, const int64_t* flag,
                   const int64_t* excl, int32_t* pg, int64_t* gstart, int32_t* gp, hipStream_t s);
void launch_km_key2(int64_t n_p, const int32_t* pg, uint64_t* keys, int32_t* vals, hipStream_t s);
void launch_gather_i32(int64_t n, const int32_t* src, const int64_t* idx, int32_t* out, hipStream_t s);

// k_mlp.hip: learned entry predictor (see that file)
void launch_mlp_features(int64_t n_p, const int64_t* ptr, const double* tiles, const int64_t* toff, int ups,
                         const uint32_t* bkeys, int pmax, float* out, hipStream_t s);
void launch_mlp_moments(int64_t nrows, const int32_t* rows, const float* X, int F, float* mu, float* sd,
                        hipStream_t s);
void launch_mlp_gather(int64_t nrows, const int32_t* rows, const float* X, int F, const float* mu,
                       const float* sd, float* Xn, const int32_t* lab_src, int32_t* lab, const int32_t* key_src,
                       int32_t* key, hipStream_t s);
void launch_gemm(int prec, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B,
                 int ldb, float* C, int ldc, float alpha, const float* bias, int relu, const float* mask,
                 int ldm, hipStream_t s);
void launch_softmax_ce(int B, int C, const float* L, int ldl, const int32_t* y, const int32_t* rkey,
                       const int32_t* ckey, float* G, int ldg, double* loss_rows, float scale, hipStream_t s);
void launch_colsum(int B, int N, const float* G, int ldg, float scale, float* out, hipStream_t s);
void launch_adam(int64_t n, float* P, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, hipStream_t s);
void launch_init_uniform(int64_t n, float* W, float a, uint64_t seed, uint64_t base, hipStream_t s);
void launch_topk(int64_t R, int C, const float* L, int ldl, int k, const int32_t* rkey, const int32_t* ckey,
                 int32_t* out, hipStream_t s);
void launch_mlp_match(int mode, int64_t nq, const int32_t* qids, const int32_t* cand, int k,
                      const int64_t* ptr, const double* tiles, const int64_t* toff, int ups,
                      const int32_t* entries, int64_t n0, const double* X0, int64_t stride, int crit, double eps,
                      const double* keynorm, int32_t* repof, int32_t* resolved, unsigned long long* counters,
                      hipStream_t s);
void launch_compact_flags(int64_t n, const int32_t* keep, int want, int64_t* f, hipStream_t s);
void launch_compact(int64_t n, const int32_t* ids, const int64_t* f, const int64_t* pos, int32_t* out,
                    hipStream_t s);
void launch_copy_at(int64_t n, const int32_t* ids, const int32_t* src, int32_t* dst, hipStream_t s);
void launch_map_at(int64_t n, const int32_t* ids, const int32_t* src, const int32_t* map, int32_t* out,
                   hipStream_t s);
void launch_sizes(int64_t n, const int32_t* ids, const int64_t* ptr, int32_t* out, hipStream_t s);
void launch_count_eq(int64_t n, const int32_t* a, int sa, const int32_t* b, unsigned long long* cnt,
                     hipStream_t s);
void launch_rows_gather(int64_t n, const int32_t* idx, const float* src, int F, float* dst, const int32_t* lsrc,
                        int32_t* ldst, const int32_t* ksrc, int32_t* kdst, hipStream_t s);
void launch_set_at(int64_t n, const int32_t* ids, int32_t v, int32_t* dst, hipStream_t s);

// k_coarse.hip: two-level combination (Eq.(2))
void launch_interp_check(int64_t n, int64_t n0, int64_t nnz, const int64_t* rp, const int32_t* ci,
                         const double* v, int32_t* flags, hipStream_t st);
int launch_csr_transpose(int64_t n, int64_t m, const int64_t* rp, const int32_t* ci, const double* v,
                         int64_t* tp, int32_t* tc, double* tv, int64_t* cnt, int64_t* fill, int32_t* uc,
                         double* uv, int64_t* scan_scr, hipStream_t st);
int coarse_gal_slots();
void launch_galerkin(int64_t n0, const int64_t* rrp, const int32_t* rci, const double* rv, const int64_t* arp,
                     const int32_t* aci, const double* av, const int64_t* prp, const int32_t* pci,
                     const double* pv, double drop, int32_t* ocnt, int32_t* ocol, double* oval,
                     int32_t* overflow, hipStream_t st);
int coarse_ap_slots();
void launch_ap(int64_t n, const int64_t* arp, const int32_t* aci, const double* av, const int64_t* prp,
               const int32_t* pci, const double* pv, int32_t* bcnt, int32_t* bcol, double* bval,
               int32_t* overflow, hipStream_t st);
void launch_rb(int64_t n0, const int64_t* rrp, const int32_t* rci, const double* rv, const int32_t* bcnt,
               const int32_t* bcol, const double* bval, double drop, int32_t* ocnt, int32_t* ocol, double* oval,
               int32_t* overflow, hipStream_t st);
void launch_rows_finish(int64_t n0, const int32_t* cnt32, int64_t* cnt64, int64_t* rp, int64_t* scan_scr,
                        hipStream_t st);
void launch_rows_compact(int64_t n0, const int64_t* rp, const int32_t* icol, const double* ival, int32_t* ocol,
                         double* oval, hipStream_t st);
void launch_bandwidth(int64_t n0, const int64_t* rp, const int32_t* ci, int32_t* bw, hipStream_t st);
void launch_dense_from_csr(int64_t n0, int64_t np, const int64_t* rp, const int32_t* ci, const double* v,
                           double* M, hipStream_t st);
void launch_gj_inverse(double* M, int s, double* Pinv, double* C, int32_t* info, hipStream_t st);
void launch_csr_rows_wave(int64_t m, const int64_t* rp, const int32_t* ci, const double* v, const double* x,
                          double* y, const int32_t* stop, hipStream_t st);
void launch_csr_rows_add(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, const double* x,
                         double* z, const int32_t* stop, hipStream_t st);
void launch_dense_gemv(int64_t np, const double* X, const double* in, double* out, const int32_t* stop,
                       hipStream_t st);
void launch_block_schur_h(int64_t n0, int s, int bi, const int64_t* rp, const int32_t* ci, const double* v,
                          const double* Hprev, double* S, hipStream_t st);
void launch_block_coupling(int64_t n0, int s, int bi, int bj, const int64_t* trp, const int32_t* tci,
                           const double* tv, const double* Sinv, double* out, hipStream_t st);
void launch_band_solve(int s, int nb, const double* Sinv, const double* G, const double* H, const double* r0,
                        double* u, double* w, double* x, const int32_t* stop, hipStream_t st);
// pr_coarse.hip: z += P0 A0^{-1} R0 r (no-op without a coarse space)
int coarse_add(pr_handle h, const double* r, double* z, const int32_t* stop);

// pr_mlp.hip: Algorithm 1 with the learned predictor, and Algorithm 1 seeded
// with the previous system's database
int run_alg1_mlp(pr_handle h);
int run_alg1_reuse(pr_handle h);
// pr_wide.hip: Algorithm 1 for handles with a patch above 32 dofs
int run_alg1_wide(pr_handle h);

// k_apply.hip
struct ApplyLaunch {
    int64_t n, n_p;
    // grouped geometry
    const int32_t* gdofs;
    const int64_t* goff;   // null when every patch has pst dofs
    int pst;
    const int32_t* gphi;
    int maxp;
    // database
    const double* db;          // FP64 row-major
    const float* db_f32;       // FP32 row-major
    const int64_t* dboff;      // null: entry j at j * dbst
    int64_t dbst;
    const uint16_t* db_lp;     // lane-ready MFMA operands
    const int64_t* dblp_off;
    const int32_t* db_exp;
    const int32_t* items;
    int64_t n_items;
    int tile_p = 0;            // > 0: every patch has tile_p dofs (fixed MFMA tiles, no items)
    // vectors
    const double* W;
    double omega;
    const double* r;
    double* z;
    // deterministic scatter
    void* Y;
    const int64_t* dof_ptr;
    const int32_t* dof_slots;
    const int32_t* ell = nullptr;  // padded dof -> slots table (ell_c per dof), or null
    int ell_c = 0;
    const int32_t* stop;       // optional device flag: skip the work when set
    // launch shape (0: defaults): threads per block of the patch kernel
    // (64, 128 or 256), block cap, threads per block of the slot sum
    int threads = 0;
    int64_t grid_cap = 0;
    int slot_threads = 0;
    int tiles_per_wave = 0;    // fixed-tile MFMA kernel: 1 or 2 (0: default)
    int xcd_remap = 0;         // fixed-tile kernel and padded slot sum: XCD-contiguous block order
    int wide = 0;              // patches above 32 dofs: 1 grouped matrix-core items, 2 one patch per block
    const double* db_t = nullptr;  // wide FP64: inverses column-major (db_f32 is column-major too)
};
// z (+)= omega M~^{-1} r.  Atomic mode accumulates into z (caller zeroes it);
// two-stage mode overwrites z.
void launch_apply(int prec, bool two_stage, const ApplyLaunch& a, hipStream_t s);
void launch_convert_db(int prec, int64_t m_p, const double* db, const int64_t* dboff,
                       const int32_t* dbps, int uniform_ps, uint16_t* db_lp,
                       const int64_t* dblp_off, int32_t* db_exp, float* db_f32, hipStream_t s);
// grouped dof lists and the dof -> slot transpose
void launch_group_gather(const int32_t* order, int64_t n_p, const int64_t* ptr, const int32_t* dofs,
                         const int64_t* goff, int pst, int32_t* gdofs, int32_t* gphi,
                         const int32_t* phi, hipStream_t s);
void launch_group_sizes(const int32_t* order, int64_t n_p, const int64_t* ptr, int64_t* sizes,
                        hipStream_t s);
void launch_transpose_fill(const int32_t* gdofs, const int64_t* goff, int pst, int64_t n_p, int pmax,
                           const int64_t* dof_ptr, int32_t* fill, int32_t* dof_slots, hipStream_t s);
void launch_transpose_sort(int64_t n, const int64_t* dof_ptr, int32_t* dof_slots, hipStream_t s);
void launch_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s);
// *out = max(*out, max_i a[i]) (caller initialises *out)
void launch_max_i32(const int32_t* a, int64_t n, int32_t* out, hipStream_t s);
// ell[i*C + u] = u-th slot of dof i, -1 past its count (C >= every count)
// grouping on the device: keys = phi << 32 | id with order = iota (bad[0] = 1
// for a phi outside [0, m)); estart[gphi[s]] = s at each new entry of the
// sorted gphi (entries without patches keep what was there)
void launch_group_keys(const int32_t* phi, int64_t n_p, int64_t m, uint64_t* keys, int32_t* order, int32_t* bad,
                       hipStream_t s);
void launch_entry_starts(const int32_t* gphi, int64_t n_p, int64_t m, int32_t* estart, hipStream_t s);
// sizes[j] = size of patch reps[j]
void launch_rep_sizes(const int32_t* reps, const int64_t* ptr, int64_t m, int32_t* sizes, hipStream_t s);
// *out += sum_i before[phi[i]] + (reps[phi[i]] != i)
void launch_naive_pairs(const int32_t* phi, const int32_t* reps, const int32_t* before, int64_t n_p, int64_t m,
                        unsigned long long* out, hipStream_t s);
void launch_build_ell(int64_t n, const int64_t* dof_ptr, const int32_t* dof_slots, int C, int32_t* ell,
                      hipStream_t s);

// k_krylov.hip  (kernels with a `stop` argument return at once when *stop != 0)
void launch_scale(const double* src, double* dst, const double* denom, int64_t n, hipStream_t s,
                  const int32_t* stop = nullptr);
void launch_axpy_dev(double* y, const double* x, double a, int64_t n, hipStream_t s);
void launch_gemv_small(const double* V, int64_t ldv, const int32_t* nvp, const double* coef, int64_t n,
                       double* out, hipStream_t s);
void launch_zero(double* x, int64_t n, hipStream_t s, const int32_t* stop = nullptr);
int gs_blocks(int64_t n);
// Plan of the hybrid copy: slen[ns + 1] (stored columns * 64 per slice, 0
// at ns, for the exclusive scan), sfmt[ns], dtmp[ns * (kSellMaxDiag + 1)]
// (the offsets of diagonal-form slices, then one entry count per slice),
// acc[5] += {diagonal slices, their offsets, entries of column-form slices,
// CSR-row slices, their entries}
// (acc zeroed by the caller).
void launch_sell_plan(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t* slen, int32_t* sfmt,
                      int32_t* dtmp, unsigned long long* acc, hipStream_t s);
// Fill after the scan of slen into soff: sval for every slice, scol for the
// column form, sdoff for the diagonal form.
void launch_sell_fill(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n, const int64_t* soff,
                      const int32_t* sfmt, const int32_t* dtmp, double* sval, int32_t* scol, int32_t* sdoff,
                      hipStream_t s);
// y = A x (b null) or y = b - A x
void launch_spmv_sell(const SellMat& M, int64_t n, const double* x, const double* b, double* y, hipStream_t s,
                      const int32_t* stop = nullptr);
// Gram-Schmidt passes.  extra (modes 0 and 1, nv < 32): also out[32] = w . w
// (mode 1: of the updated w).  Mode 2 leaves the block partials of w . w in
// partial for launch_step_end (out unused); sel (mode 2): the pass runs only
// when the selective-reorthogonalisation test on sel[32], sel[96] asks for it.
void launch_gs(int mode, const double* V, int64_t ldv, int nv, double* w, int64_t n, const double* c,
               double* partial, double* out, hipStream_t s, const int32_t* stop = nullptr,
               bool extra = false, const double* sel = nullptr);
// End of Arnoldi step j after a mode-2 pass: hd[128] = ||w||^2 (from the
// pass's partials, or sel[96] when the selective test skipped it), vnext =
// w / ||w||, and the Givens update of column j with the stopping test.  sel
// (selective mode, = hd or null): the column is hd[0..j] plus hd[64..64+j]
// only when the third pass ran.
void launch_step_end(const double* partial, const double* sel, const double* w, double* vnext, int64_t n,
                     int j, int m, double* hd, double* R, double* cs, double* sn, double* g, double* est,
                     int32_t* gctl, const double* tolp, const int64_t* itb, int64_t max_iters, hipStream_t s);
// Gram-Schmidt with delayed reorthogonalisation (nv <= 32): the dot pass's
// block partials (stride 32, V_i . w for i < nv), the update pass (v_j over
// u, the unnormalised next vector to wnext, partials of its dots, stride
// 34), and the one-block coefficient step between them
void launch_gs_partials(const double* V, int64_t ldv, int nv, double* w, int64_t n, double* partial, hipStream_t s,
                        const int32_t* stop);
void launch_gs_upd(const double* V, int64_t ldv, int nv, double* u, const double* w, double* wnext, int64_t n,
                   const double* coef, double* partial, hipStream_t s, const int32_t* stop);
void launch_dcgs_coef(int j, int m, bool last, const double* pd, const double* pu, int64_t n, double* Hu, double* R,
                      double* cs, double* sn, double* g, double* est, double* T, double* coef, int32_t* gctl,
                      const double* tolp, const int64_t* itb, int64_t max_iters, hipStream_t s);
void launch_trisolve_T(int m, const double* T, double* y, const int32_t* gctl, hipStream_t s);
void launch_trisolve(int m, const double* R, const double* g, double* y, const int32_t* gctl,
                     hipStream_t s);
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
void launch_cycle_init(double* g, int m, const double* hd, int32_t* gctl, hipStream_t s);

// k_batch.hip: GMRES over independent systems (one Krylov space per system)
struct BGeom {
    int64_t nch;               // row chunks (each inside one system)
    const int32_t* ch_sys;     // system of each chunk
    const int64_t* ch_lo;      // first row of each chunk
    const int32_t* ch_len;     // rows of each chunk
    int nsys;
    const int32_t* sys_ch0;    // first chunk of each system
    const int32_t* sys_nch;    // chunks of each system
};
constexpr int kBStride = 64;   // per-system coefficient slots
void launch_bgs(int mode, const double* V, int64_t ldv, int nv, double* w, const BGeom& g, const double* c,
                double* partial, double* out, const int32_t* sstop, const int32_t* gstop, hipStream_t s);
void launch_bscale(const double* src, double* dst, const BGeom& g, const double* denom, const int32_t* sstop,
                   const int32_t* gstop, hipStream_t s);
void launch_bgivens(int j, int m, int nsys, const double* h1, const double* h2, const double* hn, double* R,
                    double* cs, double* sn, double* gv, double* est, int32_t* sstop, int32_t* scols,
                    const double* tol_abs, const int64_t* sbase, int64_t max_iters, int32_t* gstop,
                    hipStream_t s);
void launch_btrisolve(int m, int nsys, const double* R, const double* gv, double* y, const int32_t* scols,
                      hipStream_t s);
void launch_bgemv(const double* V, int64_t ldv, const BGeom& g, const double* y, int m, const int32_t* scols,
                  double* out, hipStream_t s);
void launch_bcycle_init(int nsys, int m, const double* nrm2, const int32_t* active, double* gv, int32_t* sstop,
                        int32_t* scols, int32_t* gstop, hipStream_t s);

// k_wide.hip: patches with 33..kWideMaxPs dofs (a block of 256 threads per patch)
// range and duplicate checks of the patches above 32 dofs (flags[2], flags[3]
// as launch_validate_patches)
void launch_validate_wide(const int64_t* ptr, const int32_t* dofs, int64_t n_p, int64_t n, int32_t* flags,
                          hipStream_t s);
// tiles, boundary keys (XOR fold of the single-nonzero row mask), norms, as launch_extract
void launch_extract_wide(const int64_t* rowptr, const int32_t* col, const double* val, const int64_t* ptr,
                         const int32_t* dofs, int64_t n_p, const int64_t* toff, int uniform_ps, double* tiles,
                         uint32_t* keys, double* fnorm, double* l1norm, int32_t* flags, hipStream_t s);
// X_i = inverse of tile list[i] (list null: tile i), at X + xoff[i] (null:
// i * p * p); info[i] = 1 + the step of a zero pivot, else 0.  ptr null: a
// dense batch of uniform_ps x uniform_ps matrices.  pmax >= every p.
void launch_gj_wide(int64_t count, const int32_t* list, const int64_t* ptr, const double* tiles,
                    const int64_t* toff, int uniform_ps, int pmax, double* X, const int64_t* xoff, int32_t* info,
                    hipStream_t s);
// One round of Algorithm 1: the entry m opened by U[0] is compared with
// U[1..nu]; keep[u] = 1 for U[1+u] still open (keep[nu] = 0), phi set for
// the matched and for U[0].  counters: evaluations, pruned, refined, ties.
// Xm: inverse of the entry (spectral), scratch: grid * 2 * pmax^2 doubles.
void launch_a1w_round(int64_t nu, const int32_t* U, int32_t m, int crit, double eps, const int64_t* ptr,
                      const double* tiles, const int64_t* toff, int uniform_ps, const double* fnorm,
                      const double* l1norm, const double* Xm, double* scratch, int64_t grid, int pmax,
                      int32_t* phi, int64_t* keep, unsigned long long* counters, hipStream_t s);
int64_t a1w_spectral_grid(int64_t nu);
// out[i] = U[i] for keep[i] (positions from the exclusive scan excl)
void launch_a1w_compact(int64_t nu, const int32_t* U, const int64_t* keep, const int64_t* excl, int32_t* out,
                        hipStream_t s);
// the patch part of the apply for wide handles (a.wide: 1 grouped items, 2
// one patch per block; FP64 reads a.db_t, FP32 a.db_f32, both column-major)
void launch_apply_wide(int prec, bool two_stage, const ApplyLaunch& a, hipStream_t s);
// column-major copies of the database entries (FP64 and/or FP32)
void launch_transpose_db(int64_t m_p, const double* db, const int64_t* dboff, const int32_t* dbps,
                         double* out64, float* out32, hipStream_t s);

// pr_batch.hip: the solve over independent systems
int solve_batch(pr_handle h, const double* b, double* x, double tol);
// pr_api.hip: preconditioner (sweeps damped steps from 0) and the Krylov
// workspace, shared with the batched solve
int pr_precond_internal(pr_handle h, const double* v, double* e, double* t3, const int32_t* stop);
int pr_workspace_internal(pr_handle h, int m);
