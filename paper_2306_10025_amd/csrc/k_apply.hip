// The patch preconditioner apply, Eq.(3) (Eq.(1) when every patch is its own
// database entry): z = omega * W * sum_k V_k^T X_phi(k) V_k r.
//
// Two families of kernels:
//  * vector kernels (FP64 or FP32 arithmetic): a group of G lanes per patch,
//    lane a owns local dof a and reads row a of the inverse (row-major, so a
//    group streams the whole matrix contiguously); the restricted residual
//    is broadcast through cross-lane shuffles;
//  * grouped MFMA kernels (BF16 or FP16 operands, FP32 accumulation): the
//    patches that share database entry j are stacked, so the apply becomes
//    Y = X_j [r_k1 ... r_kN], one MFMA tile per 16 or 32 members (the
//    multiple right-hand-side solve the paper's Experiment 3 discussion
//    proposes).  The lane that gathers local dof i of a member also holds
//    output row i of that member, so gather and scatter share indices.
// Patches are visited in grouped order (by database entry, then patch id)
// through a grouped copy of the dof lists.  The scatter either adds into z
// with FP64 atomics, or (deterministic mode) writes each patch row to a slot
// buffer Y that a second kernel sums per dof in a fixed order.
#include "pr_internal.h"

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

struct ApplyGeom {
    const int32_t* gdofs;   // dof lists in grouped order
    const int64_t* goff;    // grouped offsets (null: position s starts at s * pst)
    int pst;
    const int32_t* gphi;    // database entry of grouped position s
    const int64_t* dboff;   // database offsets (null: entry j at j * dbst)
    int64_t dbst;
    const int32_t* stop;    // optional device flag: return at once when set
    int ypm;                // slot buffer tiles: 16 patches x ypm local rows (see yslot)
    int remap;              // XCD-aware block order (block_id)
};

// Slot of local row a of grouped patch s: patches in tiles of 16, inside a
// tile row-plane by row-plane (16 consecutive patches' row a contiguous).
// A block or an MFMA item writes whole tiles, and the per-dof sum finds the
// rows of neighbouring patches next to each other.
__device__ __forceinline__ int64_t yslot(int64_t s, int a, int pmax) {
    return (((s >> 4) * pmax + a) << 4) + (s & 15);
}

__device__ __forceinline__ bool skip(const ApplyGeom& g) { return g.stop && *g.stop; }

// Block order for an XCD-aware launch: workgroups go to the 8 XCDs round-
// robin, so block b runs on XCD b % 8; this bijection gives XCD x one
// contiguous range of logical blocks, so neighbouring tiles share that XCD's
// L2 (the residual entries they gather stay in one cache).
__device__ __forceinline__ int64_t block_id(bool remap) {
    const int64_t b = blockIdx.x;
    if (!remap) return b;
    const int64_t nb = gridDim.x, per = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
    return x * per + (x < rem ? x : rem) + i;
}

template <typename TX, typename TA, typename TY, int MAXP, int G, bool TWO>
__global__ __launch_bounds__(256) void k_apply_rows(int64_t count, ApplyGeom g, const TX* __restrict__ db,
                                                    const double* __restrict__ W, double omega,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ z, TY* __restrict__ Y) {
    // the stop flag is read before the stores (every wave sees the same
    // value, so all leave at the same point)
    const int a = threadIdx.x % G;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / G);
    for (int64_t s = (int64_t)blockIdx.x * (blockDim.x / G) + threadIdx.x / G; s < count; s += groups) {
        const int64_t o = g.goff ? g.goff[s] : s * g.pst;
        const int p = g.goff ? (int)(g.goff[s + 1] - o) : g.pst;
        const int32_t j = g.gphi[s];
        const TX* X = db + (g.dboff ? g.dboff[j] : (int64_t)j * g.dbst);
        // FP64: loads unconditional from clamped (valid) addresses, the
        // unused values dropped afterwards (a load under a condition becomes
        // a branch whose join waits for it).  FP32 keeps the guarded form for
        // the dof and residual (it measured twice as fast there: C4-sized
        // uneven batch, 332 against 708 us per application; FP64 461 against
        // 515 us).
        const bool act = a < p;
        const int ac = act ? a : 0;
        int32_t gd;
        TA rv;
        if constexpr (sizeof(TX) == 4) {
            gd = act ? g.gdofs[o + a] : 0;
            rv = act ? (TA)r[gd] : (TA)0;
        } else {
            gd = g.gdofs[o + ac];
            const double rl = r[gd];
            rv = act ? (TA)rl : (TA)0;
        }
        TX xr[MAXP];
        if constexpr (sizeof(TX) == 4 || MAXP <= 24) {
            // the group's p x p inverse is contiguous: G lanes read it at
            // consecutive addresses (clamped, coalesced) into LDS, then each
            // lane takes its row from there (FP64 only up to p = 24, where
            // the LDS of a block stays at 36 KB).  The group lies inside one
            // wavefront, whose LDS accesses complete in order; the fences
            // keep the compiler from moving them across each other.
            __shared__ TX s_x[(256 / G) * MAXP * MAXP];
            TX* sx = s_x + (threadIdx.x / G) * (MAXP * MAXP);
            const int pp = p * p;
            constexpr int U = (MAXP * MAXP + G - 1) / G;
            TX v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = a + u * G;
                v[u] = X[e < pp ? e : 0];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = a + u * G;
                if (e < pp) sx[e] = v[u];
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int b = 0; b < MAXP; ++b) xr[b] = (act && b < p) ? sx[ac * p + b] : (TX)0;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else if ((p & 1) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
            // even p and an aligned matrix: rows start on 16-byte boundaries, load pairs
            const double2* X2 = reinterpret_cast<const double2*>(X + (int64_t)ac * p);
#pragma unroll
            for (int b = 0; b < MAXP / 2; ++b) {
                const double2 v = X2[2 * b < p ? b : 0];
                const bool keep = act && 2 * b < p;
                xr[2 * b] = keep ? (TX)v.x : (TX)0;
                xr[2 * b + 1] = keep ? (TX)v.y : (TX)0;
            }
        } else {
#pragma unroll
            for (int b = 0; b < MAXP; ++b) {
                const TX v = X[(int64_t)ac * p + (b < p ? b : 0)];
                xr[b] = (act && b < p) ? v : (TX)0;
            }
        }
        TA acc = 0;
#pragma unroll
        for (int b = 0; b < MAXP; ++b) {
            if (b < p) {
                const TA rb = __shfl(rv, b, G);
                acc = fma((TA)xr[b], rb, acc);
            }
        }
        if (skip(g)) return;
        if (act) {
            if (TWO) Y[yslot(s, a, g.ypm)] = (TY)acc;
            else atomicAdd(&z[gd], omega * W[gd] * (double)acc);
        }
    }
}

// launch shape: T threads per block (64..256), at most `cap` blocks (the
// kernels stride over their work, so any shape covers it all)
inline unsigned shape_blocks(int64_t work, int per_block, int64_t cap) {
    int64_t blocks = (work + per_block - 1) / per_block;
    const int64_t lim = cap > 0 ? cap : 262144;
    if (blocks > lim) blocks = lim;
    return (unsigned)(blocks < 1 ? 1 : blocks);
}

template <typename TX, typename TA, typename TY, bool TWO>
void run_rows(int64_t count, const ApplyGeom& g, const TX* db, const double* W, double omega,
              const double* r, double* z, TY* Y, int maxp, int T, int64_t cap, hipStream_t s) {
    if (count <= 0) return;
    const int G = maxp <= 4 ? 4 : maxp <= 16 ? 16 : 32;
    const unsigned nb = shape_blocks(count, T / G, cap);
    if (maxp <= 4) k_apply_rows<TX, TA, TY, 4, 4, TWO><<<nb, T, 0, s>>>(count, g, db, W, omega, r, z, Y);
    else if (maxp <= 12) k_apply_rows<TX, TA, TY, 12, 16, TWO><<<nb, T, 0, s>>>(count, g, db, W, omega, r, z, Y);
    else if (maxp <= 16) k_apply_rows<TX, TA, TY, 16, 16, TWO><<<nb, T, 0, s>>>(count, g, db, W, omega, r, z, Y);
    else if (maxp <= 24) k_apply_rows<TX, TA, TY, 24, 32, TWO><<<nb, T, 0, s>>>(count, g, db, W, omega, r, z, Y);
    else k_apply_rows<TX, TA, TY, 32, 32, TWO><<<nb, T, 0, s>>>(count, g, db, W, omega, r, z, Y);
}

// z_i = omega W_i sum over the slots of dof i (ascending slot order)
template <typename TY>
__global__ __launch_bounds__(256) void k_slot_sum(int64_t n, const int64_t* __restrict__ dof_ptr,
                                                  const int32_t* __restrict__ dof_slots,
                                                  const TY* __restrict__ Y, const double* __restrict__ W,
                                                  double omega, double* __restrict__ z,
                                                  const int32_t* __restrict__ stop) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = dof_ptr[i], b = dof_ptr[i + 1];
    double acc = 0.0;
    if (b - a <= 8) {
        // short list (the usual case): one round of independent loads
        const int rem = (int)(b - a);
        int32_t sl[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sl[u] = dof_slots[a + (u < rem ? u : 0)];   // rem >= 1
        TY yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[u] = Y[sl[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < rem) acc += (double)yv[u];
    } else {
        for (int64_t t = a; t < b; ++t) acc += (double)Y[dof_slots[t]];
    }
    if (stop && *stop) return;   // read before the store only
    z[i] = omega * W[i] * acc;
}

// ---------------------------------------------------------------------------
// grouped MFMA apply; one wavefront per work item (entry, start, count, p)
// MODE 0: BF16, 1: FP16 with power-of-two scales, 2: BF16 high/low split
// ---------------------------------------------------------------------------

template <int MODE>
struct LowOp {
    // the operand pair (high, low) of an FP32 value; low is zero unless split
    static __device__ __forceinline__ void cvt(float f, short& hi, short& lo) {
        if (MODE == 1) {
            hi = (short)f32_to_f16_rne(f);
            lo = 0;
        } else {
            const uint16_t h = f32_to_bf16_rne(f);
            hi = (short)h;
            lo = MODE == 2 ? (short)f32_to_bf16_rne(f - __uint_as_float((uint32_t)h << 16)) : 0;
        }
    }
};

template <int MODE>
__device__ __forceinline__ f4 mma16(s4 a, s4 b, f4 c) {
    if (MODE == 1)
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a), __builtin_bit_cast(h4, b), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

template <int MODE>
__device__ __forceinline__ f16v mma32(s4 a, s4 b, f16v c) {
    if (MODE == 1)
        return __builtin_amdgcn_mfma_f32_32x32x8f16(__builtin_bit_cast(h4, a), __builtin_bit_cast(h4, b), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

template <int MODE, bool TWO>
__global__ __launch_bounds__(256) void k_apply_mfma(const int32_t* __restrict__ items, int64_t n_items,
                                                    ApplyGeom g,
                                                    const uint16_t* __restrict__ db_lp,
                                                    const int64_t* __restrict__ dblp_off,
                                                    const int32_t* __restrict__ db_exp,
                                                    const double* __restrict__ W, double omega,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ z, float* __restrict__ Y) {
    // the stop flag is read before the stores (uniform: every wave leaves
    // at the same point)
    constexpr bool FP16 = MODE == 1;
    constexpr bool SPLIT = MODE == 2;
    const int l = threadIdx.x & (PR_WAVE - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / PR_WAVE);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x / PR_WAVE) + threadIdx.x / PR_WAVE; it < n_items;
         it += waves) {
        // one item per wavefront: its fields are wave-uniform (scalar
        // registers, scalar branch on p)
        const int4 item = *reinterpret_cast<const int4*>(items + 4 * it);
        const int32_t j = __builtin_amdgcn_readfirstlane(item.x);
        const int32_t start = __builtin_amdgcn_readfirstlane(item.y);
        const int32_t cnt = __builtin_amdgcn_readfirstlane(item.z);
        const int p = __builtin_amdgcn_readfirstlane(item.w);
        if (p <= 16) {
            // 16x16x16: member n = l%16, local dofs 4q..4q+3 with q = l/16
            const int n = l & 15, q = l >> 4;
            const bool mv = n < cnt;
            // unconditional loads from clamped addresses (no serialising branches)
            const int64_t sn = start + (mv ? n : 0);
            const int64_t st = g.goff ? g.goff[sn] : sn * g.pst;
            int32_t gi[4];
            float rv[4];
            {
                int32_t d[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) d[t] = g.gdofs[st + (4 * q + t < p ? 4 * q + t : 0)];
                // the empty asm keeps every load unconditional and in flight
                // together (a select of a loaded value would become a branch
                // around its load)
#pragma unroll
                for (int t = 0; t < 4; ++t) __asm__ volatile("" : "+v"(d[t]));
#pragma unroll
                for (int t = 0; t < 4; ++t) gi[t] = (mv && 4 * q + t < p) ? d[t] : -1;
            }
            // the entry's operand offset loads beside the dof lists, not before
            const uint16_t* Xl = db_lp + dblp_off[j];
            const int ej = FP16 ? db_exp[j] : 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double x = r[gi[t] >= 0 ? gi[t] : 0];
                rv[t] = gi[t] >= 0 ? (float)x : 0.0f;
            }
            int f = 0;
            if (FP16) {
                float m = fmaxf(fmaxf(fabsf(rv[0]), fabsf(rv[1])), fmaxf(fabsf(rv[2]), fabsf(rv[3])));
                m = fmaxf(m, __shfl_xor(m, 16));
                m = fmaxf(m, __shfl_xor(m, 32));
                f = fp16_scale_exp(m);
            }
            s4 bh, bl;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                short hi, lo;
                LowOp<MODE>::cvt(FP16 ? ldexpf(rv[t], -f) : rv[t], hi, lo);
                bh[t] = hi;
                bl[t] = lo;
            }
            const s4 ah = *reinterpret_cast<const s4*>(Xl + 4 * l);
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16<MODE>(ah, bh, acc);
            if (SPLIT) {
                const s4 al = *reinterpret_cast<const s4*>(Xl + 256 + 4 * l);
                acc = mma16<MODE>(ah, bl, acc);
                acc = mma16<MODE>(al, bh, acc);
            }
            if (skip(g)) return;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (gi[t] >= 0) {
                    if (TWO) {
                        Y[yslot(start + n, 4 * q + t, g.ypm)] = FP16 ? ldexpf(acc[t], ej + f) : acc[t];
                    } else {
                        double y = (double)acc[t];
                        if (FP16) y = ldexp(y, ej + f);
                        atomicAdd(&z[gi[t]], omega * W[gi[t]] * y);
                    }
                }
            }
        } else {
            // 32x32x8, K in steps of 8: member n = l%32, h = l/32,
            // local dofs 8s + 4h + t for step s and t < 4
            const int n = l & 31, h = l >> 5;
            const bool mv = n < cnt;
            const int64_t sn = start + (mv ? n : 0);
            const int64_t st = g.goff ? g.goff[sn] : sn * g.pst;
            const int steps = (p + 7) >> 3;
            int32_t gi[16];
            float rv[16];
            {
                int32_t d[16];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int kk = 8 * s + 4 * h + t;
                        d[4 * s + t] = g.gdofs[st + (kk < p ? kk : 0)];
                    }
#pragma unroll
                for (int v = 0; v < 16; ++v) __asm__ volatile("" : "+v"(d[v]));
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int kk = 8 * s + 4 * h + t;
                        gi[4 * s + t] = (mv && kk < p) ? d[4 * s + t] : -1;
                    }
            }
            const uint16_t* Xl = db_lp + dblp_off[j];
            const int ej = FP16 ? db_exp[j] : 0;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const double x = r[gi[v] >= 0 ? gi[v] : 0];
                rv[v] = gi[v] >= 0 ? (float)x : 0.0f;
            }
            int f = 0;
            if (FP16) {
                float m = 0.0f;
#pragma unroll
                for (int t = 0; t < 16; ++t) m = fmaxf(m, fabsf(rv[t]));
                m = fmaxf(m, __shfl_xor(m, 32));
                f = fp16_scale_exp(m);
            }
            f16v acc = {};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (s < steps) {
                    s4 bh, bl;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        short hi, lo;
                        LowOp<MODE>::cvt(FP16 ? ldexpf(rv[4 * s + t], -f) : rv[4 * s + t], hi, lo);
                        bh[t] = hi;
                        bl[t] = lo;
                    }
                    const s4 ah = *reinterpret_cast<const s4*>(Xl + (s * 64 + l) * 4);
                    acc = mma32<MODE>(ah, bh, acc);
                    if (SPLIT) {
                        const s4 al = *reinterpret_cast<const s4*>(Xl + 1024 + (s * 64 + l) * 4);
                        acc = mma32<MODE>(ah, bl, acc);
                        acc = mma32<MODE>(al, bh, acc);
                    }
                }
            }
            if (skip(g)) return;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                if (gi[v] >= 0) {
                    if (TWO) {
                        Y[yslot(start + n, 8 * (v >> 2) + 4 * h + (v & 3), g.ypm)] =
                            FP16 ? ldexpf(acc[v], ej + f) : acc[v];
                    } else {
                        double y = (double)acc[v];
                        if (FP16) y = ldexp(y, ej + f);
                        atomicAdd(&z[gi[v]], omega * W[gi[v]] * y);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// grouped MFMA apply over fixed tiles (every patch has p dofs): tile t is the
// NB consecutive grouped positions t*NB .. t*NB+NB-1 (NB = 16 for p <= 16,
// 32 for p <= 32), one wavefront per tile, no work-item list.  A tile may
// straddle database entries: column n of an MFMA product depends on column n
// of the right operand only, so the wave runs one product per distinct entry
// of the tile (grouped order keeps them in runs) and each member keeps the
// columns of its own entry.  Results are bit-identical to the item kernel.
// ---------------------------------------------------------------------------
template <int MODE, bool TWO, bool BIG, int TPW, bool VEC4>
__global__ __launch_bounds__(256) void k_apply_tiles(int64_t n_p, int p, ApplyGeom g,
                                                     const uint16_t* __restrict__ db_lp, int64_t lp_stride,
                                                     const int32_t* __restrict__ db_exp,
                                                     const double* __restrict__ W, double omega,
                                                     const double* __restrict__ r,
                                                     double* __restrict__ z, float* __restrict__ Y) {
    // the stop flag is checked before the stores, not here: read at entry
    // it put two dependent scalar loads ahead of every wave's first vector
    // load; a stopped wave still writes nothing
    constexpr bool FP16 = MODE == 1;
    constexpr bool SPLIT = MODE == 2;
    constexpr int NB = BIG ? 32 : 16;      // members per tile
    constexpr int NV = BIG ? 16 : 4;       // rows held per lane
    constexpr int NC = NV / 4;             // K steps (groups of 4 rows) per lane
    constexpr int L = BIG ? 1024 : 256;    // elements of one lane-ready operand copy
    constexpr int EB = BIG ? 2 : 4;        // entries per operand batch
    typedef float accv __attribute__((ext_vector_type(NV)));   // f4 or f16v
    const int l = threadIdx.x & (PR_WAVE - 1);
    const int n = l & (NB - 1), h = l / NB;
    // VEC4: p % 4 == 0, rows in aligned groups of 4 dofs. A compile-time
    // choice: as a run-time branch it made the entry load wait behind the
    // dof lists, a third dependent load round trip per tile.
    constexpr bool vec4 = VEC4;
    const int steps = (p + 7) >> 3;
    const int64_t n_tiles = (n_p + NB - 1) / NB;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / PR_WAVE) * TPW;
    // TPW tiles per wave, loaded together (more loads in flight per wave)
    for (int64_t t0 = (block_id(g.remap) * (blockDim.x / PR_WAVE) + threadIdx.x / PR_WAVE) * TPW;
         t0 < n_tiles; t0 += stride) {
        int32_t jm[TPW], gi[TPW][NV];
        bool mv[TPW];
        // 1: entry and dof list of each member
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int64_t s = (t0 + u) * NB + n;
            // Every load below is unconditional from a clamped (valid)
            // address, the unused values dropped afterwards: a load under a
            // condition becomes a branch whose join waits for it, which
            // serialised the gathers.
            mv[u] = s < n_p;                                 // false for the whole tile past the end
            const int64_t sc = mv[u] ? s : n_p - 1;
            const int32_t jl = g.gphi[sc];
            jm[u] = mv[u] ? jl : 0x7fffffff;
            const int32_t* gd = g.gdofs + sc * p;
            int32_t d[NV];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int row0 = BIG ? 8 * c + 4 * h : 4 * h;   // rows row0 .. row0+3
                if (vec4) {
                    const int4 v4 = *reinterpret_cast<const int4*>(gd + (row0 < p ? row0 : 0));
                    d[4 * c + 0] = v4.x;
                    d[4 * c + 1] = v4.y;
                    d[4 * c + 2] = v4.z;
                    d[4 * c + 3] = v4.w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) d[4 * c + e] = gd[row0 + e < p ? row0 + e : 0];
                }
            }
            // Scalar loads: the empty asm consumes every loaded value after
            // all of them are issued, so each load stays unconditional and
            // in flight with the others. A select between a load and a
            // constant is otherwise turned into a branch around the load,
            // with a full wait at its join (one round trip per row).
            if (!vec4) {
#pragma unroll
                for (int v = 0; v < NV; ++v) __asm__ volatile("" : "+v"(d[v]));
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int row0 = BIG ? 8 * c + 4 * h : 4 * h;
#pragma unroll
                for (int e = 0; e < 4; ++e) gi[u][4 * c + e] = (mv[u] && row0 + e < p) ? d[4 * c + e] : -1;
            }
        }
        // 2: residual gathers, and the operand of each tile's first entry
        float rv[TPW][NV];
        int32_t cur[TPW];
        s4 ah[TPW][NC], al[TPW][NC];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double x = r[gi[u][v] >= 0 ? gi[u][v] : 0];
                rv[u][v] = gi[u][v] >= 0 ? (float)x : 0.0f;
            }
            cur[u] = __builtin_amdgcn_readfirstlane(jm[u]);    // member 0's entry (lane 0)
            const uint16_t* Xl = db_lp + (int64_t)(t0 + u < n_tiles ? cur[u] : 0) * lp_stride;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                // steps past p read step 0 again; their products are skipped
                const int cc = (!BIG || c < steps) ? c : 0;
                ah[u][c] = *reinterpret_cast<const s4*>(Xl + (cc * 64 + l) * 4);
                if (SPLIT) al[u][c] = *reinterpret_cast<const s4*>(Xl + L + (cc * 64 + l) * 4);
            }
        }
        // 3: products, one per distinct entry of a tile; 4: slot writes
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            if (t0 + u >= n_tiles) break;
            int f = 0;
            if (FP16) {
                float m = 0.0f;
#pragma unroll
                for (int v = 0; v < NV; ++v) m = fmaxf(m, fabsf(rv[u][v]));
                if (!BIG) m = fmaxf(m, __shfl_xor(m, 16));
                m = fmaxf(m, __shfl_xor(m, 32));
                f = fp16_scale_exp(m);
            }
            s4 bh[NC], bl[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    short hi, lo;
                    LowOp<MODE>::cvt(FP16 ? ldexpf(rv[u][4 * c + e], -f) : rv[u][4 * c + e], hi, lo);
                    bh[c][e] = hi;
                    bl[c][e] = lo;
                }
            accv out = {};
            int oe = 0;
            // distinct entries of the tile in batches of EB, the operands of a
            // batch loaded together (a tile over many small groups would
            // otherwise wait for one load per entry)
            int32_t j = cur[u];
            bool first = true;
            // the common case, one entry in the whole tile: one product with
            // the operand loaded ahead, none of the batch machinery
            const bool single = __ballot(mv[u] && jm[u] != j) == 0;
            if (single) {
                accv acc = {};
                if constexpr (BIG) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if (c < steps) {
                            acc = mma32<MODE>(ah[u][c], bh[c], acc);
                            if (SPLIT) {
                                acc = mma32<MODE>(ah[u][c], bl[c], acc);
                                acc = mma32<MODE>(al[u][c], bh[c], acc);
                            }
                        }
                    }
                } else {
                    acc = mma16<MODE>(ah[u][0], bh[0], acc);
                    if (SPLIT) {
                        acc = mma16<MODE>(ah[u][0], bl[0], acc);
                        acc = mma16<MODE>(al[u][0], bh[0], acc);
                    }
                }
                out = acc;
                if (FP16) oe = db_exp[j] + f;
            }
            while (!single) {
                int32_t e[EB];
                bool ex[EB];
                e[0] = j;
                ex[0] = true;
#pragma unroll
                for (int k = 1; k < EB; ++k) {
                    const uint64_t more = __ballot(mv[u] && jm[u] > e[k - 1]);
                    ex[k] = ex[k - 1] && more != 0;
                    e[k] = ex[k] ? __shfl(jm[u], (int)__builtin_ctzll(more)) : e[k - 1];
                }
                s4 xa[EB][NC], xb[EB][NC];
                int ee[EB];
#pragma unroll
                for (int k = 0; k < EB; ++k) {
                    // e[k] repeats a valid entry when the batch has fewer
                    // entries, so every load is unconditional
                    const uint16_t* Xl = db_lp + (int64_t)e[k] * lp_stride;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if (k == 0 && first) {
                            xa[k][c] = ah[u][c];
                            if (SPLIT) xb[k][c] = al[u][c];
                        } else {
                            const int cc = (!BIG || c < steps) ? c : 0;
                            xa[k][c] = *reinterpret_cast<const s4*>(Xl + (cc * 64 + l) * 4);
                            if (SPLIT) xb[k][c] = *reinterpret_cast<const s4*>(Xl + L + (cc * 64 + l) * 4);
                        }
                    }
                    ee[k] = FP16 ? db_exp[e[k]] : 0;
                }
#pragma unroll
                for (int k = 0; k < EB; ++k) {
                    if (!ex[k]) break;
                    accv acc = {};
                    if constexpr (BIG) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            if (c < steps) {
                                acc = mma32<MODE>(xa[k][c], bh[c], acc);
                                if (SPLIT) {
                                    acc = mma32<MODE>(xa[k][c], bl[c], acc);
                                    acc = mma32<MODE>(xb[k][c], bh[c], acc);
                                }
                            }
                        }
                    } else {
                        acc = mma16<MODE>(xa[k][0], bh[0], acc);
                        if (SPLIT) {
                            acc = mma16<MODE>(xa[k][0], bl[0], acc);
                            acc = mma16<MODE>(xb[k][0], bh[0], acc);
                        }
                    }
                    if (jm[u] == e[k]) {
                        out = acc;
                        if (FP16) oe = ee[k] + f;
                    }
                }
                if (!ex[EB - 1]) break;
                const uint64_t more = __ballot(mv[u] && jm[u] > e[EB - 1]);
                if (more == 0) break;
                j = __shfl(jm[u], (int)__builtin_ctzll(more));
                first = false;
            }
            if (skip(g)) return;
            const int64_t s = (t0 + u) * NB + n;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (gi[u][v] >= 0) {
                    const int row = BIG ? 8 * (v >> 2) + 4 * h + (v & 3) : 4 * h + v;
                    if (TWO) {
                        Y[yslot(s, row, g.ypm)] = FP16 ? ldexpf(out[v], oe) : out[v];
                    } else {
                        double y = (double)out[v];
                        if (FP16) y = ldexp(y, oe);
                        atomicAdd(&z[gi[u][v]], omega * W[gi[u][v]] * y);
                    }
                }
            }
        }
    }
}

// z_i = omega / c_i * sum of the c_i slots of dof i, from a padded table of
// C slots per dof (ascending, -1 after the last); 1 / c_i is W_i.  Same
// summation order, hence the same bits, as k_slot_sum.
template <typename TY, int C>
__global__ __launch_bounds__(256) void k_slot_sum_ell(int64_t n, const int32_t* __restrict__ ell,
                                                      const TY* __restrict__ Y, double omega,
                                                      double* __restrict__ z, const int32_t* __restrict__ stop,
                                                      int remap) {
    const int64_t i = block_id(remap) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t sl[C];
    if (C >= 4) {
#pragma unroll
        for (int u = 0; u < C; u += 4) {
            const int4 v = *reinterpret_cast<const int4*>(ell + i * C + u);
            sl[u] = v.x;
            sl[u + 1] = v.y;
            sl[u + 2] = v.z;
            sl[u + 3] = v.w;
        }
    } else if (C == 2) {
        const int2 v = *reinterpret_cast<const int2*>(ell + i * 2);
        sl[0] = v.x;
        sl[C - 1] = v.y;
    } else {
        sl[0] = ell[i];
    }
    TY yv[C];
#pragma unroll
    for (int u = 0; u < C; ++u) yv[u] = Y[sl[u] >= 0 ? sl[u] : 0];    // unconditional: no serialising branch
    double acc = 0.0;
    int c = 0;
#pragma unroll
    for (int u = 0; u < C; ++u) {
        if (sl[u] >= 0) {
            acc += (double)yv[u];
            ++c;
        }
    }
    // the stop flag is checked before the store only (at entry it delayed
    // every wave's first load by two dependent scalar loads)
    if (stop && *stop) return;
    z[i] = omega * (1.0 / (double)c) * acc;
}

// ---------------------------------------------------------------------------
// database conversion: one wavefront per entry
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_convert_db(int prec, int64_t m_p, const double* __restrict__ db,
                                                   const int64_t* __restrict__ dboff,
                                                   const int32_t* __restrict__ dbps, int uniform_ps,
                                                   uint16_t* __restrict__ db_lp,
                                                   const int64_t* __restrict__ dblp_off,
                                                   int32_t* __restrict__ db_exp, float* __restrict__ db_f32) {
    const int l = threadIdx.x;
    for (int64_t j = blockIdx.x; j < m_p; j += gridDim.x) {
        const int p = uniform_ps ? uniform_ps : dbps[j];
        const int64_t off = uniform_ps ? j * (int64_t)p * p : dboff[j];
        const double* X = db + off;
        // row-major FP32 copy for the FP32 vector kernel
        float m = 0.0f;
        for (int e = l; e < p * p; e += PR_WAVE) {
            const double v = X[e];
            if (db_f32) db_f32[off + e] = (float)v;
            m = fmaxf(m, fabsf((float)v));
        }
        m = wave_max(m);
        const int e = (prec == PR_FP16) ? fp16_scale_exp(m) : 0;
        if (l == 0 && db_exp) db_exp[j] = e;
        if (prec != PR_BF16 && prec != PR_FP16 && prec != PR_BF16X3) continue;
        uint16_t* out = db_lp + dblp_off[j];
        const int L = p <= 16 ? 256 : 1024;       // elements of one lane-ready copy
        for (int s = 0; s < (p <= 16 ? 1 : 4); ++s)
            for (int t = 0; t < 4; ++t) {
                int i, k;
                if (p <= 16) {
                    i = l & 15;
                    k = 4 * (l >> 4) + t;
                } else {
                    i = l & 31;
                    k = 8 * s + 4 * (l >> 5) + t;
                }
                const float v = (i < p && k < p) ? (float)X[i * p + k] : 0.0f;
                const int slot = (s * 64 + l) * 4 + t;
                if (prec == PR_FP16) {
                    out[slot] = f32_to_f16_rne(ldexpf(v, -e));
                } else {
                    const uint16_t hi = f32_to_bf16_rne(v);
                    out[slot] = hi;
                    if (prec == PR_BF16X3)
                        out[L + slot] = f32_to_bf16_rne(v - __uint_as_float((uint32_t)hi << 16));
                }
            }
    }
}

}  // namespace

void launch_apply(int prec, bool two_stage, const ApplyLaunch& a, hipStream_t s) {
    ApplyGeom g{a.gdofs, a.goff, a.pst, a.gphi, a.dboff, a.dbst, a.stop, a.maxp, a.xcd_remap};
    const int T = (a.threads == 64 || a.threads == 128) ? a.threads : 256;
    const int64_t cap = a.grid_cap;
    if (a.wide) {
        launch_apply_wide(prec, two_stage, a, s);
    } else if (prec == PR_FP64) {
        if (two_stage) run_rows<double, double, double, true>(a.n_p, g, a.db, a.W, a.omega, a.r, a.z, (double*)a.Y, a.maxp, T, cap, s);
        else run_rows<double, double, double, false>(a.n_p, g, a.db, a.W, a.omega, a.r, a.z, (double*)nullptr, a.maxp, T, cap, s);
    } else if (prec == PR_FP32) {
        if (two_stage) run_rows<float, float, float, true>(a.n_p, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)a.Y, a.maxp, T, cap, s);
        else run_rows<float, float, float, false>(a.n_p, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)nullptr, a.maxp, T, cap, s);
    } else if (a.tile_p > 0) {
        // every patch has tile_p dofs: fixed tiles, no work items
        const bool big = a.tile_p > 16;
        const int NB = big ? 32 : 16;
        const int64_t n_tiles = (a.n_p + NB - 1) / NB;
        const int mode = prec == PR_FP16 ? 1 : prec == PR_BF16X3 ? 2 : 0;
        const int64_t lp_stride = (mode == 2 ? 2 : 1) * (big ? 1024 : 256);
        // dof lists read 4 rows at a time when p % 4 == 0
        const bool vec4 = (a.tile_p & 3) == 0;
        // tiles per wave: 1 unless the shape asks for 2 or 4 (16-member
        // tiles with p % 4 == 0 only)
        const int tpw = (!big && vec4 && (a.tiles_per_wave == 2 || a.tiles_per_wave == 4)) ? a.tiles_per_wave : 1;
        if (n_tiles > 0) {
            const unsigned nb = shape_blocks((n_tiles + tpw - 1) / tpw, T / PR_WAVE, cap);
#define PR_TILE(MODE, TWO, BIG, U, V4) k_apply_tiles<MODE, TWO, BIG, U, V4><<<nb, T, 0, s>>>(a.n_p, a.tile_p, g, a.db_lp, lp_stride, a.db_exp, a.W, a.omega, a.r, a.z, (float*)a.Y)
#define PR_TILE_M(TWO, BIG, U, V4) \
    if (mode == 0) PR_TILE(0, TWO, BIG, U, V4); else if (mode == 1) PR_TILE(1, TWO, BIG, U, V4); else PR_TILE(2, TWO, BIG, U, V4)
            if (two_stage) {
                if (big && vec4) { PR_TILE_M(true, true, 1, true); }
                else if (big) { PR_TILE_M(true, true, 1, false); }
                else if (!vec4) { PR_TILE_M(true, false, 1, false); }
                else if (tpw == 4) { PR_TILE_M(true, false, 4, true); }
                else if (tpw == 2) { PR_TILE_M(true, false, 2, true); }
                else { PR_TILE_M(true, false, 1, true); }
            } else {
                if (big && vec4) { PR_TILE_M(false, true, 1, true); }
                else if (big) { PR_TILE_M(false, true, 1, false); }
                else if (!vec4) { PR_TILE_M(false, false, 1, false); }
                else if (tpw == 4) { PR_TILE_M(false, false, 4, true); }
                else if (tpw == 2) { PR_TILE_M(false, false, 2, true); }
                else { PR_TILE_M(false, false, 1, true); }
            }
#undef PR_TILE_M
#undef PR_TILE
        }
    } else {
        if (a.n_items > 0) {
            const unsigned nb = shape_blocks(a.n_items, T / PR_WAVE, cap);
#define PR_MFMA(MODE, TWO) k_apply_mfma<MODE, TWO><<<nb, T, 0, s>>>(a.items, a.n_items, g, a.db_lp, a.dblp_off, a.db_exp, a.W, a.omega, a.r, a.z, (float*)a.Y)
            const int mode = prec == PR_FP16 ? 1 : prec == PR_BF16X3 ? 2 : 0;
            if (two_stage) {
                if (mode == 0) PR_MFMA(0, true); else if (mode == 1) PR_MFMA(1, true); else PR_MFMA(2, true);
            } else {
                if (mode == 0) PR_MFMA(0, false); else if (mode == 1) PR_MFMA(1, false); else PR_MFMA(2, false);
            }
#undef PR_MFMA
        }
    }
    if (two_stage) {
        const int T2 = (a.slot_threads == 64 || a.slot_threads == 128) ? a.slot_threads : 256;
        const unsigned nb = (unsigned)((a.n + T2 - 1) / T2);
        if (a.ell_c > 0) {
#define PR_ELL(TY, C) k_slot_sum_ell<TY, C><<<nb, T2, 0, s>>>(a.n, a.ell, (const TY*)a.Y, a.omega, a.z, a.stop, a.xcd_remap)
#define PR_ELL_C(TY) \
    if (a.ell_c == 1) PR_ELL(TY, 1); else if (a.ell_c == 2) PR_ELL(TY, 2); else if (a.ell_c == 4) PR_ELL(TY, 4); else PR_ELL(TY, 8)
            if (prec == PR_FP64) { PR_ELL_C(double); } else { PR_ELL_C(float); }
#undef PR_ELL_C
#undef PR_ELL
        } else if (prec == PR_FP64)
            k_slot_sum<double><<<nb, T2, 0, s>>>(a.n, a.dof_ptr, a.dof_slots, (const double*)a.Y, a.W, a.omega, a.z, a.stop);
        else
            k_slot_sum<float><<<nb, T2, 0, s>>>(a.n, a.dof_ptr, a.dof_slots, (const float*)a.Y, a.W, a.omega, a.z, a.stop);
    }
}

void launch_convert_db(int prec, int64_t m_p, const double* db, const int64_t* dboff,
                       const int32_t* dbps, int uniform_ps, uint16_t* db_lp,
                       const int64_t* dblp_off, int32_t* db_exp, float* db_f32, hipStream_t s) {
    if (m_p <= 0) return;
    int64_t blocks = m_p < 65536 ? m_p : 65536;
    k_convert_db<<<(unsigned)blocks, 64, 0, s>>>(prec, m_p, db, dboff, dbps, uniform_ps, db_lp,
                                                dblp_off, db_exp, db_f32);
}
