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
};

// Slot of local row a of grouped patch s: patches in tiles of 16, inside a
// tile row-plane by row-plane (16 consecutive patches' row a contiguous).
// A block or an MFMA item writes whole tiles, and the per-dof sum finds the
// rows of neighbouring patches next to each other.
__device__ __forceinline__ int64_t yslot(int64_t s, int a, int pmax) {
    return (((s >> 4) * pmax + a) << 4) + (s & 15);
}

__device__ __forceinline__ bool skip(const ApplyGeom& g) { return g.stop && *g.stop; }

template <typename TX, typename TA, typename TY, int MAXP, int G, bool TWO>
__global__ __launch_bounds__(256) void k_apply_rows(int64_t count, ApplyGeom g, const TX* __restrict__ db,
                                                    const double* __restrict__ W, double omega,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ z, TY* __restrict__ Y) {
    if (skip(g)) return;
    const int a = threadIdx.x % G;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / G);
    for (int64_t s = (int64_t)blockIdx.x * (blockDim.x / G) + threadIdx.x / G; s < count; s += groups) {
        const int64_t o = g.goff ? g.goff[s] : s * g.pst;
        const int p = g.goff ? (int)(g.goff[s + 1] - o) : g.pst;
        const int32_t j = g.gphi[s];
        const TX* X = db + (g.dboff ? g.dboff[j] : (int64_t)j * g.dbst);
        const bool act = a < p;
        const int32_t gd = act ? g.gdofs[o + a] : 0;
        const TA rv = act ? (TA)r[gd] : (TA)0;
        TX xr[MAXP];
        if (sizeof(TX) == 8 && (p & 1) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
            // even p and an aligned matrix: rows start on 16-byte boundaries, load pairs
            const double2* X2 = reinterpret_cast<const double2*>(X + (int64_t)a * p);
#pragma unroll
            for (int b = 0; b < MAXP / 2; ++b) {
                const double2 v = (act && 2 * b < p) ? X2[b] : make_double2(0.0, 0.0);
                xr[2 * b] = (TX)v.x;
                xr[2 * b + 1] = (TX)v.y;
            }
        } else {
#pragma unroll
            for (int b = 0; b < MAXP; ++b) xr[b] = (act && b < p) ? X[(int64_t)a * p + b] : (TX)0;
        }
        TA acc = 0;
#pragma unroll
        for (int b = 0; b < MAXP; ++b) {
            if (b < p) {
                const TA rb = __shfl(rv, b, G);
                acc = fma((TA)xr[b], rb, acc);
            }
        }
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
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = dof_ptr[i], b = dof_ptr[i + 1];
    double acc = 0.0;
    if (b - a <= 8) {
        // short list (the usual case): one round of independent loads
        const int rem = (int)(b - a);
        int32_t sl[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sl[u] = u < rem ? dof_slots[a + u] : 0;
        TY yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[u] = u < rem ? Y[sl[u]] : (TY)0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < rem) acc += (double)yv[u];
    } else {
        for (int64_t t = a; t < b; ++t) acc += (double)Y[dof_slots[t]];
    }
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
    if (skip(g)) return;
    constexpr bool FP16 = MODE == 1;
    constexpr bool SPLIT = MODE == 2;
    const int l = threadIdx.x & (PR_WAVE - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / PR_WAVE);
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x / PR_WAVE) + threadIdx.x / PR_WAVE; it < n_items;
         it += waves) {
        const int32_t j = items[4 * it + 0];
        const int32_t start = items[4 * it + 1];
        const int32_t cnt = items[4 * it + 2];
        const int p = items[4 * it + 3];
        const uint16_t* Xl = db_lp + dblp_off[j];
        const int ej = FP16 ? db_exp[j] : 0;
        if (p <= 16) {
            // 16x16x16: member n = l%16, local dofs 4q..4q+3 with q = l/16
            const int n = l & 15, q = l >> 4;
            const bool mv = n < cnt;
            int64_t st = 0;
            if (mv) st = g.goff ? g.goff[start + n] : (int64_t)(start + n) * g.pst;
            int32_t gi[4];
            float rv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int kk = 4 * q + t;
                const bool v = mv && kk < p;
                gi[t] = v ? g.gdofs[st + kk] : -1;
                rv[t] = v ? (float)r[gi[t]] : 0.0f;
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
            int64_t st = 0;
            if (mv) st = g.goff ? g.goff[start + n] : (int64_t)(start + n) * g.pst;
            const int steps = (p + 7) >> 3;
            int32_t gi[16];
            float rv[16];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int kk = 8 * s + 4 * h + t;
                    const bool v = mv && kk < p;
                    gi[4 * s + t] = v ? g.gdofs[st + kk] : -1;
                    rv[4 * s + t] = v ? (float)r[gi[4 * s + t]] : 0.0f;
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
    ApplyGeom g{a.gdofs, a.goff, a.pst, a.gphi, a.dboff, a.dbst, a.stop, a.maxp};
    const int T = (a.threads == 64 || a.threads == 128) ? a.threads : 256;
    const int64_t cap = a.grid_cap;
    if (prec == PR_FP64) {
        if (two_stage) run_rows<double, double, double, true>(a.n_p, g, a.db, a.W, a.omega, a.r, a.z, (double*)a.Y, a.maxp, T, cap, s);
        else run_rows<double, double, double, false>(a.n_p, g, a.db, a.W, a.omega, a.r, a.z, (double*)nullptr, a.maxp, T, cap, s);
    } else if (prec == PR_FP32) {
        if (two_stage) run_rows<float, float, float, true>(a.n_p, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)a.Y, a.maxp, T, cap, s);
        else run_rows<float, float, float, false>(a.n_p, g, a.db_f32, a.W, a.omega, a.r, a.z, (float*)nullptr, a.maxp, T, cap, s);
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
        if (prec == PR_FP64)
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
