// GMRES over a block-diagonal batch of independent systems (uneven batches
// of many small problems, each solved to its own tolerance): one Krylov
// space, one Hessenberg matrix, one set of Givens rotations and one stopping
// test per system, all systems advancing in the same launches.  A system
// that has met its test is masked: its rows take no further updates.
//
// Rows are cut into chunks that never straddle two systems; every
// reduction is a per-chunk partial followed by a per-system sum over its
// chunks in order, so the result does not depend on timing and equals, for
// each system, the single-system algorithm on that system's rows.
#include "pr_internal.h"

namespace {

constexpr int kMaxVec = 32;
constexpr int kThreads = 256;

__device__ __forceinline__ bool gstopped(const int32_t* gstop) { return gstop && *gstop; }

// MODE 0: out_i = V_i . w ; MODE 1: w -= sum c_i V_i, out_i = V_i . w ;
// MODE 2: w -= sum c_i V_i, out_0 = w . w   (c and out per system)
// NC = ceil(nv / 8): the vector loads of a row carry no branches between
// them (indices past nv repeat vector nv - 1, whose terms are dropped).
template <int MODE, int NC>
__global__ __launch_bounds__(kThreads) void k_bgs(const double* __restrict__ V, int64_t ldv, int nv,
                                                  double* __restrict__ w, BGeom g, const double* __restrict__ c,
                                                  double* __restrict__ partial, const int32_t* __restrict__ sstop,
                                                  const int32_t* __restrict__ gstop) {
    if (gstopped(gstop)) return;
    constexpr int NV = 8 * NC;
    constexpr int NO = (MODE == 2) ? 1 : NV;
    __shared__ double s_red[kThreads / PR_WAVE][kMaxVec];
    const int nout = (MODE == 2) ? 1 : nv;
    int64_t vo[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vo[i] = (int64_t)(i < nv ? i : (nv > 0 ? nv - 1 : 0)) * ldv;
    for (int64_t ch = blockIdx.x; ch < g.nch; ch += gridDim.x) {
        const int sys = g.ch_sys[ch];
        if (sstop && sstop[sys]) continue;
        double cf[NV];
        if (MODE >= 1) {
#pragma unroll
            for (int i = 0; i < NV; ++i) cf[i] = (i < nv) ? c[(int64_t)sys * kBStride + i] : 0.0;
        }
        double acc[NO];
#pragma unroll
        for (int i = 0; i < NO; ++i) acc[i] = 0.0;
        const int64_t lo = g.ch_lo[ch], hi = lo + g.ch_len[ch];
        for (int64_t q = lo + threadIdx.x; q < hi; q += kThreads) {
            double wq = w[q];
            double v[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] = V[vo[i] + q];
            __builtin_amdgcn_sched_barrier(0);   // all loads of the row in flight together
            if (MODE == 0) {
#pragma unroll
                for (int i = 0; i < NV; ++i) acc[i] = fma(v[i], wq, acc[i]);
            } else {
#pragma unroll
                for (int i = 0; i < NV; ++i) wq = fma(-cf[i], v[i], wq);    // cf = 0 past nv
                w[q] = wq;
                if (MODE == 1) {
#pragma unroll
                    for (int i = 0; i < NV; ++i) acc[i] = fma(v[i], wq, acc[i]);
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
            for (int w2 = 0; w2 < kThreads / PR_WAVE; ++w2) t += s_red[w2][threadIdx.x];
            partial[ch * kMaxVec + threadIdx.x] = t;
        }
        __syncthreads();
    }
}

// out[sys][obase + i] = sum over the chunks of sys (in order) of partial[ch][i]
__global__ void k_bgs_final(int nout, BGeom g, const double* __restrict__ partial, double* __restrict__ out,
                            int obase, const int32_t* __restrict__ sstop, const int32_t* __restrict__ gstop) {
    if (gstopped(gstop)) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.nsys * nout) return;
    const int sys = (int)(t / nout), i = (int)(t % nout);
    if (sstop && sstop[sys]) return;
    const int64_t c0 = g.sys_ch0[sys], nc = g.sys_nch[sys];
    double s = 0.0;
    for (int64_t c = 0; c < nc; ++c) s += partial[(c0 + c) * kMaxVec + i];
    out[(int64_t)sys * kBStride + obase + i] = s;
}

// dst = src / sqrt(denom[sys][0]) on the rows of active systems
__global__ void k_bscale(const double* __restrict__ src, double* __restrict__ dst, BGeom g,
                         const double* __restrict__ denom, const int32_t* __restrict__ sstop,
                         const int32_t* __restrict__ gstop) {
    if (gstopped(gstop)) return;
    for (int64_t ch = blockIdx.x; ch < g.nch; ch += gridDim.x) {
        const int sys = g.ch_sys[ch];
        if (sstop && sstop[sys]) continue;
        const double d = sqrt(denom[(int64_t)sys * kBStride]);
        const int64_t lo = g.ch_lo[ch], hi = lo + g.ch_len[ch];
        for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) dst[q] = d > 0.0 ? src[q] / d : 0.0;
    }
}

// per system: column j of the Hessenberg matrix, rotations, residual
// estimate and the stopping test; one block, systems strided over threads;
// gstop = 1 once every system has stopped
__global__ __launch_bounds__(1024) void k_bgivens(int j, int m, int nsys, const double* __restrict__ h1,
                                                  const double* __restrict__ h2, const double* __restrict__ hn,
                                                  double* __restrict__ Rall, double* __restrict__ csall,
                                                  double* __restrict__ snall, double* __restrict__ gall,
                                                  double* __restrict__ est, int32_t* __restrict__ sstop,
                                                  int32_t* __restrict__ scols, const double* __restrict__ tol_abs,
                                                  const int64_t* __restrict__ sbase, int64_t max_iters,
                                                  int32_t* __restrict__ gstop) {
    __shared__ int active;
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    if (gstop && *gstop) return;
    int mine = 0;
    for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
        if (sstop[s]) continue;
        double* R = Rall + (int64_t)s * (m + 1) * m;
        double* cs = csall + (int64_t)s * m;
        double* sn = snall + (int64_t)s * m;
        double* g = gall + (int64_t)s * (m + 1);
        const int64_t o = (int64_t)s * kBStride;
        for (int i = 0; i <= j; ++i) R[(int64_t)i * m + j] = h1[o + i] + h2[o + i];
        const double hnv = sqrt(fmax(hn[o], 0.0));
        for (int i = 0; i < j; ++i) {
            const double a = R[(int64_t)i * m + j], b = R[(int64_t)(i + 1) * m + j];
            R[(int64_t)i * m + j] = cs[i] * a + sn[i] * b;
            R[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
        }
        const double a = R[(int64_t)j * m + j];
        const double den = hypot(a, hnv);
        cs[j] = den > 0.0 ? a / den : 1.0;
        sn[j] = den > 0.0 ? hnv / den : 0.0;
        R[(int64_t)j * m + j] = den;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        scols[s] = j + 1;
        est[s] = fabs(g[j + 1]);
        if (!(fabs(g[j + 1]) > tol_abs[s]) || sbase[s] + j + 1 >= max_iters || j + 1 >= m) sstop[s] = 1;
        else mine = 1;
    }
    if (mine) atomicOr(&active, 1);
    __syncthreads();
    if (threadIdx.x == 0 && gstop) *gstop = active ? 0 : 1;
}

// y[sys] = R[sys]^{-1} g[sys] over its columns done
__global__ void k_btrisolve(int m, int nsys, const double* __restrict__ Rall, const double* __restrict__ gall,
                            double* __restrict__ yall, const int32_t* __restrict__ scols) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    const double* R = Rall + (int64_t)s * (m + 1) * m;
    const double* g = gall + (int64_t)s * (m + 1);
    double* y = yall + (int64_t)s * m;
    const int mm = scols[s];
    for (int i = mm - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < mm; ++k) t -= R[(int64_t)i * m + k] * y[k];
        y[i] = t / R[(int64_t)i * m + i];
    }
}

// out = sum_{i < cols[sys]} y[sys][i] V_i on every row (0 where cols = 0)
__global__ void k_bgemv(const double* __restrict__ V, int64_t ldv, BGeom g, const double* __restrict__ yall,
                        int m, const int32_t* __restrict__ scols, double* __restrict__ out) {
    for (int64_t ch = blockIdx.x; ch < g.nch; ch += gridDim.x) {
        const int sys = g.ch_sys[ch];
        const int nv = scols[sys];
        const double* y = yall + (int64_t)sys * m;
        const int64_t lo = g.ch_lo[ch], hi = lo + g.ch_len[ch];
        for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) {
            double acc = 0.0;
            for (int i = 0; i < nv; ++i) acc = fma(y[i], V[(int64_t)i * ldv + q], acc);
            out[q] = acc;
        }
    }
}

// cycle start: active systems get g = (||r_s||, 0, ...), the rest are masked
__global__ __launch_bounds__(1024) void k_bcycle_init(int nsys, int m, const double* __restrict__ nrm2,
                                                      const int32_t* __restrict__ act, double* __restrict__ gall,
                                                      int32_t* __restrict__ sstop, int32_t* __restrict__ scols,
                                                      int32_t* __restrict__ gstop) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int mine = 0;
    for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
        double* g = gall + (int64_t)s * (m + 1);
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = sqrt(nrm2[(int64_t)s * kBStride]);
        sstop[s] = act[s] ? 0 : 1;
        scols[s] = 0;
        mine |= act[s] ? 1 : 0;
    }
    if (mine) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0) *gstop = any ? 0 : 1;
}

inline unsigned grid_for(int64_t nch) { return (unsigned)(nch < 65536 ? nch : 65536); }

}  // namespace

void launch_bgs(int mode, const double* V, int64_t ldv, int nv, double* w, const BGeom& g, const double* c,
                double* partial, double* out, const int32_t* sstop, const int32_t* gstop, hipStream_t s) {
    if (g.nch <= 0) return;
    const unsigned grid = grid_for(g.nch);
    for (int base = 0; base < nv || (nv == 0 && base == 0); base += kMaxVec) {
        const int cnt = nv - base < kMaxVec ? nv - base : kMaxVec;
        const double* Vb = V + (int64_t)base * ldv;
        const int nout = mode == 2 ? 1 : cnt;
        const int nc = (cnt + 7) / 8;
#define PR_BGS(M, CC) \
    k_bgs<M, CC><<<grid, kThreads, 0, s>>>(Vb, ldv, cnt, w, g, (M) == 0 ? c : c + base, partial, sstop, gstop)
#define PR_BGS_NC(M)                \
    if (nc <= 1) PR_BGS(M, 1);      \
    else if (nc == 2) PR_BGS(M, 2); \
    else if (nc == 3) PR_BGS(M, 3); \
    else PR_BGS(M, 4)
        if (mode == 0) {
            PR_BGS_NC(0);
        } else if (mode == 1) {
            PR_BGS_NC(1);
        } else {
            PR_BGS_NC(2);
        }
#undef PR_BGS_NC
#undef PR_BGS
        const int64_t nt = (int64_t)g.nsys * nout;
        k_bgs_final<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(nout, g, partial, out, mode == 2 ? 0 : base,
                                                                 sstop, gstop);
        if (nv == 0) break;
    }
}

void launch_bscale(const double* src, double* dst, const BGeom& g, const double* denom, const int32_t* sstop,
                   const int32_t* gstop, hipStream_t s) {
    if (g.nch > 0) k_bscale<<<grid_for(g.nch), 256, 0, s>>>(src, dst, g, denom, sstop, gstop);
}

void launch_bgivens(int j, int m, int nsys, const double* h1, const double* h2, const double* hn, double* R,
                    double* cs, double* sn, double* gv, double* est, int32_t* sstop, int32_t* scols,
                    const double* tol_abs, const int64_t* sbase, int64_t max_iters, int32_t* gstop,
                    hipStream_t s) {
    k_bgivens<<<1, 1024, 0, s>>>(j, m, nsys, h1, h2, hn, R, cs, sn, gv, est, sstop, scols, tol_abs, sbase,
                                 max_iters, gstop);
}

void launch_btrisolve(int m, int nsys, const double* R, const double* gv, double* y, const int32_t* scols,
                      hipStream_t s) {
    k_btrisolve<<<(unsigned)((nsys + 63) / 64), 64, 0, s>>>(m, nsys, R, gv, y, scols);
}

void launch_bgemv(const double* V, int64_t ldv, const BGeom& g, const double* y, int m, const int32_t* scols,
                  double* out, hipStream_t s) {
    if (g.nch > 0) k_bgemv<<<grid_for(g.nch), 256, 0, s>>>(V, ldv, g, y, m, scols, out);
}

void launch_bcycle_init(int nsys, int m, const double* nrm2, const int32_t* active, double* gv, int32_t* sstop,
                        int32_t* scols, int32_t* gstop, hipStream_t s) {
    k_bcycle_init<<<1, 1024, 0, s>>>(nsys, m, nrm2, active, gv, sstop, scols, gstop);
}
