// Algorithm 2 (spectral clustering construction, Section 3.2) and its
// variants on the device: entrywise k-means (l1 distance to the cluster
// mean), spectral k-means (||I - A B^{-1}||_2 to the inverse of the mean),
// variance-minimising clustering (spectral distance, centre = the member
// nearest the mean) and bootstrapping (initial centres from Algorithm 1).
// Patches are clustered within their group (boundary key and size); each
// group runs its own passes until no assignment changes.
//
// Assignment of patch i: the spectral distance to every centre of its group
// is bracketed by [largest column norm of E, ||E||_F] with E = I - A_i X_j;
// only centres whose lower bound lies within the tie band of the smallest
// upper bound can be in the argmin's band.  When there are several such
// candidates their brackets are narrowed by repeated squaring of E^T E, and
// only the candidates still in the band get the exact largest singular
// value.  The band is
// {j : d_j <= d_min (1 + tie) + tie s_i}, s_i = 1 for the spectral distance
// and sum |A_i| for the l1 distance, so that distances at rounding level tie;
// the current centre is kept if it lies in the band, otherwise the lowest
// centre index in the band is taken.
#include "dense_dev.h"

#include <algorithm>
#include <climits>

namespace {

using namespace pr_dev;

// one wavefront per patch; centres of group g are [gc0[g], gc1[g])
__global__ __launch_bounds__(64, 2) void k_km_assign(int64_t n_p, const int64_t* __restrict__ ptr,
                                                  const double* __restrict__ tiles,
                                                  const int64_t* __restrict__ toff, int uniform_ps,
                                                  const int32_t* __restrict__ pg,
                                                  const int32_t* __restrict__ gc0,
                                                  const int32_t* __restrict__ gc1,
                                                  const int32_t* __restrict__ gactive, int crit,
                                                  const double* __restrict__ l1n,
                                                  const double* __restrict__ cen, int64_t stride,
                                                  double tie, int32_t* __restrict__ phi,
                                                  int32_t* __restrict__ gchanged,
                                                  double* __restrict__ lbscr, int64_t lbld,
                                                  unsigned long long* __restrict__ counters) {
    __shared__ double sA[kMaxPs * kMaxPs];
    __shared__ double sX[kMaxPs * kMaxPs];
    __shared__ double sE[kMaxPs * kMaxPs];
    const int lane = threadIdx.x;
    for (int64_t i = blockIdx.x; i < n_p; i += gridDim.x) {
        const int32_t g = pg[i];
        if (!gactive[g]) continue;
        const int p = (int)(ptr[i + 1] - ptr[i]);
        const int pp = p * p;
        const double* Ai = tiles + (uniform_ps ? i * (int64_t)uniform_ps * uniform_ps : toff[i]);
        lds_load(sA, Ai, pp, lane);
        __syncthreads();
        const int j0 = gc0[g], j1 = gc1[g];
        const double floor_abs = tie * (crit == PR_CRIT_L1 ? l1n[i] : 1.0);
        double* lb = lbscr + (int64_t)blockIdx.x * lbld;
        unsigned long long nev = 0, nex = 0, nsq = 0;
        double dmin, ubmin = INFINITY;
        if (crit == PR_CRIT_L1) {
            // entrywise: exact l1 distances; lb holds the distance itself
            dmin = INFINITY;
            for (int j = j0; j < j1; ++j) {
                const double* B = cen + (int64_t)j * stride;
                double acc = 0.0;
                for (int e = lane; e < pp; e += PR_WAVE) acc += fabs(sA[e] - B[e]);
                acc = wave_sum(acc);
                if (lane == 0) lb[j - j0] = acc;
                dmin = fmin(dmin, acc);
                ++nev;
            }
        } else {
            // pass 1: bracket every distance
            for (int j = j0; j < j1; ++j) {
                const double* X = cen + (int64_t)j * stride;
                lds_load(sX, X, pp, lane);
                __syncthreads();
                double lb2;
                const double fro2 = form_E(sA, sX, sE, p, lane, &lb2);
                __syncthreads();
                if (lane == 0) lb[j - j0] = sqrt(lb2);
                ubmin = fmin(ubmin, sqrt(fro2));
                __syncthreads();
                ++nev;
            }
            // pass 2: candidates of the tie band of the smallest upper bound.
            // Their brackets are narrowed by repeated squaring; a candidate
            // whose lower bound clears the band of the smallest narrowed
            // upper bound is out, and only several survivors need exact
            // values.
            double thr = (ubmin * (1.0 + tie) + floor_abs) * (1.0 + 1e-12);
            int ncand = 0;
            for (int j = j0; j < j1; ++j) ncand += (lb[j - j0] <= thr) ? 1 : 0;
            if (ncand > 1) {
                for (int j = j0; j < j1; ++j) {
                    if (!(lb[j - j0] <= thr)) continue;
                    const double* X = cen + (int64_t)j * stride;
                    lds_load(sX, X, pp, lane);
                    __syncthreads();
                    double lo2;
                    const double fro2 = form_E(sA, sX, sE, p, lane, &lo2);
                    __syncthreads();
                    double hi2 = fro2;
                    const double cut = thr;
                    // stop once this candidate is out of the current band
                    auto out = [cut](double lo, double) { return sqrt(lo) * (1.0 - 1e-12) > cut; };
                    sigma2_bracket(sE, sX, sE, p, lane, kSquarings, lo2, hi2, out);
                    ++nsq;
                    __syncthreads();
                    if (lane == 0) lb[j - j0] = sqrt(lo2) * (1.0 - 1e-12);
                    __syncthreads();
                    thr = fmin(thr, (sqrt(hi2) * (1.0 + 1e-12) * (1.0 + tie) + floor_abs) * (1.0 + 1e-12));
                }
                ncand = 0;
                for (int j = j0; j < j1; ++j) ncand += (lb[j - j0] <= thr) ? 1 : 0;
            }
            dmin = INFINITY;
            for (int j = j0; j < j1; ++j) {
                if (!(lb[j - j0] <= thr)) {
                    if (lane == 0) lb[j - j0] = INFINITY;      // outside the band for sure
                    continue;
                }
                double d;
                if (ncand == 1) {
                    d = 0.0;                                    // the only candidate is the argmin
                } else {
                    const double* X = cen + (int64_t)j * stride;
                    lds_load(sX, X, pp, lane);
                    __syncthreads();
                    form_E(sA, sX, sE, p, lane);
                    __syncthreads();
                    d = sqrt(sigma_max2_jacobi(sE, sX, p, lane));
                    __syncthreads();
                    ++nex;
                }
                if (lane == 0) lb[j - j0] = d;
                dmin = fmin(dmin, d);
            }
        }
        __syncthreads();
        // tie band, keep the current centre if it is in it
        const double lim = dmin * (1.0 + tie) + floor_abs;
        const int32_t cur = phi[i];
        int32_t pick = -1;
        bool keep = false;
        for (int j = j0; j < j1; ++j) {
            const bool inband = lb[j - j0] <= lim;
            if (inband && pick < 0) pick = j;
            if (inband && j == cur) keep = true;
        }
        if (lane == 0) {
            if (!keep) {
                phi[i] = pick;
                atomicAdd(&gchanged[g], 1);
            }
            atomicAdd(&counters[0], nev);
            if (nex) atomicAdd(&counters[1], nex);
            if (nsq) atomicAdd(&counters[3], nsq);
        }
        __syncthreads();
    }
}

// Centre update, one wavefront per centre j of an updating group.  Members
// (patches with phi == j) are mem[cptr[j] .. cptr[j+1]) in ascending id.
// mean: B_j = entrywise mean (Eq.(6)); medoid: B_j = the member nearest the
// mean (Frobenius), lowest id among those with squared distance at most
// delta_min (1 + tie) + tie^2 ||mean||_F^2.  Empty clusters keep B_j.
__global__ __launch_bounds__(64) void k_km_update(int64_t m_p, const int32_t* __restrict__ cgroup,
                                                  const int32_t* __restrict__ gupd,
                                                  const int64_t* __restrict__ cptr,
                                                  const int32_t* __restrict__ mem,
                                                  const int32_t* __restrict__ cps, int medoid,
                                                  const double* __restrict__ tiles,
                                                  const int64_t* __restrict__ toff, int uniform_ps,
                                                  double* __restrict__ B, int64_t stride,
                                                  int32_t* __restrict__ rep_patch, double tie,
                                                  unsigned long long* __restrict__ counters) {
    __shared__ double sM[kMaxPs * kMaxPs];
    const int lane = threadIdx.x;
    for (int64_t j = blockIdx.x; j < m_p; j += gridDim.x) {
        if (!gupd[cgroup[j]]) continue;
        const int64_t a = cptr[j], b = cptr[j + 1];
        if (a == b) {
            if (lane == 0) atomicAdd(&counters[2], 1ull);
            continue;
        }
        const int p = cps[j];
        const int pp = p * p;
        for (int e = lane; e < pp; e += PR_WAVE) {
            double s = 0.0;
            for (int64_t t = a; t < b; ++t) {
                const int32_t k = mem[t];
                s += tiles[(uniform_ps ? k * (int64_t)uniform_ps * uniform_ps : toff[k]) + e];
            }
            sM[e] = s / (double)(b - a);
        }
        __syncthreads();
        double* Bj = B + j * stride;
        if (!medoid) {
            for (int e = lane; e < pp; e += PR_WAVE) Bj[e] = sM[e];
            if (lane == 0) rep_patch[j] = -1;
        } else {
            double msq = 0.0;
            for (int e = lane; e < pp; e += PR_WAVE) msq += sM[e] * sM[e];
            msq = wave_sum(msq);
            double dmin = INFINITY;
            for (int64_t t = a; t < b; ++t) {
                const int32_t k = mem[t];
                const double* Ak = tiles + (uniform_ps ? k * (int64_t)uniform_ps * uniform_ps : toff[k]);
                double acc = 0.0;
                for (int e = lane; e < pp; e += PR_WAVE) {
                    const double v = Ak[e] - sM[e];
                    acc += v * v;
                }
                dmin = fmin(dmin, wave_sum(acc));
            }
            const double lim = dmin * (1.0 + tie) + tie * tie * msq;
            int32_t best = -1;
            for (int64_t t = a; t < b && best < 0; ++t) {
                const int32_t k = mem[t];
                const double* Ak = tiles + (uniform_ps ? k * (int64_t)uniform_ps * uniform_ps : toff[k]);
                double acc = 0.0;
                for (int e = lane; e < pp; e += PR_WAVE) {
                    const double v = Ak[e] - sM[e];
                    acc += v * v;
                }
                if (wave_sum(acc) <= lim) best = k;
            }
            const double* Ab = tiles + (uniform_ps ? best * (int64_t)uniform_ps * uniform_ps : toff[best]);
            for (int e = lane; e < pp; e += PR_WAVE) Bj[e] = Ab[e];
            if (lane == 0) rep_patch[j] = best;
        }
        __syncthreads();
    }
}

// B_j <- tile of patch rep[j]
__global__ void k_km_init(int64_t m_p, const int32_t* __restrict__ rep, const int64_t* __restrict__ ptr,
                          const double* __restrict__ tiles, const int64_t* __restrict__ toff,
                          int uniform_ps, double* __restrict__ B, int64_t stride) {
    for (int64_t j = blockIdx.x; j < m_p; j += gridDim.x) {
        const int32_t k = rep[j];
        const int p = (int)(ptr[k + 1] - ptr[k]);
        const double* A = tiles + (uniform_ps ? k * (int64_t)uniform_ps * uniform_ps : toff[k]);
        for (int e = threadIdx.x; e < p * p; e += blockDim.x) B[j * stride + e] = A[e];
    }
}

// sort key (centre, patch id) of every patch of an updating group
__global__ void k_km_keys(int64_t n_p, const int32_t* __restrict__ phi, const int32_t* __restrict__ pg,
                          const int32_t* __restrict__ gupd, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ vals, unsigned long long* __restrict__ ccount) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_p) return;
    const bool u = gupd[pg[i]] != 0;
    const uint32_t c = u ? (uint32_t)phi[i] : 0xFFFFFFFFu;
    keys[i] = ((uint64_t)c << 32) | (uint32_t)i;
    vals[i] = (int32_t)i;
    if (u) atomicAdd(&ccount[phi[i]], 1ull);
}

// group key of patch i: (size, boundary key) or size alone
__global__ void k_km_key1(int64_t n_p, const int64_t* __restrict__ ptr, const uint32_t* __restrict__ bkeys,
                          int partition, uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_p) return;
    const uint64_t p = (uint64_t)(ptr[i + 1] - ptr[i]);
    keys[i] = (p << 32) | (partition ? (uint64_t)bkeys[i] : 0ull);
    vals[i] = (int32_t)i;
}

// flag[t] = 1 where a new group starts in the sorted key sequence; flag[n] = 0
__global__ void k_km_flags(int64_t n, const uint64_t* __restrict__ keys, int64_t* __restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n) return;
    flag[t] = (t < n && (t == 0 || keys[t] != keys[t - 1])) ? 1 : 0;
}

// group index of every patch; gstart[g] (sorted position) and the size of group g
__global__ void k_km_gid(int64_t n, const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                         const int64_t* __restrict__ flag, const int64_t* __restrict__ excl,
                         int32_t* __restrict__ pg, int64_t* __restrict__ gstart, int32_t* __restrict__ gp) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t g = excl[t] + flag[t] - 1;
    pg[vals[t]] = (int32_t)g;
    if (flag[t]) {
        gstart[g] = t;
        gp[g] = (int32_t)(keys[t] >> 32);
    }
    if (t == n - 1) gstart[g + 1] = n;
}

// (group, patch id) keys: members of a group in ascending id after sorting
__global__ void k_km_key2(int64_t n_p, const int32_t* __restrict__ pg, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_p) return;
    keys[i] = ((uint64_t)(uint32_t)pg[i] << 32) | (uint32_t)i;
    vals[i] = (int32_t)i;
}

__global__ void k_gather_i32(int64_t n, const int32_t* __restrict__ src, const int64_t* __restrict__ idx,
                             int32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = src[idx[t]];
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int64_t km_assign_grid(int64_t n_p, int64_t lbld) {
    int64_t g = n_p < 16384 ? n_p : 16384;
    const int64_t cap = (int64_t)1 << 26;            // scratch of at most 512 MiB
    if (lbld > 0 && g * lbld > cap) g = std::max<int64_t>(1024, cap / lbld);
    return std::max<int64_t>(1, std::min<int64_t>(g, n_p));
}

void launch_km_assign(int64_t grid, int64_t n_p, const int64_t* ptr, const double* tiles, const int64_t* toff,
                      int uniform_ps, const int32_t* pg, const int32_t* gc0, const int32_t* gc1,
                      const int32_t* gactive, int crit, const double* l1n, const double* cen, int64_t stride,
                      double tie, int32_t* phi, int32_t* gchanged, double* lbscr, int64_t lbld,
                      unsigned long long* counters, hipStream_t s) {
    k_km_assign<<<(unsigned)grid, 64, 0, s>>>(n_p, ptr, tiles, toff, uniform_ps, pg, gc0, gc1, gactive, crit,
                                              l1n, cen, stride, tie, phi, gchanged, lbscr, lbld, counters);
}

void launch_km_update(int64_t m_p, const int32_t* cgroup, const int32_t* gupd, const int64_t* cptr,
                      const int32_t* mem, const int32_t* cps, int medoid, const double* tiles,
                      const int64_t* toff, int uniform_ps, double* B, int64_t stride, int32_t* rep_patch,
                      double tie, unsigned long long* counters, hipStream_t s) {
    const unsigned g = (unsigned)(m_p < 16384 ? m_p : 16384);
    k_km_update<<<g, 64, 0, s>>>(m_p, cgroup, gupd, cptr, mem, cps, medoid, tiles, toff, uniform_ps, B, stride,
                                 rep_patch, tie, counters);
}

void launch_km_init(int64_t m_p, const int32_t* rep, const int64_t* ptr, const double* tiles,
                    const int64_t* toff, int uniform_ps, double* B, int64_t stride, hipStream_t s) {
    const unsigned g = (unsigned)(m_p < 16384 ? m_p : 16384);
    k_km_init<<<g, 256, 0, s>>>(m_p, rep, ptr, tiles, toff, uniform_ps, B, stride);
}

void launch_km_keys(int64_t n_p, const int32_t* phi, const int32_t* pg, const int32_t* gupd, uint64_t* keys,
                    int32_t* vals, unsigned long long* ccount, hipStream_t s) {
    k_km_keys<<<nb(n_p, 256), 256, 0, s>>>(n_p, phi, pg, gupd, keys, vals, ccount);
}

void launch_km_key1(int64_t n_p, const int64_t* ptr, const uint32_t* bkeys, int partition, uint64_t* keys,
                    int32_t* vals, hipStream_t s) {
    k_km_key1<<<nb(n_p, 256), 256, 0, s>>>(n_p, ptr, bkeys, partition, keys, vals);
}

void launch_km_flags(int64_t n, const uint64_t* keys, int64_t* flag, hipStream_t s) {
    k_km_flags<<<nb(n + 1, 256), 256, 0, s>>>(n, keys, flag);
}

void launch_km_gid(int64_t n, const uint64_t* keys, const int32_t* vals, const int64_t* flag,
                   const int64_t* excl, int32_t* pg, int64_t* gstart, int32_t* gp, hipStream_t s) {
    k_km_gid<<<nb(n, 256), 256, 0, s>>>(n, keys, vals, flag, excl, pg, gstart, gp);
}

void launch_km_key2(int64_t n_p, const int32_t* pg, uint64_t* keys, int32_t* vals, hipStream_t s) {
    k_km_key2<<<nb(n_p, 256), 256, 0, s>>>(n_p, pg, keys, vals);
}

void launch_gather_i32(int64_t n, const int32_t* src, const int64_t* idx, int32_t* out, hipStream_t s) {
    if (n > 0) k_gather_i32<<<nb(n, 256), 256, 0, s>>>(n, src, idx, out);
}
