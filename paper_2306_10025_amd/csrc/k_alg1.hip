// Algorithm 1 (patch tolerance construction, Section 3.1) on the device.
//
// The sequential algorithm visits patches in order, compares each with the
// database entries in append order and keeps the first entry within eps, or
// appends the patch.  Pairs that cannot match are known in advance from a
// certified bound on a cheap per-patch key (the subset search suggested
// after Algorithm 1):
//   spectral: d(A,B) = ||(B-A)B^{-1}||_2 >= ||B-A||_2/||B||_2
//             >= | ||A||_F - ||B||_F | / (sqrt(p) ||B||_F),
//   l1 / Frobenius: d(A,B) >= | key(A) - key(B) | with key the same norm.
// Sorting patches by (size, key) and cutting wherever two neighbours are
// further apart than any match allows splits the patches into components
// that never match across.  Algorithm 1 restricted to one component gives
// exactly the sequential result for its patches (entries of other components
// never match them), so all components run their rounds at once:
//   round: the lowest unresolved member of each component becomes an entry;
//          it is inverted; every unresolved member is tested against it and
//          resolved on a match.
// When the rounds run long (one large component adds about one entry per
// round), every still unresolved patch is inverted in one batched launch and
// later rounds copy the new entries' inverses from that batch (the same
// elimination on the same tile, so the same bits, without a latency-bound
// single-matrix inversion per round) and open several entries per round
// (see the rounds of up to kA1Spec entries below).
// A member is thus compared with its component's entries in append order
// until the first match, as in the sequential algorithm.  Entries are
// finally numbered in ascending patch id (the append order).
#include "dense_dev.h"

#include <climits>

namespace {

using namespace pr_dev;

// ctl (int32[8]): [0] entries so far  [1] active components this round
//                 [2] done            [3] candidates this round
//                 [4] rounds started  [5] first singular entry patch + 1

// position s holds patch subset[s] (patch s without a subset)
__global__ void k_a1_keys(int64_t n_p, const int32_t* __restrict__ subset, const int64_t* __restrict__ ptr,
                          const double* __restrict__ keynorm, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ vals) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_p) return;
    const int32_t i = subset ? subset[s] : (int32_t)s;
    const uint64_t p = (uint64_t)(ptr[i + 1] - ptr[i]);
    const uint64_t bits = (uint64_t)__double_as_longlong(keynorm[i]);  // key >= 0: monotone
    keys[s] = (p << 58) | (bits >> 5);
    vals[s] = i;
}

__global__ void k_a1_comp_flags(int64_t n_p, const int32_t* __restrict__ sidx,
                                const int64_t* __restrict__ ptr, const double* __restrict__ keynorm,
                                int crit, double eps, int prune, int64_t* __restrict__ flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_p) return;
    if (s == n_p) {
        flag[s] = 0;
        return;
    }
    if (s == 0) {
        flag[s] = 1;
        return;
    }
    const int32_t i = sidx[s], j = sidx[s - 1];
    const int pi = (int)(ptr[i + 1] - ptr[i]), pj = (int)(ptr[j + 1] - ptr[j]);
    const double ks = keynorm[i], kp = keynorm[j];
    const double c = (pi * pi + 64) * 2.3e-16;
    const double half = (crit == PR_CRIT_SPECTRAL) ? (eps * sqrt((double)pi) * (1.0 + 1e-10) + c) * ks
                                                   : eps * (1.0 + 1e-10) + c * ks;
    flag[s] = (pi != pj || (prune && ks - kp > half)) ? 1 : 0;
}

__global__ void k_a1_key2(int64_t n_p, const int64_t* __restrict__ flag,
                          const int64_t* __restrict__ excl, const int32_t* __restrict__ sidx,
                          uint64_t* __restrict__ key2, int32_t* __restrict__ val2) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_p) return;
    const uint64_t comp = (uint64_t)(excl[s] + flag[s] - 1);
    key2[s] = (comp << 32) | (uint32_t)sidx[s];
    val2[s] = sidx[s];
}

__global__ void k_a1_cstart(int64_t n_p, int64_t n_comp, const uint64_t* __restrict__ key2,
                            int32_t* __restrict__ pos_comp, int32_t* __restrict__ cstart,
                            int32_t* __restrict__ next) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_p) return;
    const int32_t c = (int32_t)(key2[s] >> 32);
    pos_comp[s] = c;
    if (s == 0 || (int32_t)(key2[s - 1] >> 32) != c) {
        cstart[c] = (int32_t)s;
        next[c] = (int32_t)s;
    }
    if (s == 0) cstart[n_comp] = (int32_t)n_p;
}

__global__ void k_a1_begin(int32_t* ctl) {
    if (ctl[2]) return;
    if (ctl[4] > 0 && ctl[1] == 0) {
        ctl[2] = 1;
        return;
    }
    ctl[1] = 0;
    ctl[3] = 0;
    ctl[4] += 1;
}

// lowest unresolved member of each component becomes its next entry
__global__ void k_a1_pick(int64_t n_comp, int32_t* ctl, const int32_t* __restrict__ cstart,
                          int32_t* __restrict__ next, const int32_t* __restrict__ mem,
                          int32_t* __restrict__ status, int32_t* __restrict__ rep_slot,
                          int32_t* __restrict__ rep_patch, int32_t* __restrict__ slot_of_patch,
                          int32_t* __restrict__ repof, int32_t* __restrict__ active) {
    if (ctl[2]) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_comp) return;
    const int32_t s = next[c];
    if (s < cstart[c + 1]) {
        status[s] = 1;
        const int32_t pid = mem[s];
        const int32_t slot = atomicAdd(&ctl[0], 1);
        rep_slot[c] = slot;
        rep_patch[slot] = pid;
        slot_of_patch[pid] = slot;
        repof[pid] = pid;
        active[atomicAdd(&ctl[1], 1)] = (int32_t)c;
        next[c] = cstart[c + 1];      // lowered by the evaluation to the next unresolved member
    } else {
        rep_slot[c] = -1;
    }
}

template <int MAXP, int G>
__global__ __launch_bounds__(256) void k_a1_invert(const int32_t* ctl, const int32_t* __restrict__ active,
                                                   const int32_t* __restrict__ rep_slot,
                                                   const int32_t* __restrict__ rep_patch,
                                                   const int64_t* __restrict__ ptr,
                                                   const double* __restrict__ tiles,
                                                   const int64_t* __restrict__ toff, int uniform_ps,
                                                   double* __restrict__ dbt, int64_t stride,
                                                   int32_t* sing) {
    if (ctl[2]) return;
    const int na = ctl[1];
    const int64_t gsz = 256 / G;
    const int r = threadIdx.x % G;
    for (int64_t g = (int64_t)blockIdx.x * gsz + threadIdx.x / G; g < na; g += (int64_t)gridDim.x * gsz) {
        const int32_t c = active[g];
        const int32_t slot = rep_slot[c];
        const int32_t pid = rep_patch[slot];
        const int p = (int)(ptr[pid + 1] - ptr[pid]);
        const double* A = tiles + (uniform_ps ? (int64_t)pid * uniform_ps * uniform_ps : toff[pid]);
        const int inf = gj_invert<MAXP, G>(A, dbt + (int64_t)slot * stride, p, r);
        if (r == 0 && inf != 0) atomicCAS(sing, 0, pid + 1);
    }
}

// batched inversion of every unresolved position s (status 0) into
// inv + s * stride, with its zero-pivot report in info[s]
template <int MAXP, int G>
__global__ __launch_bounds__(256) void k_a1_preinvert(int64_t n_p, const int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ mem,
                                                      const int64_t* __restrict__ ptr,
                                                      const double* __restrict__ tiles,
                                                      const int64_t* __restrict__ toff, int uniform_ps,
                                                      double* __restrict__ inv, int64_t stride,
                                                      int32_t* __restrict__ info) {
    const int64_t gsz = 256 / G;
    const int r = threadIdx.x % G;
    for (int64_t s = (int64_t)blockIdx.x * gsz + threadIdx.x / G; s < n_p; s += (int64_t)gridDim.x * gsz) {
        if (status[s] != 0) continue;          // same s for the whole group
        const int32_t pid = mem[s];
        const int p = (int)(ptr[pid + 1] - ptr[pid]);
        const double* A = tiles + (uniform_ps ? (int64_t)pid * uniform_ps * uniform_ps : toff[pid]);
        const int inf = gj_invert<MAXP, G>(A, inv + s * stride, p, r);
        if (r == 0) info[s] = inf;
    }
}

// unresolved members of the components that opened an entry this round,
// with the indices the test needs ({patch, component, slot, entry patch}),
// so the evaluation does not walk that chain of loads one candidate at a time
__global__ void k_a1_filter(int64_t n_p, int32_t* ctl, const int32_t* __restrict__ status,
                            const int32_t* __restrict__ pos_comp, const int32_t* __restrict__ rep_slot,
                            const int32_t* __restrict__ mem, const int32_t* __restrict__ rep_patch,
                            int32_t* __restrict__ cand, int4* __restrict__ cinfo) {
    if (ctl[2]) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sc = s < n_p ? s : n_p - 1;
    const int32_t comp = pos_comp[sc];
    const int32_t slot = rep_slot[comp];
    const bool want = s < n_p && status[sc] == 0 && slot >= 0;
    const unsigned long long m = __ballot(want);
    if (m == 0) return;
    const int lane = threadIdx.x & (PR_WAVE - 1);
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&ctl[3], (int)__popcll(m));
    base = __shfl(base, leader);
    if (want) {
        const int q = base + (int)__popcll(m & ((1ull << lane) - 1ull));
        cand[q] = (int32_t)s;
        cinfo[q] = make_int4(mem[s], comp, slot, rep_patch[slot]);
    }
}

// One test d(A, B) < eps, wavefront-wide, with sA holding the patch tile and
// sX the entry (its inverse for the spectral criterion, else its tile),
// both loaded and synchronised.  The spectral value is bracketed by the
// column-norm bound and the Frobenius norm, then narrowed by repeated
// squaring, and only an undecided pair takes the exact singular value; a
// decision counts only when it clears eps^2 by a rounding margin.  sE is
// scratch; the bracket and the exact value also use sA and sX as scratch
// and then set clobbered.
__device__ bool a1_match(int crit, double eps, double* sA, double* sX, double* sE, int p, int lane,
                         unsigned long long& nex, unsigned long long& nsq, bool& clobbered) {
    if (crit == PR_CRIT_SPECTRAL) {
        double lb2;
        const double fro2 = form_E(sA, sX, sE, p, lane, &lb2);
        __syncthreads();
        const double e2 = eps * eps;
        auto decided = [e2](double lo, double hi) {
            return hi * (1.0 + 1e-11) < e2 || lo * (1.0 - 1e-11) >= e2;
        };
        double lo = lb2, hi = fro2;   // largest column norm^2 <= sigma_max^2 <= ||E||_F^2
        if (!decided(lo, hi)) {
            __syncthreads();
            sigma2_bracket(sE, sA, sX, p, lane, kSquarings, lo, hi, decided);
            ++nsq;
            clobbered = true;
        }
        if (decided(lo, hi)) return hi * (1.0 + 1e-11) < e2;
        __syncthreads();
        ++nex;
        clobbered = true;
        return sqrt(sigma_max2_jacobi(sE, sA, p, lane)) < eps;
    }
    double acc = 0.0;
    for (int e = lane; e < p * p; e += PR_WAVE) {
        const double v = sA[e] - sX[e];
        acc += (crit == PR_CRIT_L1) ? fabs(v) : v * v;
    }
    acc = wave_sum(acc);
    return ((crit == PR_CRIT_L1) ? acc : sqrt(acc)) < eps;
}

__device__ __forceinline__ const double* a1_tile(const double* tiles, const int64_t* toff, int uniform_ps,
                                                 int32_t i) {
    return tiles + (uniform_ps ? (int64_t)i * uniform_ps * uniform_ps : toff[i]);
}

// one wavefront per candidate: test against its component's current entry.
// The three p x p work tiles are dynamic LDS of pm^2 doubles each (pm: the
// largest patch size), so small patches leave room for more resident waves.
__global__ __launch_bounds__(64) void k_a1_eval(const int32_t* ctl, int crit, double eps, int pm,
                                                const int32_t* __restrict__ cand,
                                                const int4* __restrict__ cinfo,
                                                const int64_t* __restrict__ ptr,
                                                const double* __restrict__ tiles,
                                                const int64_t* __restrict__ toff, int uniform_ps,
                                                const double* __restrict__ dbt, int64_t stride,
                                                int32_t* __restrict__ status, int32_t* __restrict__ repof,
                                                int32_t* __restrict__ next,
                                                unsigned long long* __restrict__ counters) {
    if (ctl[2]) return;
    const int nc = ctl[3];
    if ((int)blockIdx.x >= nc) return;
    extern __shared__ double s_dyn[];
    double* sA = s_dyn;
    double* sX = s_dyn + pm * pm;
    double* sE = s_dyn + 2 * pm * pm;
    const int lane = threadIdx.x;
    unsigned long long nev = 0, nex = 0, nsq = 0;
    for (int q = blockIdx.x; q < nc; q += gridDim.x) {
        const int32_t s = cand[q];
        const int4 ci = cinfo[q];
        const int32_t i = ci.x, comp = ci.y, slot = ci.z, r = ci.w;
        const int p = (int)(ptr[i + 1] - ptr[i]);
        const int pp = p * p;
        const double* Br = (crit == PR_CRIT_SPECTRAL) ? dbt + (int64_t)slot * stride
                                                      : a1_tile(tiles, toff, uniform_ps, r);
        lds_load(sA, a1_tile(tiles, toff, uniform_ps, i), pp, lane);
        lds_load(sX, Br, pp, lane);
        __syncthreads();
        ++nev;
        bool clob = false;
        const bool match = a1_match(crit, eps, sA, sX, sE, p, lane, nex, nsq, clob);
        if (lane == 0) {
            if (match) {
                status[s] = 1;
                repof[i] = r;
            } else {
                atomicMin(&next[comp], s);
            }
        }
        __syncthreads();
    }
    if (lane == 0) {
        atomicAdd(&counters[0], nev);
        if (nex) atomicAdd(&counters[1], nex);
        if (nsq) atomicAdd(&counters[3], nsq);
    }
}

// ---- rounds of up to kA1Spec entries (after the batched inversion) ---------
// The kA1Spec lowest unresolved members u_0 < u_1 < ... of a component are
// taken together.  u_0 is the next entry for sure; u_j is an entry exactly
// when no entry among u_0..u_{j-1} matches it, and otherwise belongs to the
// first that does (every earlier entry of the component was already tested
// against it).  All pairs (u_i, u_j), i < j, are tested in parallel, one
// thread settles the chain in order, and the remaining members are then
// tested against the round's entries in append order, up to the first
// match: the sequential algorithm's result, in about kA1Spec times fewer
// rounds.  Only the tests the sequential algorithm makes are counted as
// evaluations (the pair tests past a member's first match are not).

// the speculative members of each component (positions in order), scanned
// from its lowest unresolved position over at most kA1SpecWindow positions,
// 64 at a time by one wavefront per component
__global__ __launch_bounds__(64) void k_a1s_pick(int64_t n_comp, int32_t* ctl, const int32_t* __restrict__ cstart,
                                                 int32_t* __restrict__ next, const int32_t* __restrict__ status,
                                                 int32_t* __restrict__ spec, int32_t* __restrict__ spec_n,
                                                 int32_t* __restrict__ pairm, int32_t* __restrict__ rep_slot,
                                                 int32_t* __restrict__ active) {
    if (ctl[2]) return;
    const int lane = threadIdx.x;
    for (int64_t c = blockIdx.x; c < n_comp; c += gridDim.x) {
        const int32_t s0 = next[c], end = cstart[c + 1];
        const int32_t lim = (end - s0 > kA1SpecWindow) ? s0 + kA1SpecWindow : end;
        int n = 0;
        for (int32_t b = s0; b < lim && n < kA1Spec; b += PR_WAVE) {
            const int32_t sp = b + lane;
            const int32_t st = status[sp < lim ? sp : s0];        // clamped: s0 < lim here
            const bool un = sp < lim && st == 0;
            const unsigned long long m = __ballot(un);
            const int rank = n + (int)__popcll(m & ((1ull << lane) - 1ull));
            if (un && rank < kA1Spec) {
                spec[c * kA1Spec + rank] = sp;
                pairm[c * kA1Spec + rank] = 0;
            }
            n += (int)__popcll(m);
        }
        if (n > kA1Spec) n = kA1Spec;
        if (lane == 0) {
            rep_slot[c] = -1;
            spec_n[c] = n;
            if (n > 0) {
                active[atomicAdd(&ctl[1], 1)] = (int32_t)c;
                next[c] = end;  // lowered by the evaluation to the next unresolved member
            }
        }
    }
}

// all pairs (u_i, u_j), i < j, of the active components: bit i of
// pairm[c][j] is set when u_i's entry test matches u_j
__global__ __launch_bounds__(64) void k_a1s_pairs(const int32_t* ctl, int crit, double eps, int pm,
                                                  const int32_t* __restrict__ active,
                                                  const int32_t* __restrict__ spec,
                                                  const int32_t* __restrict__ spec_n,
                                                  const int32_t* __restrict__ mem,
                                                  const int64_t* __restrict__ ptr,
                                                  const double* __restrict__ tiles,
                                                  const int64_t* __restrict__ toff, int uniform_ps,
                                                  const double* __restrict__ inv, int64_t stride,
                                                  int32_t* __restrict__ pairm,
                                                  unsigned long long* __restrict__ counters) {
    if (ctl[2]) return;
    constexpr int NP = kA1Spec * (kA1Spec - 1) / 2;
    const int64_t work = (int64_t)ctl[1] * NP;
    extern __shared__ double s_dyn[];
    double* sA = s_dyn;
    double* sX = s_dyn + pm * pm;
    double* sE = s_dyn + 2 * pm * pm;
    const int lane = threadIdx.x;
    unsigned long long nex = 0, nsq = 0;
    for (int64_t w = blockIdx.x; w < work; w += gridDim.x) {
        const int32_t c = active[w / NP];
        int pr = (int)(w % NP), j = 1;
        while (pr >= j) {        // pairs in the order (0,1), (0,2), (1,2), (0,3), ...
            pr -= j;
            ++j;
        }
        const int i = pr;
        if (j >= spec_n[c]) continue;
        const int32_t ui = spec[c * kA1Spec + i], uj = spec[c * kA1Spec + j];
        const int32_t pj = mem[uj];
        const int p = (int)(ptr[pj + 1] - ptr[pj]);
        const double* Br = (crit == PR_CRIT_SPECTRAL) ? inv + (int64_t)ui * stride
                                                      : a1_tile(tiles, toff, uniform_ps, mem[ui]);
        lds_load(sA, a1_tile(tiles, toff, uniform_ps, pj), p * p, lane);
        lds_load(sX, Br, p * p, lane);
        __syncthreads();
        bool clob = false;
        const bool match = a1_match(crit, eps, sA, sX, sE, p, lane, nex, nsq, clob);
        if (lane == 0 && match) atomicOr(&pairm[c * kA1Spec + j], 1 << i);
        __syncthreads();
    }
    if (lane == 0) {
        if (nex) atomicAdd(&counters[1], nex);
        if (nsq) atomicAdd(&counters[3], nsq);
    }
}

// one thread per active component settles its speculative members in order
__global__ void k_a1s_resolve(int32_t* ctl, const int32_t* __restrict__ active,
                              const int32_t* __restrict__ spec, const int32_t* __restrict__ spec_n,
                              const int32_t* __restrict__ pairm, const int32_t* __restrict__ mem,
                              const int32_t* __restrict__ inv_info,
                              int32_t* __restrict__ status, int32_t* __restrict__ repof,
                              int32_t* __restrict__ rep_slot, int32_t* __restrict__ rep_patch,
                              int32_t* __restrict__ slot_of_patch, int32_t* __restrict__ ent,
                              int32_t* __restrict__ ent_n, int32_t* __restrict__ ent_slot,
                              unsigned long long* __restrict__ counters) {
    if (ctl[2]) return;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ctl[1]) return;
    const int32_t c = active[g];
    const int n = spec_n[c];
    unsigned emask = 0;          // bit j: u_j is an entry
    int m = 0;
    unsigned long long nev = 0;
    for (int j = 0; j < n; ++j) {
        const int32_t u = spec[c * kA1Spec + j];
        const int32_t pid = mem[u];
        const unsigned bits = (unsigned)pairm[c * kA1Spec + j];
        int hit = -1;
        for (int e = 0; e < j; ++e) {
            if (!((emask >> e) & 1u)) continue;
            ++nev;
            if ((bits >> e) & 1u) {
                hit = e;
                break;
            }
        }
        status[u] = 1;
        if (hit >= 0) {
            repof[pid] = mem[spec[c * kA1Spec + hit]];
        } else {
            const int32_t slot = atomicAdd(&ctl[0], 1);
            rep_patch[slot] = pid;
            slot_of_patch[pid] = slot;
            repof[pid] = pid;
            ent[c * kA1Spec + m] = u;
            ent_slot[c * kA1Spec + m] = slot;
            ++m;
            emask |= 1u << j;
            if (inv_info[u] != 0) atomicCAS(&ctl[5], 0, pid + 1);
        }
    }
    ent_n[c] = m;
    rep_slot[c] = ent_slot[c * kA1Spec];      // m >= 1: u_0 is always an entry
    if (nev) atomicAdd(&counters[0], nev);
}

// the round's entries' inverses, copied from the batch to their slots
__global__ __launch_bounds__(64) void k_a1s_take(const int32_t* ctl, const int32_t* __restrict__ active,
                                                 const int32_t* __restrict__ ent,
                                                 const int32_t* __restrict__ ent_n,
                                                 const int32_t* __restrict__ ent_slot,
                                                 const int32_t* __restrict__ mem,
                                                 const int64_t* __restrict__ ptr,
                                                 const double* __restrict__ inv, double* __restrict__ dbt,
                                                 int64_t stride) {
    if (ctl[2]) return;
    const int64_t work = (int64_t)ctl[1] * kA1Spec;
    for (int64_t w = blockIdx.x; w < work; w += gridDim.x) {
        const int32_t c = active[w / kA1Spec];
        const int m = (int)(w % kA1Spec);
        if (m >= ent_n[c]) continue;
        const int32_t u = ent[c * kA1Spec + m];
        const int32_t pid = mem[u];
        const int p = (int)(ptr[pid + 1] - ptr[pid]);
        const double* src = inv + (int64_t)u * stride;
        double* dst = dbt + (int64_t)ent_slot[c * kA1Spec + m] * stride;
        for (int e = threadIdx.x; e < p * p; e += 64) dst[e] = src[e];
    }
}

// one wavefront per remaining member: tested against the round's entries of
// its component in append order, up to the first match
__global__ __launch_bounds__(64, 2) void k_a1s_eval(const int32_t* ctl, int crit, double eps, int pm,
                                                 const int32_t* __restrict__ cand,
                                                 const int4* __restrict__ cinfo,
                                                 const int64_t* __restrict__ ptr,
                                                 const double* __restrict__ tiles,
                                                 const int64_t* __restrict__ toff, int uniform_ps,
                                                 const double* __restrict__ inv, int64_t stride,
                                                 const int32_t* __restrict__ ent,
                                                 const int32_t* __restrict__ ent_n,
                                                 const int32_t* __restrict__ mem,
                                                 int32_t* __restrict__ status, int32_t* __restrict__ repof,
                                                 int32_t* __restrict__ next,
                                                 unsigned long long* __restrict__ counters) {
    if (ctl[2]) return;
    const int nc = ctl[3];
    if ((int)blockIdx.x >= nc) return;
    extern __shared__ double s_dyn[];
    double* sA = s_dyn;
    double* sX = s_dyn + pm * pm;
    double* sE = s_dyn + 2 * pm * pm;
    const int lane = threadIdx.x;
    unsigned long long nev = 0, nex = 0, nsq = 0;
    for (int q = blockIdx.x; q < nc; q += gridDim.x) {
        const int32_t s = cand[q];
        const int4 ci = cinfo[q];
        const int32_t i = ci.x, comp = ci.y;
        const int p = (int)(ptr[i + 1] - ptr[i]);
        const int pp = p * p;
        const double* Ai = a1_tile(tiles, toff, uniform_ps, i);
        const int n = ent_n[comp];
        int32_t hit = -1;
        bool clob = true;
        for (int m = 0; m < n; ++m) {
            const int32_t u = ent[comp * kA1Spec + m];
            const double* Br = (crit == PR_CRIT_SPECTRAL) ? inv + (int64_t)u * stride
                                                          : a1_tile(tiles, toff, uniform_ps, mem[u]);
            if (clob) lds_load(sA, Ai, pp, lane);
            lds_load(sX, Br, pp, lane);
            __syncthreads();
            ++nev;
            clob = false;
            const bool match = a1_match(crit, eps, sA, sX, sE, p, lane, nex, nsq, clob);
            __syncthreads();
            if (match) {
                hit = mem[u];
                break;
            }
        }
        if (lane == 0) {
            if (hit >= 0) {
                status[s] = 1;
                repof[i] = hit;
            } else {
                atomicMin(&next[comp], s);
            }
        }
        __syncthreads();
    }
    if (lane == 0) {
        atomicAdd(&counters[0], nev);
        if (nex) atomicAdd(&counters[1], nex);
        if (nsq) atomicAdd(&counters[3], nsq);
    }
}

__global__ void k_a1_repflags(int64_t n_p, const int32_t* __restrict__ repof, int64_t* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_p) f[i] = (repof[i] == (int32_t)i) ? 1 : 0;
    else if (i == n_p) f[i] = 0;
}

__global__ void k_a1_finish(int64_t n_p, const int32_t* __restrict__ repof,
                            const int64_t* __restrict__ rank, int32_t* __restrict__ phi,
                            int32_t* __restrict__ reps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_p) return;
    const int32_t r = repof[i];
    phi[i] = (int32_t)rank[r];
    if (r == (int32_t)i) reps[rank[i]] = (int32_t)i;
}

// subset form of the numbering: entries of the subset in ascending patch id
__global__ void k_a1_subflags(int64_t ns, const int32_t* __restrict__ subset, const int32_t* __restrict__ repof,
                              int64_t* __restrict__ f) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns) f[s] = (repof[subset[s]] == subset[s]) ? 1 : 0;
    else if (s == ns) f[s] = 0;
}

__global__ void k_a1_subrank(int64_t ns, const int32_t* __restrict__ subset, const int64_t* __restrict__ f,
                             const int64_t* __restrict__ rank, int32_t base, int32_t* __restrict__ entries,
                             int32_t* __restrict__ rank_of_patch) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns || !f[s]) return;
    entries[rank[s]] = subset[s];
    rank_of_patch[subset[s]] = base + (int32_t)rank[s];
}

// entry j (ascending patch id) <- its temporary slot
__global__ void k_a1_copy_db(int64_t m_p, const int32_t* __restrict__ reps,
                             const int32_t* __restrict__ slot_of_patch, const int64_t* __restrict__ ptr,
                             const double* __restrict__ dbt, double* __restrict__ db, int64_t stride) {
    for (int64_t j = blockIdx.x; j < m_p; j += gridDim.x) {
        const int32_t pid = reps[j];
        const int p = (int)(ptr[pid + 1] - ptr[pid]);
        const double* src = dbt + (int64_t)slot_of_patch[pid] * stride;
        for (int e = threadIdx.x; e < p * p; e += blockDim.x) db[j * stride + e] = src[e];
    }
}

// ---------------------------------------------------------------------------
// Closest matching (the variant proposed in the remarks after Algorithm 1):
// the database is Algorithm 1's (a patch becomes an entry exactly when no
// earlier entry lies within eps, whichever would match), and every other
// patch i is mapped to the closest of the entries within eps that exist when
// i is visited, i.e. entries j < rank[i] (entries are numbered in ascending
// patch id).  Equal distances: the entries with d_j < eps and
// d_j <= d_min (1 + tie) + tie s_i tie (s_i = 1 spectral, sum |A_i| for l1,
// ||A_i||_F for Frobenius); the lowest index among them wins.
//
// One wavefront per patch.  Entries of another size, and entries whose key
// (Frobenius or l1 norm) rules out d < eps by the certified bound of the
// file header, are skipped by a lane-parallel filter.  Spectral distances
// are bracketed first ([largest column norm of E, ||E||_F]); only entries
// that may lie in the band of the smallest certain match are narrowed by
// repeated squaring, and only several survivors get exact values (cyclic
// Jacobi), as in the clustering assignment.
// ---------------------------------------------------------------------------
__global__ void k_a1_entry_keys(int64_t m_p, const int32_t* __restrict__ reps, const int64_t* __restrict__ ptr,
                                const double* __restrict__ keynorm, double* __restrict__ ekey,
                                int32_t* __restrict__ esz) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m_p) return;
    const int32_t r = reps[j];
    ekey[j] = keynorm[r];
    esz[j] = (int32_t)(ptr[r + 1] - ptr[r]);
}

__global__ __launch_bounds__(64, 2) void k_a1_closest(
    int64_t n_p, const int64_t* __restrict__ ptr, const double* __restrict__ tiles,
    const int64_t* __restrict__ toff, int ups, const int32_t* __restrict__ reps,
    const int64_t* __restrict__ rank, const double* __restrict__ ekey, const int32_t* __restrict__ esz,
    const double* __restrict__ db, int64_t stride, int crit, double eps, double tie,
    const double* __restrict__ keynorm, int32_t* __restrict__ phi, double* __restrict__ lbscr, int64_t lbld,
    unsigned long long* __restrict__ counters) {
    __shared__ double sA[kMaxPs * kMaxPs];
    __shared__ double sX[kMaxPs * kMaxPs];
    __shared__ double sE[kMaxPs * kMaxPs];
    const int lane = threadIdx.x;
    double* lb = lbscr + (int64_t)blockIdx.x * lbld;
    unsigned long long nev = 0, nex = 0, nsq = 0;
    for (int64_t i = blockIdx.x; i < n_p; i += gridDim.x) {
        const int32_t cur = phi[i];
        if (reps[cur] == (int32_t)i) continue;            // an entry keeps itself
        const int p = (int)(ptr[i + 1] - ptr[i]);
        const int pp = p * p;
        const int64_t J = rank[i];                        // entries that exist when i is visited
        const double* Ai = tiles + (ups ? i * (int64_t)ups * ups : toff[i]);
        const double ki = keynorm[i];
        const double floor_abs = tie * (crit == PR_CRIT_SPECTRAL ? 1.0 : ki);
        const double c = (p * p + 64) * 2.3e-16;
        lds_load(sA, Ai, pp, lane);
        __syncthreads();
        // filter: same size and a key compatible with d < eps; lb = INF elsewhere
        for (int64_t jb = 0; jb < J; jb += PR_WAVE) {
            const int64_t j = jb + lane;
            bool ok = false;
            if (j < J) {
                const double kj = ekey[j];
                const double half = (crit == PR_CRIT_SPECTRAL)
                                        ? (eps * sqrt((double)p) * (1.0 + 1e-10) + c) * fmax(ki, kj)
                                        : eps * (1.0 + 1e-10) + c * fmax(ki, kj);
                ok = esz[j] == p && fabs(ki - kj) <= half;
                lb[j] = ok ? 0.0 : INFINITY;
            }
        }
        __syncthreads();
        double ubmin = INFINITY;                         // least upper bound of a certain match
        // pass 1: exact l1 / Frobenius distances, or the spectral bracket
        for (int64_t jb = 0; jb < J; jb += PR_WAVE) {
            const int64_t jl = jb + lane;
            unsigned long long mask = __ballot(jl < J && lb[jl] == 0.0);
            while (mask) {
                const int64_t j = jb + __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                double v;
                if (crit == PR_CRIT_SPECTRAL) {
                    lds_load(sX, db + j * stride, pp, lane);
                    __syncthreads();
                    double lb2;
                    const double fro2 = form_E(sA, sX, sE, p, lane, &lb2);
                    __syncthreads();
                    const double lo = sqrt(lb2) * (1.0 - 1e-12), hi = sqrt(fro2) * (1.0 + 1e-12);
                    v = lo < eps ? lo : INFINITY;
                    if (hi < eps) ubmin = fmin(ubmin, hi);
                } else {
                    const int32_t r = reps[j];
                    const double* B = tiles + (ups ? (int64_t)r * ups * ups : toff[r]);
                    double acc = 0.0;
                    for (int e = lane; e < pp; e += PR_WAVE) {
                        const double t = sA[e] - B[e];
                        acc += (crit == PR_CRIT_L1) ? fabs(t) : t * t;
                    }
                    acc = wave_sum(acc);
                    if (crit == PR_CRIT_FRO) acc = sqrt(acc);
                    v = acc < eps ? acc : INFINITY;
                }
                ++nev;
                if (lane == 0) lb[j] = v;
            }
        }
        __syncthreads();
        if (crit == PR_CRIT_SPECTRAL) {
            // the closest match has d <= ubmin (a certain match) or d < eps
            double thr = (fmin(ubmin, eps) * (1.0 + tie) + floor_abs) * (1.0 + 1e-12);
            int ncand = 0;
            for (int64_t jb = 0; jb < J; jb += PR_WAVE) {
                const int64_t jl = jb + lane;
                ncand += __popcll(__ballot(jl < J && lb[jl] <= thr));
            }
            if (ncand > 1) {
                for (int64_t jb = 0; jb < J; jb += PR_WAVE) {
                    const int64_t jl = jb + lane;
                    unsigned long long mask = __ballot(jl < J && lb[jl] <= thr);
                    while (mask) {
                        const int64_t j = jb + __ffsll((long long)mask) - 1;
                        mask &= mask - 1;
                        lds_load(sX, db + j * stride, pp, lane);
                        __syncthreads();
                        double lo2;
                        double hi2 = form_E(sA, sX, sE, p, lane, &lo2);
                        __syncthreads();
                        const double cut = thr;
                        auto done = [cut, eps](double lo, double) {
                            const double l = sqrt(lo) * (1.0 - 1e-12);
                            return l > cut || l >= eps;
                        };
                        sigma2_bracket(sE, sX, sE, p, lane, kSquarings, lo2, hi2, done);
                        ++nsq;
                        __syncthreads();
                        const double lo = sqrt(lo2) * (1.0 - 1e-12), hi = sqrt(hi2) * (1.0 + 1e-12);
                        if (lane == 0) lb[j] = lo < eps ? lo : INFINITY;
                        if (hi < eps) thr = fmin(thr, (hi * (1.0 + tie) + floor_abs) * (1.0 + 1e-12));
                        __syncthreads();
                    }
                }
                ncand = 0;
                for (int64_t jb = 0; jb < J; jb += PR_WAVE) {
                    const int64_t jl = jb + lane;
                    ncand += __popcll(__ballot(jl < J && lb[jl] <= thr));
                }
            }
            // survivors: the only one is the closest match; several get exact values
            for (int64_t jb = 0; jb < J; jb += PR_WAVE) {
                const int64_t jl = jb + lane;
                const bool in = jl < J && lb[jl] <= thr;
                if (jl < J && !in) lb[jl] = INFINITY;
                unsigned long long mask = __ballot(in);
                __syncthreads();
                while (mask) {
                    const int64_t j = jb + __ffsll((long long)mask) - 1;
                    mask &= mask - 1;
                    double d = 0.0;
                    if (ncand > 1) {
                        lds_load(sX, db + j * stride, pp, lane);
                        __syncthreads();
                        form_E(sA, sX, sE, p, lane);
                        __syncthreads();
                        d = sqrt(sigma_max2_jacobi(sE, sX, p, lane));
                        __syncthreads();
                        ++nex;
                    }
                    if (lane == 0) lb[j] = d < eps ? d : INFINITY;
                }
            }
            __syncthreads();
        }
        // band around the least distance; lowest entry index in it
        double dmin = INFINITY;
        for (int64_t jb = 0; jb < J; jb += PR_WAVE) {
            const int64_t jl = jb + lane;
            dmin = fmin(dmin, jl < J ? lb[jl] : INFINITY);
        }
        dmin = -wave_max(-dmin);
        const double lim = dmin * (1.0 + tie) + floor_abs;
        int64_t pick = -1;
        for (int64_t jb = 0; jb < J && pick < 0; jb += PR_WAVE) {
            const int64_t jl = jb + lane;
            const unsigned long long mask = __ballot(jl < J && lb[jl] <= lim);
            if (mask) pick = jb + __ffsll((long long)mask) - 1;
        }
        if (lane == 0 && pick >= 0 && dmin < eps) phi[i] = (int32_t)pick;
        __syncthreads();
    }
    if (lane == 0) {
        atomicAdd(&counters[0], nev);
        if (nex) atomicAdd(&counters[1], nex);
        if (nsq) atomicAdd(&counters[3], nsq);
    }
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <int MAXP, int G>
void run_a1_invert(int64_t n_comp, const int32_t* ctl, const int32_t* active, const int32_t* rep_slot,
                   const int32_t* rep_patch, const int64_t* ptr, const double* tiles, const int64_t* toff,
                   int uniform_ps, double* dbt, int64_t stride, int32_t* sing, hipStream_t s) {
    const int per = 256 / G;
    int64_t blocks = (n_comp + per - 1) / per;
    if (blocks > 4096) blocks = 4096;
    k_a1_invert<MAXP, G><<<(unsigned)blocks, 256, 0, s>>>(ctl, active, rep_slot, rep_patch, ptr, tiles,
                                                         toff, uniform_ps, dbt, stride, sing);
}

template <int MAXP, int G>
void run_a1_preinvert(const A1Dev& d, hipStream_t s) {
    const int per = 256 / G;
    int64_t blocks = (d.n_p + per - 1) / per;
    if (blocks > 65536) blocks = 65536;
    k_a1_preinvert<MAXP, G><<<(unsigned)blocks, 256, 0, s>>>(d.n_p, d.status, d.mem, d.ptr, d.tiles, d.toff,
                                                            d.uniform_ps, d.inv, d.stride, d.inv_info);
}

}  // namespace

void launch_a1_keys(int64_t n_p, const int32_t* subset, const int64_t* ptr, const double* keynorm,
                    uint64_t* keys, int32_t* vals, hipStream_t s) {
    k_a1_keys<<<nb(n_p, 256), 256, 0, s>>>(n_p, subset, ptr, keynorm, keys, vals);
}

void launch_a1_subset_entries(int64_t ns, const int32_t* subset, const int32_t* repof, int64_t* flags,
                              int64_t* rank, int64_t* scr, int32_t base, int32_t* entries,
                              int32_t* rank_of_patch, hipStream_t s) {
    k_a1_subflags<<<nb(ns + 1, 256), 256, 0, s>>>(ns, subset, repof, flags);
    launch_exclusive_scan_i64(flags, rank, ns + 1, scr, s);
    k_a1_subrank<<<nb(ns, 256), 256, 0, s>>>(ns, subset, flags, rank, base, entries, rank_of_patch);
}

void launch_a1_comp_flags(int64_t n_p, const int32_t* sidx, const int64_t* ptr, const double* keynorm,
                          int crit, double eps, int prune, int64_t* flag, hipStream_t s) {
    k_a1_comp_flags<<<nb(n_p + 1, 256), 256, 0, s>>>(n_p, sidx, ptr, keynorm, crit, eps, prune, flag);
}

void launch_a1_key2(int64_t n_p, const int64_t* flag, const int64_t* excl, const int32_t* sidx,
                    uint64_t* key2, int32_t* val2, hipStream_t s) {
    k_a1_key2<<<nb(n_p, 256), 256, 0, s>>>(n_p, flag, excl, sidx, key2, val2);
}

void launch_a1_cstart(int64_t n_p, int64_t n_comp, const uint64_t* key2, int32_t* pos_comp,
                      int32_t* cstart, int32_t* next, hipStream_t s) {
    k_a1_cstart<<<nb(n_p, 256), 256, 0, s>>>(n_p, n_comp, key2, pos_comp, cstart, next);
}

// The template choice is the one the rounds use, so that an inverse is the
// same whether it was taken in a round or in the batch.
void launch_a1_preinvert(const A1Dev& d, int max_ps, hipStream_t s) {
    if (d.n_p <= 0 || !d.inv || !d.inv_info) return;
    if (max_ps <= 4) run_a1_preinvert<4, 4>(d, s);
    else if (max_ps <= 12) run_a1_preinvert<12, 16>(d, s);
    else if (max_ps <= 16) run_a1_preinvert<16, 16>(d, s);
    else if (max_ps <= 24) run_a1_preinvert<24, 32>(d, s);
    else run_a1_preinvert<32, 32>(d, s);
}

void launch_a1_rounds(int rounds, const A1Dev& d, int crit, double eps, int max_ps, hipStream_t s) {
    const unsigned cb = nb(d.n_comp, 256);
    const unsigned fb = nb(d.n_p, 256);
    const unsigned eb = (unsigned)(d.n_p < 8192 ? d.n_p : 8192);
    const int pm = max_ps > 0 && max_ps <= kMaxPs ? max_ps : kMaxPs;
    const size_t lds = (size_t)3 * pm * pm * sizeof(double);
    for (int t = 0; t < rounds; ++t) {
        k_a1_begin<<<1, 1, 0, s>>>(d.ctl);
        k_a1_pick<<<cb, 256, 0, s>>>(d.n_comp, d.ctl, d.cstart, d.next, d.mem, d.status, d.rep_slot,
                                     d.rep_patch, d.slot_of_patch, d.repof, d.active);
        if (max_ps <= 4)
            run_a1_invert<4, 4>(d.n_comp, d.ctl, d.active, d.rep_slot, d.rep_patch, d.ptr, d.tiles, d.toff, d.uniform_ps, d.dbt, d.stride, d.ctl + 5, s);
        else if (max_ps <= 12)
            run_a1_invert<12, 16>(d.n_comp, d.ctl, d.active, d.rep_slot, d.rep_patch, d.ptr, d.tiles, d.toff, d.uniform_ps, d.dbt, d.stride, d.ctl + 5, s);
        else if (max_ps <= 16)
            run_a1_invert<16, 16>(d.n_comp, d.ctl, d.active, d.rep_slot, d.rep_patch, d.ptr, d.tiles, d.toff, d.uniform_ps, d.dbt, d.stride, d.ctl + 5, s);
        else if (max_ps <= 24)
            run_a1_invert<24, 32>(d.n_comp, d.ctl, d.active, d.rep_slot, d.rep_patch, d.ptr, d.tiles, d.toff, d.uniform_ps, d.dbt, d.stride, d.ctl + 5, s);
        else
            run_a1_invert<32, 32>(d.n_comp, d.ctl, d.active, d.rep_slot, d.rep_patch, d.ptr, d.tiles, d.toff, d.uniform_ps, d.dbt, d.stride, d.ctl + 5, s);
        k_a1_filter<<<fb, 256, 0, s>>>(d.n_p, d.ctl, d.status, d.pos_comp, d.rep_slot, d.mem, d.rep_patch, d.cand,
                                       d.cinfo);
        k_a1_eval<<<eb, 64, lds, s>>>(d.ctl, crit, eps, pm, d.cand, d.cinfo,
                                    d.ptr, d.tiles, d.toff, d.uniform_ps, d.dbt, d.stride, d.status,
                                    d.repof, d.next, d.counters);
    }
}

void launch_a1_spec_rounds(int rounds, const A1Dev& d, int crit, double eps, int max_ps, hipStream_t s) {
    const unsigned cb = nb(d.n_comp, 256);
    const unsigned fb = nb(d.n_p, 256);
    const unsigned eb = (unsigned)(d.n_p < 8192 ? d.n_p : 8192);
    constexpr int64_t NP = kA1Spec * (kA1Spec - 1) / 2;
    const unsigned pb = (unsigned)(d.n_comp * NP < 8192 ? d.n_comp * NP : 8192);
    const unsigned tb = (unsigned)(d.n_comp * kA1Spec < 4096 ? d.n_comp * kA1Spec : 4096);
    const int pm = max_ps > 0 && max_ps <= kMaxPs ? max_ps : kMaxPs;
    const size_t lds = (size_t)3 * pm * pm * sizeof(double);
    for (int t = 0; t < rounds; ++t) {
        k_a1_begin<<<1, 1, 0, s>>>(d.ctl);
        k_a1s_pick<<<(unsigned)(d.n_comp < 4096 ? d.n_comp : 4096), 64, 0, s>>>(
            d.n_comp, d.ctl, d.cstart, d.next, d.status, d.spec, d.spec_n, d.pairm, d.rep_slot, d.active);
        k_a1s_pairs<<<pb, 64, lds, s>>>(d.ctl, crit, eps, pm, d.active, d.spec, d.spec_n, d.mem, d.ptr, d.tiles,
                                        d.toff, d.uniform_ps, d.inv, d.stride, d.pairm, d.counters);
        k_a1s_resolve<<<cb, 256, 0, s>>>(d.ctl, d.active, d.spec, d.spec_n, d.pairm, d.mem, d.inv_info,
                                         d.status, d.repof, d.rep_slot, d.rep_patch, d.slot_of_patch, d.ent,
                                         d.ent_n, d.ent_slot, d.counters);
        k_a1s_take<<<tb, 64, 0, s>>>(d.ctl, d.active, d.ent, d.ent_n, d.ent_slot, d.mem, d.ptr, d.inv, d.dbt,
                                     d.stride);
        k_a1_filter<<<fb, 256, 0, s>>>(d.n_p, d.ctl, d.status, d.pos_comp, d.rep_slot, d.mem, d.rep_patch, d.cand,
                                       d.cinfo);
        k_a1s_eval<<<eb, 64, lds, s>>>(d.ctl, crit, eps, pm, d.cand, d.cinfo, d.ptr, d.tiles, d.toff,
                                       d.uniform_ps, d.inv, d.stride, d.ent, d.ent_n, d.mem, d.status, d.repof,
                                       d.next, d.counters);
    }
}

void launch_a1_finish(int64_t n_p, const int32_t* repof, int64_t* flags, int64_t* rank, int64_t* scr,
                      int32_t* phi, int32_t* reps, hipStream_t s) {
    k_a1_repflags<<<nb(n_p + 1, 256), 256, 0, s>>>(n_p, repof, flags);
    launch_exclusive_scan_i64(flags, rank, n_p + 1, scr, s);
    k_a1_finish<<<nb(n_p, 256), 256, 0, s>>>(n_p, repof, rank, phi, reps);
}

void launch_a1_closest(int64_t n_p, const int64_t* ptr, const double* tiles, const int64_t* toff, int ups,
                       const int32_t* reps, int64_t m_p, const int64_t* rank, const double* keynorm,
                       double* ekey, int32_t* esz, const double* db, int64_t stride, int crit, double eps,
                       double tie, int32_t* phi, double* lbscr, int64_t grid, unsigned long long* counters,
                       hipStream_t s) {
    if (n_p <= 0 || m_p <= 0) return;
    k_a1_entry_keys<<<nb(m_p, 256), 256, 0, s>>>(m_p, reps, ptr, keynorm, ekey, esz);
    k_a1_closest<<<(unsigned)grid, 64, 0, s>>>(n_p, ptr, tiles, toff, ups, reps, rank, ekey, esz, db, stride,
                                               crit, eps, tie, keynorm, phi, lbscr, m_p, counters);
}

void launch_a1_copy_db(int64_t m_p, const int32_t* reps, const int32_t* slot_of_patch, const int64_t* ptr,
                       const double* dbt, double* db, int64_t stride, hipStream_t s) {
    if (m_p <= 0) return;
    k_a1_copy_db<<<(unsigned)(m_p < 65536 ? m_p : 65536), 256, 0, s>>>(m_p, reps, slot_of_patch, ptr, dbt,
                                                                     db, stride);
}
