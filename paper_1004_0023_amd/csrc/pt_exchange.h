// pt_exchange.h -- the replica-exchange step of one instance as a device function, shared
// by the exchange launch and the sweep kernels that run an instance's exchange themselves.
#pragma once

#include "pt_common.h"

namespace ptq {

// The value of v in lane src of the calling wave (64-bit values as two halves).
__device__ __forceinline__ int lane_get(int v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ long long lane_get64(long long v, int src)
{
    const int lo = __shfl((int)(uint32_t)(uint64_t)v, src, 64);
    const int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src, 64);
    return (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The exchange step of an instance of R <= 64 replicas by one whole wave: lane t takes
// rung t (its replica, its pair's constants and statistics, its accumulators) and replica t
// (its label, E_cl and C), all loaded in one round of independent loads; the pairs, the
// labels and the accumulators then read each other's values with lane shuffles, and every
// lane stores its own words.  The arithmetic and its order are those of the general form
// below; only the dependent trips to memory are gone.
template <bool COHERENT_EC>
__device__ __forceinline__ void exchange_wave(const DevState &st, const InstDesc &d, int n, uint32_t key0,
                                              uint32_t key1, uint32_t t_add)
{
    auto ld64 = [&](const int64_t *p) -> int64_t {
        if constexpr (COHERENT_EC)
            return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return *p;
    };
    const int t = (int)threadIdx.x & 63;
    const int R = d.R, base = d.rep_base, pb = d.pair_base;
    const bool in = t < R;
    const int s = in ? t : 0;          // lanes past R read slot 0 and store nothing
    const int q = t < R - 1 ? t : 0;   // pair index (R >= 2)
    const uint64_t e = __hip_atomic_load(&st.ctr[n].e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int par = (int)(e & 1u);
    const int rep = st.replica_of[base + s];
    const int lab = st.label[base + s];
    const int64_t Ev = ld64(st.E + base + s), Cv = ld64(st.C + base + s);
    const double db = st.db[pb + q], dK = st.dK[pb + q];
    uint64_t att = st.att[pb + q], acc = st.acc[pb + q];
    uint64_t nup = st.nup[base + s], ndown = st.ndown[base + s];
    int64_t sE = st.sumE[base + s], sC = st.sumC[base + s];
    int64_t sE2 = st.sumE2[base + s], sC2 = st.sumC2[base + s];
    // pairs (t, t + 1) with t = par mod 2
    const bool lower = t + 1 < R && t >= par && ((t - par) & 1) == 0;
    const bool upper = t >= 1 && t < R && t - 1 >= par && ((t - 1 - par) & 1) == 0;
    const int y = lane_get(rep, t + 1 < 64 ? t + 1 : t);
    const int64_t Ex = lane_get64(Ev, rep), Ey = lane_get64(Ev, y);
    const int64_t Cx = lane_get64(Cv, rep), Cy = lane_get64(Cv, y);
    int accept = 0;
    if (lower) {
        const double dE = (double)(Ex - Ey);
        const double dC = (double)(Cx - Cy);
        const double D = db * dE - dK * dC;
        const uint32_t thr = threshold(-D);
        const uint32_t u = philox10((uint32_t)t, (uint32_t)e, 0u, (uint32_t)n, key0, key1).w[0];
        accept = u <= thr ? 1 : 0;
        att += 1;
        acc += (uint64_t)accept;
    }
    const int acc_below = lane_get(accept, t >= 1 ? t - 1 : 0);
    const int rep_below = lane_get(rep, t >= 1 ? t - 1 : 0);
    int nrep = rep;
    if (lower && accept) nrep = y;
    if (upper && acc_below) nrep = rep_below;
    // round-trip labels of the replicas now at the coldest and the hottest rung
    const int cold = lane_get(nrep, 0), hot = lane_get(nrep, R - 1);
    int nlab = lab;
    bool trip = false;
    if (in && t == cold) {
        if (nlab == 2) {
            trip = true;
            nlab = 1;
        } else if (nlab == 0) {
            nlab = 1;
        }
    }
    if (in && t == hot && nlab == 1) nlab = 2;
    // per rung: visit counts and accumulators of the replica now there
    const int labc = lane_get(nlab, nrep);
    const int64_t Ec = lane_get64(Ev, nrep), Cc = lane_get64(Cv, nrep);
    if (labc == 1) nup += 1;
    if (labc == 2) ndown += 1;
    sE += Ec;
    sC += Cc;
    sE2 += Ec * Ec;
    sC2 += Cc * Cc;
    if (in) {
        st.replica_of[base + t] = nrep;
        st.rung_of[base + nrep] = t;
        st.label[base + t] = nlab;
        if (trip) st.rt[base + t] += 1;
        st.nup[base + t] = nup;
        st.ndown[base + t] = ndown;
        st.sumE[base + t] = sE;
        st.sumC[base + t] = sC;
        st.sumE2[base + t] = sE2;
        st.sumC2[base + t] = sC2;
    }
    if (lower) {
        st.att[pb + t] = att;
        st.acc[pb + t] = acc;
    }
    if (t == 0) {
        st.ctr[n].e = e + 1;
        st.ctr[n].n_acc += 1;
        st.ctr[n].t += t_add;
    }
}

// One even/odd exchange step of instance n by the calling workgroup (any size of at least
// one wave; instances of R <= 64 go to its first wave, above): pairs, FP64 D, SWAP-domain
// draws, label swap, statistics, round-trip labels, per-rung visit counts and
// accumulators; then e += 1 and t += t_add.  COHERENT_EC: the replicas' E_cl
// and C were written in the same launch by workgroups that may sit on other XCDs, with
// agent-scope atomic stores, and are read here the same way (every other word the step
// reads was written by earlier launches).
template <bool COHERENT_EC = false>
__device__ __forceinline__ void exchange_instance(const DevState &st, int n, uint32_t key0, uint32_t key1,
                                  uint32_t t_add)
{
    auto ld64 = [&](const int64_t *p) -> int64_t {
        if constexpr (COHERENT_EC)
            return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return *p;
    };
    const InstDesc d = st.inst[n];
    if (d.R <= 64) {
        // one wave; the callers' workgroups have at least one
        if (threadIdx.x < 64) exchange_wave<COHERENT_EC>(st, d, n, key0, key1, t_add);
        return;
    }
    const int R = d.R;
    const int base = d.rep_base;
    const int pb = d.pair_base;
    // a vector load: a workgroup that runs several cycles in one launch updates e itself
    const uint64_t e = __hip_atomic_load(&st.ctr[n].e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int par = (int)(e & 1u);
    for (int j = threadIdx.x;; j += blockDim.x) {
        const int r = par + 2 * j;
        if (r + 1 >= R) break;
        const int x = st.replica_of[base + r];
        const int y = st.replica_of[base + r + 1];
        const double dE = (double)(ld64(st.E + base + x) - ld64(st.E + base + y));
        const double dC = (double)(ld64(st.C + base + x) - ld64(st.C + base + y));
        const double D = st.db[pb + r] * dE - st.dK[pb + r] * dC;
        const uint32_t thr = threshold(-D);
        const uint32_t u = philox10((uint32_t)r, (uint32_t)e, 0u, (uint32_t)n, key0, key1).w[0];
        st.att[pb + r] += 1;
        if (u <= thr) {
            st.replica_of[base + r] = y;
            st.replica_of[base + r + 1] = x;
            st.rung_of[base + y] = r;
            st.rung_of[base + x] = r + 1;
            st.acc[pb + r] += 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int cold = st.replica_of[base];
        const int hot = st.replica_of[base + R - 1];
        const int lc = st.label[base + cold];
        if (lc == 2) {
            st.rt[base + cold] += 1;
            st.label[base + cold] = 1;
        } else if (lc == 0) {
            st.label[base + cold] = 1;
        }
        if (st.label[base + hot] == 1) st.label[base + hot] = 2;
    }
    __syncthreads();  // labels are final
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const int c = st.replica_of[base + r];
        const int lab = st.label[base + c];
        if (lab == 1) st.nup[base + r] += 1;
        if (lab == 2) st.ndown[base + r] += 1;
        const long long E = ld64(st.E + base + c);
        const long long C = ld64(st.C + base + c);
        st.sumE[base + r] += E;
        st.sumC[base + r] += C;
        st.sumE2[base + r] += E * E;
        st.sumC2[base + r] += C * C;
    }
    if (threadIdx.x == 0) {
        st.ctr[n].e = e + 1;
        st.ctr[n].n_acc += 1;
        st.ctr[n].t += t_add;
    }
}

}  // namespace ptq
