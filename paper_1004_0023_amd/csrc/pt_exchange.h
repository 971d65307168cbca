// pt_exchange.h -- the replica-exchange step of one instance as a device function, shared
// by the exchange launch and the sweep kernels that run an instance's exchange themselves.
#pragma once

#include "pt_common.h"

namespace ptq {

// One even/odd exchange step of instance n by the calling workgroup (any size): pairs,
// FP64 D, SWAP-domain draws, label swap, statistics, round-trip labels, per-rung visit
// counts and accumulators; then e += 1 and t += t_add.  COHERENT_EC: the replicas' E_cl
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
