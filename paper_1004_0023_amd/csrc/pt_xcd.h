// pt_xcd.h -- placing work on XCDs.  Workgroups go to the XCDs round robin by index from an
// XCD that changes from launch to launch: workgroups b and b + 8 of a launch always share an
// XCD (and its L2), but which XCD b = 0 lands on is not fixed.
#pragma once

#include "pt_common.h"

namespace ptq {

constexpr int kXcds = 8;

__device__ __forceinline__ int xcc_id()
{
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7;  // HW_REG_XCC_ID, 4 bits
}

// Index b of a launch of n workgroups runs item (b mod 8) * q + b / 8 for b < 8 q, q = n / 8,
// and the tail keeps its index: each run of q consecutive items shares an XCD.  A bijection
// for any XCD count; on a device with another count only the locality is lost.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n / kXcds;
    if (b >= kXcds * q) return b;
    return (b % kXcds) * q + b / kXcds;
}

// Workgroup b of a launch that relies on b and b + 8 sharing an XCD: records the XCD offset
// (XCC_ID - b) mod 8 in *seen (zeroed before the launch) and sets the error word's bit
// `err` if another workgroup of the launch found a different one (or, with `force`, a test
// hook, always from workgroup 0).
__device__ __forceinline__ void xcd_check(const DevState &st, uint32_t *seen, int b, uint32_t err,
                                          bool force)
{
    if (threadIdx.x == 0) {
        const uint32_t bit = 1u << ((xcc_id() - b) & 7);
        const uint32_t old = atomicOr(seen, bit);
        if ((old | bit) != bit || (force && b == 0)) atomicOr(st.err, err);
    }
}

// A list position for a workgroup of a launch that takes its work from per-XCD lists (q:
// 9 offsets, then the lists; cnt: 8 counts taken and a count of workgroups done): the next
// one of its own XCD's list, else of the next XCD's list that has one left.  The launch has
// one workgroup per position, so each finds one.  The last workgroup to take its position
// resets the counts for the next launch (every other has taken its own by then).  Returns
// -1 only if every list was empty.
__device__ __forceinline__ int xcd_take(const int32_t *q, int32_t *cnt, int grid)
{
    const int x0 = xcc_id();
    int got = -1;
    for (int j = 0; j < kXcds && got < 0; ++j) {
        const int x = (x0 + j) & 7;
        const int len = q[x + 1] - q[x];
        if (__hip_atomic_load(&cnt[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len) continue;
        const int t = __hip_atomic_fetch_add(&cnt[x], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t < len) got = q[9 + q[x] + t];
    }
    if (__hip_atomic_fetch_add(&cnt[8], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == grid - 1)
        for (int x = 0; x < 9; ++x) __hip_atomic_store(&cnt[x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return got;
}

}  // namespace ptq
