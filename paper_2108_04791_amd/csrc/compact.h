// compact.h -- one round of an in-place, order-keeping compaction of a
// survivor region, shared by the kernels that drop entries from the regions
// written by classify_kernel (the second filter stage and the wheel).
#pragma once

#include "internal.h"

namespace isp {

// Every thread of a BLOCK-thread workgroup holds one entry `e` of the round
// (entries r0 .. r0 + BLOCK - 1 of the region, read before this call) and a
// flag `keep`.  The kept entries of the round go, in their order, right after
// the `kept` entries kept by earlier rounds; `kept` grows by the round's
// total on every thread.  Every written position is at most the writer's own
// position, and all of the round's entries are read before the first
// barrier, so nothing unread is overwritten.  wave_cnt: LDS, one word per
// wavefront.
template <int BLOCK>
__device__ __forceinline__ void compact_round(Survivor *__restrict__ region, const Survivor &e,
                                              bool keep, uint32_t &kept, uint32_t *wave_cnt)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t m = __ballot(keep);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0)
        wave_cnt[wave] = (uint32_t)__popcll(m);
    __syncthreads();  // every entry of this round is read; the counts are in
    uint32_t before = 0, total = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
        const uint32_t c = wave_cnt[w];
        before += w < wave ? c : 0u;
        total += c;
    }
    if (keep)
        region[kept + before + (uint32_t)__popcll(m & lt)] = e;
    kept += total;
    __syncthreads();  // wave_cnt is rewritten by the next round
}

}  // namespace isp
