// wheel.hip -- trial division on the 2/3/5/7 wheel, the paper's method for
// medium integers (section 3), as an optional stage between the filter and
// Miller-Rabin: every survivor below 2^wheel_log2 (at most 2^40) is decided
// here by dividing it by 3, 5, 7 and the wheel numbers up to its square
// root, and only the others go on to the Miller-Rabin kernels.
//
// The wheel numbers are those coprime to 210 from 11 up: 1 plus the running
// sum of the period-210 difference cycle (Eq. 5 and 6), i.e. 210 q + R[i]
// with R the 48 residues coprime to 210 in [11, 211].
//
// GPU mapping: several workgroups per classify region, one survivor per
// lane; a decided entry is marked and a second kernel compacts each region
// in place, like the second filter stage.  All lanes of a wavefront test
// the same divisor at the same time: lane j computes the inverse modulo 2^64
// of divisor k0 + j once per 64 divisors and the wavefront reads them back
// from LDS one at a time.  The wavefront stops after the chunk that passes
// the square root of every lane still undecided.
//
// The test: with q = n * d^-1 mod 2^64, d | n gives q = n / d < 2^40 / 3 <
// 2^43; conversely q < 2^43 and d < 2^21 give q * d < 2^64, so q * d = n
// exactly.  For n < 2^40 and d < 2^21, d | n holds iff the high 32 bits of q
// are below 2^11: four VALU instructions per divisor and lane (their
// running minimum is taken three at a time), no division.  Every tested
// divisor is below 2^21: a chunk of 64 is entered only while some root
// (< 2^20) lies beyond the previous chunk's last divisor, so it starts at
// most one gap (10) above that root and spans less than 64 * 10.  A divisor
// above a lane's own root that divides it still shows a composite (d < 2^21
// < n), so whole chunks are tested.
#include "compact.h"
#include "internal.h"

#include <math.h>

#include <algorithm>

namespace isp {

namespace {

constexpr int WHEEL_BLOCK = 256;
constexpr int WHEEL_WAVES = WHEEL_BLOCK / 64;
constexpr uint32_t WHEEL_MIN_GROUPS = 2048;  // 8 wavefronts per SIMD
constexpr uint32_t WHEEL_Q_HI = 1u << 11;  // d | n iff hi32(n * d^-1 mod 2^64) < this

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t ce_gcd(uint32_t a, uint32_t b) { return b ? ce_gcd(b, a % b) : a; }

// The 48 residues coprime to 210 in [11, 211], in increasing order.
struct WheelResidues {
    uint32_t r[48];
    constexpr WheelResidues() : r()
    {
        int k = 0;
        for (uint32_t v = 11; v <= 211; ++v)
            if (ce_gcd(v, 210) == 1)
                r[k++] = v;
    }
};
constexpr WheelResidues WHEEL{};
static_assert(WHEEL.r[0] == 11 && WHEEL.r[5] == 29 && WHEEL.r[47] == 211, "wheel residues");

// Inverse of an odd d modulo 2^64 by Newton's iteration (each step doubles
// the correct low bits; (3d) xor 2 is correct to 5 bits).
__device__ __forceinline__ uint64_t inv64_of(uint32_t d)
{
    uint32_t x = (3u * d) ^ 2u;
    x *= 2u - d * x;
    x *= 2u - d * x;
    x *= 2u - d * x;
    uint64_t y = x;
    y *= 2ull - (uint64_t)d * y;
    return y;
}


__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Decides the survivors below `bound` of each classify region, writes their
// output bytes and marks their entries with n = 0.  `split` workgroups share
// a region, and its wavefronts take the region's entries 64 at a time, so
// the launch is not limited to one workgroup per region and the wavefronts
// need no workgroup barrier.  Workgroup sub * regions + g serves region g:
// the first entries of every region (the busy wavefronts when regions are
// short) go to the first workgroups, which the dispatcher spreads over all
// XCDs and CUs.
__global__ void __launch_bounds__(WHEEL_BLOCK) wheel_kernel(Survivor *__restrict__ surv,
                                                            const uint32_t *__restrict__ counts,
                                                            uint64_t total,
                                                            const uint64_t *total_dev,
                                                            uint64_t bound, uint32_t split)
{
    __shared__ __attribute__((aligned(16))) uint32_t inv_lds[WHEEL_WAVES][64][2];
    __shared__ uint32_t res[48];
    if (threadIdx.x < 48)
        res[threadIdx.x] = WHEEL.r[threadIdx.x];
    __syncthreads();
    const uint32_t regions = gridDim.x / split;  // the classify grid
    const uint32_t sub = blockIdx.x / regions, g = blockIdx.x - sub * regions;
    const uint64_t chunk = classify_chunk(total_dev ? *total_dev : total, regions);
    Survivor *region = surv + (uint64_t)g * chunk;
    const uint32_t count = counts[g];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t(*inv)[2] = inv_lds[wave];
    for (uint32_t base = (sub * WHEEL_WAVES + wave) * 64; base < count;
         base += split * WHEEL_BLOCK) {
        const uint32_t i = base + lane;
        Survivor e;
        e.n = 0;
        e.out = nullptr;
        bool mine = false;  // decided here: 2^32 <= n < bound
        if (i < count) {
            e = region[i];
            mine = e.n < bound;
        }
        const uint32_t nl = (uint32_t)e.n, nh = (uint32_t)(e.n >> 32);
        const uint32_t root = mine ? (uint32_t)isqrt_u64(e.n) : 0u;
        uint32_t hmin = ~0u;  // smallest high word of n * d^-1 so far
        // chunks of 64 divisors (lane j: divisor k0 + j of 3, 5, 7, 11, ...)
        // while some undecided lane's root lies beyond the last one tested
        bool more = __ballot(mine) != 0;
        for (uint32_t k0 = 0; more; k0 += 64) {
            const uint32_t t = k0 + lane;
            uint32_t d = 3 + 2 * t;
            if (t >= 3) {
                const uint32_t u = t - 3, q = u / 48;
                d = 210 * q + res[u - 48 * q];
            }
            const uint64_t y = inv64_of(d);
            inv[lane][0] = (uint32_t)y;
            inv[lane][1] = (uint32_t)(y >> 32);
            wave_sync_lds();
            // a running minimum in a VGPR keeps the compares off the scalar
            // unit; the inverses of the next 8 divisors are read while the
            // current 8 are tested (4 x 16 bytes, two divisors per read)
            const u32x4 *inv4 = reinterpret_cast<const u32x4 *>(&inv[0][0]);
            u32x4 cur[4], nxt[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                cur[q] = inv4[q];
#pragma unroll
            for (int blk = 0; blk < 8; ++blk) {
                if (blk < 7) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        nxt[q] = inv4[4 * (blk + 1) + q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t h0 = __umulhi(nl, cur[q].x) + nl * cur[q].y + nh * cur[q].x;
                    const uint32_t h1 = __umulhi(nl, cur[q].z) + nl * cur[q].w + nh * cur[q].z;
                    hmin = min(hmin, min(h0, h1));
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    cur[q] = nxt[q];
            }
            wave_sync_lds();  // the next chunk rewrites inv
            const uint32_t dlast = __builtin_amdgcn_readlane(d, 63);
            more = __ballot(mine && hmin >= WHEEL_Q_HI && root > dlast) != 0;
        }
        if (mine) {
            *e.out = hmin < WHEEL_Q_HI ? 0 : 1;  // a divisor in [3, root] or none
            region[i].n = 0;                      // decided: dropped by the compaction
        }
    }
}

// Drops the entries marked n = 0 from each region, order kept, and rewrites
// the region's count (one workgroup per region).
__global__ void __launch_bounds__(WHEEL_BLOCK) wheel_compact_kernel(Survivor *__restrict__ surv,
                                                                    uint32_t *__restrict__ counts,
                                                                    uint64_t total,
                                                                    const uint64_t *total_dev)
{
    __shared__ uint32_t wave_cnt[WHEEL_WAVES];
    const uint32_t g = blockIdx.x;
    const uint64_t chunk = classify_chunk(total_dev ? *total_dev : total, gridDim.x);
    Survivor *region = surv + (uint64_t)g * chunk;
    const uint32_t count = counts[g];
    uint32_t kept = 0;  // entries kept so far (block-uniform)
    for (uint32_t r0 = 0; r0 < count; r0 += WHEEL_BLOCK) {
        const uint32_t i = r0 + threadIdx.x;
        Survivor e;
        e.n = 0;
        e.out = nullptr;
        if (i < count)
            e = region[i];
        compact_round<WHEEL_BLOCK>(region, e, e.n != 0, kept, wave_cnt);
    }
    if (threadIdx.x == 0)
        counts[g] = kept;
}

}  // namespace

hipError_t launch_wheel(Survivor *surv, uint32_t *counts, unsigned grid, uint64_t total,
                        const uint64_t *total_dev, int log2_bound, hipStream_t s)
{
    if (log2_bound < WHEEL_MIN_LOG2 || log2_bound > WHEEL_MAX_LOG2 || grid == 0)
        return hipErrorInvalidValue;
    // enough workgroups to fill the part whatever the classify grid was
    const uint32_t split = std::max(1u, WHEEL_MIN_GROUPS / grid);
    wheel_kernel<<<grid * split, WHEEL_BLOCK, 0, s>>>(surv, counts, total, total_dev,
                                                      (uint64_t)1 << log2_bound, split);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    wheel_compact_kernel<<<grid, WHEEL_BLOCK, 0, s>>>(surv, counts, total, total_dev);
    return hipGetLastError();
}

}  // namespace isp
