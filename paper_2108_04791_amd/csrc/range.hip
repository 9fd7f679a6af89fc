// range.hip -- primality of every integer in a contiguous interval
// [lo, lo + len), without an input array.
//
// Paper: section 6.1.3 sieves all primes up to the maximum once and then
// only tests membership; section 1 describes the sieve of Eratosthenes.
// For an interval that is the natural way to work: the part below 2^32 is
// copied out of the device table, bit by bit; above it, each workgroup sieves
// one segment of the interval in LDS by the odd primes up to
// sqrt(segment end) while that is below 2^25 (segment end below 2^50); then
// the survivors are exactly the primes.  Above it, a long piece runs in
// bucket mode (below): the primes above 2^21 up to the square root are
// sorted into per-segment buckets first, and the segments are complete
// again.  A short piece is sieved by the odd primes below 2^22 (below 2^18
// when it has fewer than 256 full segments of 2^19 numbers; it is then cut
// into up to 256 shorter ones, since so few workgroups would wait on the
// sieve's latency)
// and the survivors (about 3.4% of the numbers with no factor below 2^22,
// 4.5% below 2^18) go to the same two Miller-Rabin kernels as array inputs,
// through the same per-workgroup regions and counts.
//
// Segment layout: workgroup g covers numbers [lo + g*chunk, lo + (g+1)*chunk)
// with chunk = classify_chunk(len, grid) (a multiple of 64, at most
// RANGE_SEG = 2^20: that in bucket mode and where the sieving primes pass
// 2^20 over at least 256 segments, else at most 2^19); bit j of its LDS
// bitset stands for the odd number o0 + 2j.
// The multiples of 3 .. 31 come from periodic word masks (pre-sieve);
// primes 37 .. 4093 are crossed off by whole wavefronts (lane l takes the
// multiples l, l+64, ... of the stride), larger primes one per thread.  The
// first odd multiple of p at or above o0 needs o0 mod p: the piece's residue
// (lo | 1) mod p, computed once per piece with a precomputed
// floor((2^64 - 1) / p) (one 64-bit multiply-high, no division), plus the
// segment's offset reduced with floor(2^32 / p).  The sieving primes are below 2^25 and o0 is at least 2^32, so
// every multiple crossed off is a proper one (no start at p^2 is needed).
//
// Output: 16 consecutive numbers per thread per pass, consecutive threads on
// consecutive 16-byte pieces.  Their 8 odd members are 8 consecutive bits;
// each group of 4 bits becomes 8 output bytes by one multiply that spreads
// bit i to byte 2i (or 2i + 1), and the piece goes out as one 16-byte store.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace isp {

namespace {

constexpr int RANGE_THREADS = 1024;
// primes below this: wavefront per prime (measured against 8192, 2048 and
// 1024: 2^28 numbers at 2^34 0.101 -> 0.099 ms, at 2^44 0.194 -> 0.189)
constexpr uint32_t WAVE_PRIME_LIMIT = 4096;
constexpr int PRESIEVED = 10;                 // 3 .. 31: index of 37 in the prime list
constexpr uint32_t SMALL_PRIMES[PRESIEVED] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31};

// Bits j < 32 with j = 0 (mod p).
__host__ __device__ constexpr uint32_t period_mask(uint32_t p)
{
    uint32_t m = 0;
    for (uint32_t j = 0; j < 32; j += p)
        m |= 1u << j;
    return m;
}

// Bits 0..3 of `nib` moved to bits 0, 16, 32, 48 (bytes 0, 2, 4, 6): the
// product nib * (1 + 2^15 + 2^30 + 2^45) holds bit i + 15k for every set bit
// i and every k < 4, all distinct, and i + 15k = 16m only for i = k = m.
__device__ __forceinline__ uint64_t spread4(uint32_t nib)
{
    return ((uint64_t)nib * 0x0000200040008001ull) & 0x0001000100010001ull;
}

__device__ __forceinline__ uint64_t umulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// x mod p for 64-bit x and p < 2^32, with inv = floor((2^64 - 1) / p).
__device__ __forceinline__ uint64_t mod_small(uint64_t x, uint32_t p, uint64_t inv)
{
    const uint64_t q = umulhi64(x, inv);  // q <= floor(x / p), off by at most 1
    uint64_t r = x - q * p;
    if (r >= p)
        r -= p;
    if (r >= p)
        r -= p;
    return r;
}

// The interval sieve's primes: the odd primes below 2^25 from the device
// table (bits of odd numbers below 2^25 are its first 2^19 words), in order,
// with floor((2^64 - 1) / p).  Two passes of RANGE_LIST_GROUPS workgroups,
// each over 1024 consecutive words: count, then write at the group's offset.
constexpr int LIST_WORDS = (1 << (RANGE_PRIME_LOG2 - 6)) / RANGE_LIST_GROUPS;  // per group
static_assert(LIST_WORDS == 1024, "one word per thread-slot below");

__global__ void __launch_bounds__(256) range_count_kernel(const uint32_t *__restrict__ table,
                                                         uint32_t *__restrict__ counts)
{
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t w0 = blockIdx.x * LIST_WORDS + tid * 4;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        c += __popc(table[w0 + k]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o, 64);
    if (lane == 0)
        wsum[wave] = c;
    __syncthreads();
    if (tid == 0)
        counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ void __launch_bounds__(256) range_list_kernel(const uint32_t *__restrict__ table,
                                                        uint32_t *__restrict__ counts,
                                                        uint32_t *__restrict__ primes,
                                                        uint64_t *__restrict__ inv)
{
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // this group's offset: the counts of the groups before it
    uint32_t before = 0;
    for (uint32_t g = tid; g < blockIdx.x; g += blockDim.x)
        before += counts[g];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        before += __shfl_xor(before, o, 64);
    if (lane == 0)
        wsum[wave] = before;
    __syncthreads();
    if (tid == 0)
        base = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    const uint32_t w0 = blockIdx.x * LIST_WORDS + tid * 4;
    uint32_t word[4], c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        word[k] = table[w0 + k];
        c += __popc(word[k]);
    }
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += y;
    }
    __syncthreads();  // wsum is reused
    if (lane == 63)
        wsum[wave] = incl;
    __syncthreads();
    uint32_t pos = base + incl - c;
    for (int w = 0; w < wave; ++w)
        pos += wsum[w];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t x = word[k];
        while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1;
            const uint32_t p = 2u * (32u * (w0 + k) + (uint32_t)b) + 1u;
            primes[pos] = p;
            inv[pos] = ~(uint64_t)0 / p;
            ++pos;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && tid == blockDim.x - 1)
        counts[RANGE_LIST_GROUPS] = pos;  // the total
}

// out[i] = primality of lo + i for lo + len <= 2^32: one table bit per odd
// number.  A wavefront writes 4096 consecutive bytes in four stores of 1 KiB:
// in store k, lane l writes the 16 bytes of numbers 1024k + 16l .. + 15 of
// the wavefront's block, whose 8 odd members are 8 consecutive table bits.
__global__ void __launch_bounds__(256) range_table_kernel(uint64_t lo, uint8_t *__restrict__ out,
                                                         uint64_t len,
                                                         const uint32_t *__restrict__ table)
{
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t block0 = wave * 4096;
    if (block0 >= len)
        return;  // uniform over the wavefront
    const int odd_at = (int)(~lo & 1) * 8;  // odd numbers at bytes 1, 3, .. (lo even) or 0, 2, ..
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2), aligned(1)));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t i0 = block0 + 1024 * k + 16 * lane;
        if (i0 >= len)
            break;
        const uint64_t v0 = lo + i0;          // < 2^32
        const uint64_t b = (v0 | 1) >> 1;     // table bit of the first odd number
        const uint64_t w = b >> 5;
        const uint64_t pair = (uint64_t)table[w] |
                              (w + 1 < TABLE_WORDS ? (uint64_t)table[w + 1] << 32 : 0ull);
        const uint32_t bits = (uint32_t)(pair >> (b & 31));
        u64x2 q;
        q.x = spread4(bits & 0xfu) << odd_at;
        q.y = spread4((bits >> 4) & 0xfu) << odd_at;
        if (v0 <= 2 && v0 + 16 > 2) {
            const int at = (int)(2 - v0);  // 2 is prime; its table bit is that of 1
            q.x |= 1ull << (8 * at);
        }
        if (i0 + 16 <= len) {
            *reinterpret_cast<u64x2 *>(out + i0) = q;
        } else {
            for (uint64_t i = i0; i < len; ++i) {
                const uint64_t word = (i - i0) < 8 ? q.x : q.y;
                out[i] = (uint8_t)(word >> (8 * ((i - i0) & 7)));
            }
        }
    }
}

struct RangeArgs {
    uint64_t lo;         // first number of this piece (>= 2^32)
    uint64_t len;        // numbers in this piece
    uint64_t chunk;      // numbers per segment (the last one may be shorter)
    uint8_t *out;        // out[i] <-> lo + i
    const uint32_t *primes;
    const SievePrime *res;  // res[k]: primes[k], floor(2^32 / primes[k]) and
                            // (lo | 1) mod primes[k], for every prime the piece uses
    uint32_t nprimes;
    Survivor *surv;      // grid regions of `chunk` entries
    uint32_t *counts;    // [grid]
    // bucket mode: the primes above BUCKET_SMALL come as precomputed hits
    const uint32_t *hit_start;  // [grid + 1]: the hits of segment g are
                                // hits[hit_start[g] .. hit_start[g + 1])
    const uint32_t *hits;       // bit indices within their segment
    uint64_t hit_cap;           // entries allocated in hits
    uint32_t groups;            // 0: no buckets
    uint32_t partial_log2;      // where the sieve cannot be complete: primes below 2^this
    uint32_t complete_log2;     // segments whose root is below 2^this are complete
};


__global__ void __launch_bounds__(RANGE_THREADS) range_sieve_kernel(RangeArgs a)
{
    constexpr int MAX_WORDS = (int)(RANGE_SEG / 64);  // 2^14 words of odd-number bits
    __shared__ uint32_t bits[MAX_WORDS + 1];          // + one zero word past the end
    __shared__ uint32_t wsum[RANGE_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63;
    // the wavefront index as a scalar (the wavefront loop below is uniform)
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    const uint64_t chunk = a.chunk;
    const uint64_t r0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t r1 = r0 + chunk < a.len ? r0 + chunk : a.len;
    if (r0 >= r1) {
        if (tid == 0 && a.counts)
            a.counts[blockIdx.x] = 0;
        return;
    }
    const uint64_t s_lo = a.lo + r0;          // first number of the segment
    const uint64_t s_last = a.lo + r1 - 1;    // last number (no overflow: <= 2^64 - 1)
    // first odd number; s_lo | 1 cannot wrap (s_lo = 2^64 - 1 is already odd)
    const uint64_t o0 = s_lo | 1;
    const uint32_t nbits = o0 > s_last ? 0u : (uint32_t)((s_last - o0) / 2 + 1);
    const uint32_t nwords = (nbits + 31) / 32;

    // pre-sieve: bit j of word w (j = 32w + i) is o0 + 2j, which p divides
    // iff j = jp (mod p) with jp = -o0 / 2 mod p
    {
        uint32_t jp[PRESIEVED], dp[PRESIEVED], rp[PRESIEVED];
        const uint32_t per = (nwords + blockDim.x - 1) / blockDim.x;
        const uint32_t ws = tid * per;
#pragma unroll
        for (int q = 0; q < PRESIEVED; ++q) {
            const uint32_t p = SMALL_PRIMES[q];
            jp[q] = (uint32_t)(((p - o0 % p) % p) * ((p + 1) / 2) % p);
            dp[q] = (p - 32u % p) % p;  // position shift from one word to the next
            rp[q] = (jp[q] + p - (32u * ws) % p) % p;
        }
        for (uint32_t w = ws; w < ws + per && w < nwords; ++w) {
            uint32_t word = w + 1 < nwords || (nbits & 31) == 0 ? 0xffffffffu
                                                                 : (1u << (nbits & 31)) - 1u;
#pragma unroll
            for (int q = 0; q < PRESIEVED; ++q) {
                word &= ~(period_mask(SMALL_PRIMES[q]) << rp[q]);
                rp[q] += dp[q];
                if (rp[q] >= SMALL_PRIMES[q])
                    rp[q] -= SMALL_PRIMES[q];
            }
            bits[w] = word;
        }
        if (tid == 0)
            bits[nwords] = 0;
    }
    __syncthreads();
    const uint64_t root = isqrt_u64(s_last);
    // Crossing off every prime up to the root costs about one reduction per
    // prime and segment; below a root of 2^25 (2 million primes) that is
    // cheaper than Miller-Rabin on the survivors, and the sieve alone decides
    // the segment.  Above it the segment is sieved by the primes below
    // 2^partial_log2 (2^22 for long pieces: about 3.4% of the numbers
    // survive) and its survivors go to Miller-Rabin.
    // (in bucket mode the primes above BUCKET_SMALL arrive as hits, and every
    // segment is complete)
    const bool buckets = a.groups != 0;
    const bool complete = buckets || root < ((uint64_t)1 << a.complete_log2);
    const uint64_t bound = buckets ? (root < BUCKET_SMALL ? root : BUCKET_SMALL)
                           : complete ? root : ((uint64_t)1 << a.partial_log2) - 1;
    // the list is sorted: use the primes up to `bound`
    uint32_t np = a.nprimes;
    {
        uint32_t lo_i = 0, hi_i = np;  // first index with prime > bound
        while (lo_i < hi_i) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if ((uint64_t)a.primes[mid] <= bound)
                lo_i = mid + 1;
            else
                hi_i = mid;
        }
        np = lo_i;
    }
    // first bit index of the odd multiples of p at or above o0 (> p), or
    // "none" (all offsets are taken from o0, so nothing wraps near 2^64).
    // o0 = (lo | 1) + r0 (the chunk is even), so o0 mod p is the piece's
    // residue res[k] plus r0 mod p; r0 < 2^30 is reduced with m = floor(2^32
    // / p), the high word of floor((2^64 - 1) / p) (p odd): the estimate
    // umulhi(r0, m) is floor(r0 / p) or one less, leaving a remainder below 2p
    const uint64_t span = s_last - o0;  // valid only when nbits > 0
    const uint32_t off0 = (uint32_t)r0;
    auto first_bit = [&](uint32_t p, uint32_t m, uint32_t res) -> uint32_t {
        uint32_t u = off0 - __umulhi(off0, m) * p;
        u = u >= p ? u - p : u;
        uint32_t r = res + u;  // o0 mod p, before one subtraction
        r = r >= p ? r - p : r;
        uint32_t off = r ? p - r : 0u;  // o0 + off: first multiple of p at or above o0
        if (off & 1u)
            off += p;                    // o0 is odd: an odd offset gives an even multiple
        return (uint64_t)off > span ? ~0u : off >> 1;
    };
    // primes 37 .. WAVE_PRIME_LIMIT: one wavefront per prime
    uint32_t k_split;
    {
        uint32_t lo_i = 0, hi_i = np;  // first index with prime >= WAVE_PRIME_LIMIT
        while (lo_i < hi_i) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if (a.primes[mid] < WAVE_PRIME_LIMIT)
                lo_i = mid + 1;
            else
                hi_i = mid;
        }
        k_split = lo_i;
    }
    // (the wavefront's primes are k = PRESIEVED + wave + m nwaves; their
    // first bits are computed 64 at a time, one per lane, and each crossing
    // loop takes its prime and start from a lane: the reductions run on the
    // vector units instead of the compute unit's one scalar unit)
    for (uint32_t kb = PRESIEVED + wave; kb < k_split; kb += 64u * nwaves) {
        const uint32_t k = kb + (uint32_t)lane * nwaves;
        uint32_t pl = 0, jl = ~0u;
        if (k < k_split) {
            const SievePrime e = a.res[k];
            pl = e.p;
            const uint32_t j0 = first_bit(e.p, e.m, e.res);
            jl = j0 < nbits ? j0 : ~0u;
        }
        const uint32_t cnt = min(64u, (k_split - kb + nwaves - 1) / nwaves);
        for (uint32_t i = 0; i < cnt; ++i) {
            const uint32_t p = __builtin_amdgcn_readlane(pl, i);
            const uint32_t j0 = __builtin_amdgcn_readlane(jl, i);
            if (j0 == ~0u)
                continue;
            // bit indices below 2^19: 32-bit arithmetic
            const uint32_t stride = 64u * p;
            for (uint32_t j = j0 + (uint32_t)lane * p; j < nbits; j += stride)
                atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
        }
    }
    // larger primes: one thread per prime, four at a time; the thread's next
    // four primes and their constants are loaded while the current ones are
    // crossed off (the loads' latency, not the arithmetic, bounds this loop:
    // at 2^44, one workgroup per CU, four in flight instead of one took the
    // 2^28-number interval from 0.241 to 0.203 ms)
    {
        constexpr int U = 4;
        const uint32_t stride = blockDim.x;
        uint32_t p[U], m[U], rs[U];
        auto load = [&](uint32_t kb) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t k = kb + u * stride;
                p[u] = m[u] = rs[u] = 0;
                if (k < np) {
                    const SievePrime e = a.res[k];
                    p[u] = e.p;
                    m[u] = e.m;
                    rs[u] = e.res;
                }
            }
        };
        load(k_split + tid);
        for (uint32_t kb = k_split + tid; kb < np; kb += U * stride) {
            uint32_t cp[U], cm[U], cr[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cp[u] = p[u];
                cm[u] = m[u];
                cr[u] = rs[u];
            }
            load(kb + U * stride);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (kb + u * stride < np)
                    for (uint32_t j = first_bit(cp[u], cm[u], cr[u]); j < nbits; j += cp[u])
                        atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
        }
    }
    // bucket mode: the hits of the primes above BUCKET_SMALL in this segment,
    // one contiguous run (the clamp only keeps reads inside the allocation),
    // eight per thread and round, all read before any is applied and the
    // next round's read while this one is (streaming loads: this is their
    // last use, and the caches are left to the hits still to be sorted)
    if (buckets) {
        const uint32_t h0 = a.hit_start[blockIdx.x];
        const uint32_t h1 = (uint32_t)min((uint64_t)a.hit_start[blockIdx.x + 1], a.hit_cap);
        constexpr int UNROLL = 8;
        uint32_t next[UNROLL];
        auto load = [&](uint64_t h) {
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                const uint64_t i = h + (uint64_t)k * blockDim.x;
                next[k] = i < h1 ? __builtin_nontemporal_load(&a.hits[i]) : ~0u;
            }
        };
        load(h0 + tid);
        for (uint64_t h = h0 + tid; h < h1; h += (uint64_t)UNROLL * blockDim.x) {
            uint32_t j[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k)
                j[k] = next[k];
            load(h + (uint64_t)UNROLL * blockDim.x);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k)
                if (j[k] < nbits)
                    atomicAnd(&bits[j[k] >> 5], ~(1u << (j[k] & 31)));
        }
    }
    __syncthreads();
    // outputs: 16 consecutive numbers per thread per pass, consecutive threads
    // on consecutive 16-byte pieces (8 odd numbers: bits 8m .. 8m + 7, m =
    // the piece's index in the segment); the survivors of an incomplete sieve
    // go to the Miller-Rabin kernels (their bytes are 0 until then)
    Survivor *region = a.surv + r0;
    const int odd_at = (int)(~s_lo & 1) * 8;
    uint32_t filled = 0;
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2), aligned(1)));
    for (uint64_t p0 = r0; p0 < r1; p0 += 16ull * blockDim.x) {
        const uint64_t i0 = p0 + 16ull * tid;
        const uint32_t m = (uint32_t)((i0 - r0) >> 4);
        uint32_t b8 = 0;
        if (i0 < r1)
            b8 = (bits[m >> 2] >> (8 * (m & 3))) & 0xffu;
        const uint32_t cnt = complete ? 0u : (uint32_t)__popc(b8);
        if (i0 < r1) {
            const uint32_t shown = complete ? b8 : 0u;
            u64x2 q;
            q.x = spread4(shown & 0xfu) << odd_at;
            q.y = spread4(shown >> 4) << odd_at;
            if (i0 + 16 <= r1) {
                *reinterpret_cast<u64x2 *>(a.out + i0) = q;
            } else {
                for (uint64_t i = i0; i < r1; ++i) {
                    const uint64_t word = (i - i0) < 8 ? q.x : q.y;
                    a.out[i] = (uint8_t)(word >> (8 * ((i - i0) & 7)));
                }
            }
        }
        if (complete)
            continue;  // uniform over the workgroup
        // block-wide exclusive scan of cnt
        uint32_t incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o)
                incl += y;
        }
        if (lane == 63)
            wsum[wave] = incl;
        __syncthreads();
        uint32_t pos = filled + incl - cnt, all = 0;
        for (int w = 0; w < nwaves; ++w) {
            pos += w < wave ? wsum[w] : 0u;
            all += wsum[w];
        }
        uint32_t rest = b8;
        const uint64_t first_odd = (a.lo + i0) | 1;
        while (rest) {
            const int t = __ffs(rest) - 1;
            rest &= rest - 1;
            Survivor sv;
            sv.n = first_odd + 2ull * (uint64_t)t;
            sv.out = a.out + (sv.n - a.lo);
            region[pos++] = sv;
        }
        filled += all;
        __syncthreads();  // wsum is rewritten next pass
    }
    if (tid == 0 && a.counts)
        a.counts[blockIdx.x] = filled;
}

// ---- bucket mode: crossing off by the primes above BUCKET_SMALL ----------
//
// A prime p > 2^19 has at most one odd multiple in a segment of 2^20
// numbers (bucket mode's segments; BUCKET_SMALL is above that bound), so
// visiting every such prime in every segment costs one reduction per prime
// and segment.  Bucket mode inverts the loop (the bucket sieve of segmented
// sieving): the odd primes in (BUCKET_SMALL, sqrt(end)] are read from the
// device table, each prime's odd multiples at or above lo (which exceeds
// every such prime) are enumerated once over the whole piece, and each
// becomes a hit (its bit index) in the bucket of its segment.  `groups`
// workgroups share the primes; no global atomic is needed:
//   0. split (one workgroup): each group's table words;
//   1. bound: an upper bound on each group's hits, floor((len - 1) / 2p) + 1
//      per prime p (at most that many odd multiples of p lie in len
//      consecutive numbers): prime counts from the chunk count table for
//      the primes above len / 2, the quotient for those below;
//   2. plan (one workgroup): each group's stretch of the stream (its bound)
//      and its number of sort tiles;
//   3. fill: each group enumerates its hits and appends them, in the order
//      found, to its stretch of the stream (one contiguous store per
//      wavefront step), and records how many it found;
//   4. histogram: per tile of a group's stretch, its hits per segment;
//   5. an exclusive scan of those counts, laid out (segment, tile), which is
//      exactly the order of the hits: each segment's together, by tile
//      within it, so each count's scanned value is where that tile's hits of
//      that segment go;
//   6. starts: the first hit of each segment;
//   7. scatter: each tile's hits, put in segment order in LDS, written to
//      their places, consecutive threads at consecutive places.
// Writing each hit straight to its bucket from the enumeration would keep
// groups x segments partly written 128-byte lines open at once (32 MB for
// 512 groups and 512 segments, the whole L2): measured, each line reached
// HBM about 2.5 times over and the pass took twice the enumeration.  The
// segment kernel then applies its segment's one run of hits.
// With every prime up to the square root crossed off, the segments are
// complete at any magnitude below 2^64.

struct BucketArgs {
    uint64_t lo, len;        // the piece
    uint64_t w_begin, w_end; // table words holding the odd primes in (BUCKET_SMALL, root]
    uint64_t w_mid;          // the bound pass takes words w_begin .. w_mid - 1 prime by prime
    uint64_t root;
    const uint32_t *table;
    const uint32_t *chunk_primes;  // [TABLE_CHUNKS + 1]: odd primes below 4096 c
    uint32_t nseg;           // segments of RANGE_SEG numbers
    uint32_t groups;         // workgroups of the count and fill passes
    uint32_t tile;           // hits per sort tile (a multiple of BUCKET_SORT_SUB)
    uint32_t max_tiles;      // workgroups of the per-tile kernels (at least the tiles)
    uint32_t bound_per;      // table words per thread of the bound pass
    uint32_t *wsplit;        // [groups + 1]: each group's first table word
    uint32_t *totals;        // [groups]: bound on the hits of each group
    uint32_t *filled;        // [groups]: hits each group found
    uint32_t *sbase;         // [groups + 1]: each group's first place in the stream
    uint32_t *tprefix;       // [groups + 1]: each group's first tile
    uint32_t *tcounts;       // [nseg * max_tiles + 1]: hits per (group, segment, tile),
                             // scanned in place
    uint32_t *hs;            // [nseg + 1]: the first hit of each segment
    uint32_t *hits;          // hit_cap entries: bit indices within their segment
    uint32_t *stream;        // hit_cap entries: segment << HIT_BITS | bit index
    uint64_t hit_cap;
};

// A hit in the stream: the segment (at most MAX_BUCKET_SEGS = 2^10) above
// the bit index (below 2^19).
constexpr int HIT_BITS = RANGE_SEG_LOG2 - 1;
static_assert(MAX_BUCKET_SEGS <= (1 << (32 - HIT_BITS)), "segment fits above the bit index");
// Hits per LDS round of the scatter kernel (1024 threads x 4).
constexpr uint32_t BUCKET_SORT_SUB = 4096;
// Full sort tiles the layout keeps at least while it lengthens them: about
// 1.3 waves of the per-tile kernels at two 1024-thread workgroups on each of
// the 256 compute units (measured on 2^28 numbers at 2^60, 47 M hits: 2^16-hit
// tiles 0.615 ms against 0.657 with 2^15, which 768 chose there).
constexpr uint64_t SCATTER_MIN_TILES = 650;

// x mod d for integers 2^19 <= d < 2^34, in double precision with exact
// remainder arithmetic.  The reciprocal is the hardware estimate refined by
// two Newton steps (relative error a few units of 2^-53); x rounded to 53
// bits times it is within 2^-7 of x / d < 2^45, so q = floor(x * (1/d) - 1/2)
// is floor(x / d) or one less, and r = x - q d lies in [0, 2d).  r is formed
// from the exact halves xh = x - (x mod 2^32) and xl = x mod 2^32 as
// fma(-q, d, xh) + xl: the fused product-sum is exact because its result,
// r - xl, is an integer of magnitude below 2^35, and so is the sum.  One
// conditional subtraction of d ends it.
__device__ __forceinline__ double mod_double(uint64_t x, double d)
{
    const double xh = (double)(x & ~(uint64_t)0xffffffffu), xl = (double)(uint32_t)x;
    double inv = __builtin_amdgcn_rcp(d);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    const double q = floor(fma((double)x, inv, -0.5));
    const double r = fma(-q, d, xh) + xl;
    return r >= d ? r - d : r;
}

// Offset from lo of p's first odd multiple at or above lo when it is below
// len, else len (a piece holds at most 2^30 numbers, so the offset fits 32
// bits).  Bucket mode's lo exceeds its primes (lo > root), so every such
// multiple is a proper one: starting at p^2 would only skip multiples that
// a smaller prime also crosses off.
__device__ __forceinline__ uint32_t bucket_first(const BucketArgs &a, uint32_t p)
{
    // the odd multiples of p are the numbers congruent to p mod 2p: with
    // m = lo mod 2p, the first at or above lo is lo + p - m (m <= p) or
    // lo + 3p - m (all exact in double precision: below 2^35)
    const double pd = (double)p;
    const double m = mod_double(a.lo, 2.0 * pd);
    const double off = (m <= pd ? pd : 3.0 * pd) - m;
    return off < (double)a.len ? (uint32_t)off : (uint32_t)a.len;
}

// Cost of the primes below x, up to constants: one first-hit computation per
// prime (x / ln x primes) and one bucket entry per hit (len/2 * sum 1/p, which
// grows like ln ln x).  Group g takes the primes whose cumulative cost falls
// in its equal share, so the low primes with hundreds of hits each and the
// high primes with at most one are spread evenly.  (Single precision with
// the fast logarithm and quotient: the split only balances the work, and
// every split gives the same bits.)
__device__ __forceinline__ float bucket_cost(float x, float len)
{
    const float lx = __logf(x);
    return __fdividef(24.0f * x, lx) + 2.0f * len * __logf(lx);
}

// The prime bound where the cumulative cost reaches `target` (bisection
// down to the resolution of single precision).
__device__ float bucket_split(float target, float lo, float hi, float len)
{
    for (int it = 0; it < 26; ++it) {
        const float mid = 0.5f * (lo + hi);
        if (bucket_cost(mid, len) < target)
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

constexpr int BUCKET_THREADS = 1024;
// Dense prime list per wavefront and chunk of 64 table words (4096
// consecutive integers).  An interval of y >= 2 integers holds at most
// 2y / ln y primes (Montgomery and Vaughan, Mathematika 20, 1973): 985 for
// y = 4096; a chunk that still had more would take the per-lane path.
constexpr uint32_t BUCKET_PBUF = 1024;

// Each odd multiple of p in the piece appended to the group's stream: the
// lanes with a hit at a step take consecutive places in the stream, so each
// step is one contiguous store of the wavefront.
__device__ __forceinline__ void bucket_hits(const BucketArgs &a, uint32_t p, uint32_t *fill,
                                            uint64_t gbase, uint64_t gend)
{
    const uint32_t len = (uint32_t)a.len;  // at most 2^30
    const uint32_t first = bucket_first(a, p);
    if (first >= len)
        return;
    const uint32_t span = len - 1 - first;
    // K = floor(span / 2p) + 1: a single multiple when 2p > span, and
    // otherwise 2p <= span < 2^30
    uint32_t K = 1;
    if (p <= span / 2)
        K = span / (2u * p) + 1u;
    uint32_t off = first;
    for (uint32_t j = 0; j < K; ++j) {
        // one place per lane still in the loop (the compiler combines the
        // wavefront's increments into one LDS atomic and numbers the lanes
        // in order, so the places are consecutive)
        const uint64_t at = gbase + atomicAdd(fill, 1u);
        // segment off >> RANGE_SEG_LOG2 above bit index (off mod RANGE_SEG) / 2,
        // which with HIT_BITS = RANGE_SEG_LOG2 - 1 is off / 2
        if (at < gend)
            a.stream[at] = off >> 1;
        off += 2u * p;  // (only read again while j < K, when 2p < 2^30)
    }
}

// The groups' table words: wsplit[g] = the first word of group g, so that
// the groups take equal shares of the cost between BUCKET_SMALL and root
// (a choice of work split only, which changes no output bit).  One thread
// per boundary; launched with one workgroup of at least groups + 1 threads.
__global__ void __launch_bounds__(1024) bucket_split_kernel(BucketArgs a)
{
    __shared__ uint32_t wmax[16];
    const uint32_t g = threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (g < a.groups)
        a.totals[g] = 0;  // summed by the bound pass
    uint32_t w = g == 0 ? (uint32_t)a.w_begin : (uint32_t)a.w_end;
    if (g > 0 && g < a.groups) {
        const float len = (float)a.len, x0 = (float)BUCKET_SMALL, x1 = (float)a.root + 1.0f;
        const float c0 = bucket_cost(x0, len), c1 = bucket_cost(x1, len);
        const float x = bucket_split(c0 + (c1 - c0) * ((float)g / (float)a.groups), x0, x1, len);
        const uint64_t wx = (uint64_t)x >> 6;
        w = (uint32_t)(wx < a.w_begin ? a.w_begin : (wx > a.w_end ? a.w_end : wx));
    }
    // the boundaries made nondecreasing whatever the rounding (an inclusive
    // maximum scan over the threads; thread groups holds w_end, the largest)
    uint32_t m = g <= a.groups ? w : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(m, o, 64);
        if (lane >= o)
            m = max(m, y);
    }
    if (lane == 63)
        wmax[wave] = m;
    __syncthreads();
    for (int k = 0; k < wave; ++k)
        m = max(m, wmax[k]);
    if (g <= a.groups)
        a.wsplit[g] = m;
}

// Sum of v over a workgroup of up to 1024 threads (wsum: one word per
// wavefront; ends with the workgroup's threads past a barrier).
__device__ __forceinline__ uint32_t block_sum_1024(uint32_t v, uint32_t *wsum)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    if (lane == 0)
        wsum[wave] = v;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
        t += wsum[w];
    return t;
}

// Bound pass: totals[group] >= the group's hits (zeroed by the split
// kernel).  Each prime p in (BUCKET_SMALL, root] adds floor((len - 1) / 2p)
// + 1, which is 1 for p > (len - 1) / 2.  Words w_begin .. w_mid - 1 (whose
// numbers do not all exceed max(BUCKET_SMALL, (len - 1) / 2)) are taken
// prime by prime: split evenly over the first workgroups (1024 x bound_per
// words each, whatever the groups), each adding its sum over each group's
// words to that group's total.  The words from w_mid on add their prime
// counts: for each group boundary w, C(w) = the primes in the words below
// w, from the chunk counts and the popcounts of at most 63 words (one
// wavefront per boundary, in the last workgroups), added to the total of
// the group it ends and subtracted from that of the group it starts (modulo
// 2^32: every partial sum cancels); the last word is counted up to root.
constexpr uint32_t BUCKET_BOUND_PER = 8;  // the most words per thread

__device__ __forceinline__ uint32_t bucket_bound_word(const BucketArgs &a, uint32_t word,
                                                      uint64_t w, uint64_t lo_p)
{
    const uint64_t v0 = 64 * w + 1, v1 = 64 * w + 63;  // the word's first and last number
    if (v0 > lo_p && v1 <= a.root)
        return (uint32_t)__popc(word);
    uint32_t c = 0;
    while (word) {
        const int b = __ffs(word) - 1;
        word &= word - 1;
        const uint64_t p = v0 + 2 * (uint64_t)b;
        if (p > BUCKET_SMALL && p <= a.root)  // len - 1 < 2^30: 32-bit quotients
            c += (2 * p > a.len - 1 ? 0u : (uint32_t)(a.len - 1) / (uint32_t)(2 * p)) + 1u;
    }
    return c;
}

// The chunk-count part of the bound pass: one wavefront per group boundary
// g = 16 b + wavefront, g <= groups.
__device__ __forceinline__ void bucket_bound_counts(const BucketArgs &a, uint32_t b)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = b * 16 + (threadIdx.x >> 6);
    if (g > a.groups)
        return;  // (uniform per wavefront)
    // the boundary clamped to the counted words [w_mid, w_top): the last
    // word, which may hold numbers above root, is counted on its own
    const uint64_t w_top = max(a.w_mid, a.w_end - 1);
    const uint64_t w = min(max((uint64_t)a.wsplit[g], a.w_mid), w_top);
    const uint64_t c = w >> 6;
    uint32_t v = lane < (uint32_t)(w & 63) ? (uint32_t)__popc(a.table[(c << 6) + lane]) : 0u;
    if (g == a.groups && a.w_mid < a.w_end && lane == 0) {
        // word w_end - 1 holds 64 (w_end - 1) + 2i + 1 for i < 32; those up
        // to root are the first (r + 1) / 2, r = root mod 64
        const uint32_t nb = (uint32_t)((a.root & 63) + 1) >> 1;
        const uint32_t mask = nb >= 32 ? ~0u : (1u << nb) - 1u;
        atomicAdd(&a.totals[a.groups - 1], (uint32_t)__popc(a.table[a.w_end - 1] & mask));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    const uint32_t count = a.chunk_primes[c] + v;  // C(w)
    if (lane == 0) {
        if (g > 0)
            atomicAdd(&a.totals[g - 1], count);
        if (g < a.groups)
            atomicSub(&a.totals[g], count);
    }
}

__global__ void __launch_bounds__(1024) bucket_bound_kernel(BucketArgs a, uint32_t enum_blocks)
{
    __shared__ uint32_t wsum[16];
    if (blockIdx.x >= enum_blocks) {
        bucket_bound_counts(a, blockIdx.x - enum_blocks);
        return;  // (uniform)
    }
    const uint32_t per = a.bound_per;  // 1 .. BUCKET_BOUND_PER
    const uint64_t w0 = a.w_begin + (uint64_t)blockIdx.x * 1024 * per;
    if (w0 >= a.w_mid)
        return;  // (uniform)
    const uint64_t w1 = min(w0 + 1024 * per, a.w_mid);
    const uint64_t pcut = (a.len - 1) / 2;  // primes above it have at most one hit
    const uint64_t lo_p = pcut > BUCKET_SMALL ? pcut : BUCKET_SMALL;
    // every word read before any is used
    uint32_t words[BUCKET_BOUND_PER];
#pragma unroll
    for (uint32_t k = 0; k < BUCKET_BOUND_PER; ++k) {
        const uint64_t w = w0 + k * 1024 + threadIdx.x;
        words[k] = k < per && w < w1 ? a.table[w] : 0u;
    }
    uint32_t c[BUCKET_BOUND_PER];
#pragma unroll
    for (uint32_t k = 0; k < BUCKET_BOUND_PER; ++k)
        c[k] = k < per ? bucket_bound_word(a, words[k], w0 + k * 1024 + threadIdx.x, lo_p) : 0u;
    // the groups holding words w0 .. w1 - 1: q with wsplit[q] <= w < wsplit[q + 1]
    auto group_of = [&](uint64_t w) {
        uint32_t lo = 0, hi = a.groups;  // wsplit[lo] <= w < wsplit[hi] (w < w_end)
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.wsplit[mid] <= w)
                lo = mid;
            else
                hi = mid;
        }
        return lo;
    };
    const uint32_t q0 = group_of(w0), q1 = group_of(w1 - 1);
    for (uint32_t q = q0; q <= q1; ++q) {
        const uint64_t lo = max(w0, (uint64_t)a.wsplit[q]);
        const uint64_t hi = min(w1, (uint64_t)a.wsplit[q + 1]);
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t k = 0; k < BUCKET_BOUND_PER; ++k) {
            const uint64_t w = w0 + k * 1024 + threadIdx.x;
            sum += k < per && w >= lo && w < hi ? c[k] : 0u;
        }
        sum = block_sum_1024(sum, wsum);
        if (threadIdx.x == 0 && sum)
            atomicAdd(&a.totals[q], sum);
        __syncthreads();  // wsum is reused for the next group
    }
}

// Fill pass: the group's hits appended to its stretch [sbase[group],
// sbase[group + 1]) of the stream, their number to filled[group].  The
// wavefront-scope fences below order LDS accesses between the lanes of one
// wavefront (whose LDS operations complete in order) without waiting for
// its global stores.
__global__ void __launch_bounds__(BUCKET_THREADS) range_fill_kernel(BucketArgs a)
{
    __shared__ uint32_t pbuf[BUCKET_THREADS / 64][BUCKET_PBUF];
    __shared__ uint32_t fill;
    // (the clamps only keep writes inside the stream: the bounds sum to at
    // most hit_cap)
    const uint64_t gbase = min((uint64_t)a.sbase[blockIdx.x], a.hit_cap);
    const uint64_t gend = min((uint64_t)a.sbase[blockIdx.x + 1], a.hit_cap);
    if (threadIdx.x == 0)
        fill = 0;
    __syncthreads();
    const uint64_t wb = a.wsplit[blockIdx.x];
    const uint64_t we = max((uint64_t)a.wsplit[blockIdx.x + 1], wb);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nwaves = blockDim.x >> 6;
    uint32_t *buf = pbuf[wave];
    auto take = [&](uint32_t p) {
        if (p > BUCKET_SMALL && p <= a.root)
            bucket_hits(a, p, &fill, gbase, gend);
    };
    // the primes of a chunk of 64 words (w0 .. w0 + 63; lane l holds word
    // w0 + l) are listed densely in LDS (a wavefront prefix sum of the
    // words' popcounts) and then taken one per lane; all lanes active
    auto chunk = [&](uint64_t w0, uint32_t word) {
        const uint64_t w = w0 + lane;
        const uint32_t c = (uint32_t)__popc(word);
        // inclusive wavefront scan of c by data-parallel primitives: shifts
        // by 1, 2, 4, 8 lanes within each row of 16 (lanes shifted in from
        // outside a row read 0), then lane 15's sum added to rows 1 and 3
        // and lane 31's to rows 2 and 3 (row broadcasts; the rows masked off
        // add 0): six adds, no LDS round trips
        uint32_t inc = c;
        inc += __builtin_amdgcn_update_dpp(0u, inc, 0x111, 0xf, 0xf, true);   // row_shr:1
        inc += __builtin_amdgcn_update_dpp(0u, inc, 0x112, 0xf, 0xf, true);   // row_shr:2
        inc += __builtin_amdgcn_update_dpp(0u, inc, 0x114, 0xf, 0xf, true);   // row_shr:4
        inc += __builtin_amdgcn_update_dpp(0u, inc, 0x118, 0xf, 0xf, true);   // row_shr:8
        inc += __builtin_amdgcn_update_dpp(0u, inc, 0x142, 0xa, 0xf, false);  // row_bcast:15
        inc += __builtin_amdgcn_update_dpp(0u, inc, 0x143, 0xc, 0xf, false);  // row_bcast:31
        const uint32_t total = __builtin_amdgcn_readlane(inc, 63);
        if (total <= BUCKET_PBUF) {
            uint32_t at = inc - c;
            while (word) {
                const int b = __ffs(word) - 1;
                word &= word - 1;
                buf[at++] = (uint32_t)(2 * (32 * w + (uint64_t)b) + 1);
            }
            // the list is read by the other lanes of the wavefront
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (uint32_t i = lane; i < total; i += 64)
                take(buf[i]);
            // and overwritten by the next chunk
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            while (word) {
                const int b = __ffs(word) - 1;
                word &= word - 1;
                take((uint32_t)(2 * (32 * w + (uint64_t)b) + 1));
            }
        }
    };
    // each chunk's words are loaded while the chunk before is processed
    const uint64_t nch = we > wb ? (we - wb + 63) / 64 : 0;
    auto load = [&](uint64_t ch) {
        const uint64_t w = wb + 64 * ch + lane;
        return ch < nch && w < we ? a.table[w] : 0u;
    };
    uint32_t next = load(wave);
    for (uint64_t ch = wave; ch < nch; ch += nwaves) {
        const uint32_t word = next;
        next = load(ch + nwaves);
        chunk(wb + 64 * ch, word);
    }
    __syncthreads();
    if (threadIdx.x == 0)
        a.filled[blockIdx.x] = fill < gend - gbase ? fill : (uint32_t)(gend - gbase);
}

// One workgroup of 1024 threads: sbase = the exclusive scan of the groups'
// totals (their stretches of the stream), tprefix = that of their tile
// counts ceil(total / tile); both with the sum at [groups].
__global__ void __launch_bounds__(1024) bucket_plan_kernel(BucketArgs a)
{
    __shared__ uint32_t wsum[2][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t q = threadIdx.x;
    const uint32_t h = q < a.groups ? a.totals[q] : 0u;
    const uint32_t t = (h + a.tile - 1) / a.tile;
    uint32_t ih = h, it = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t yh = __shfl_up(ih, o, 64), yt = __shfl_up(it, o, 64);
        if (lane >= o) {
            ih += yh;
            it += yt;
        }
    }
    if (lane == 63) {
        wsum[0][wave] = ih;
        wsum[1][wave] = it;
    }
    __syncthreads();
    uint32_t bh = 0, bt = 0;
    for (int w = 0; w < wave; ++w) {
        bh += wsum[0][w];
        bt += wsum[1][w];
    }
    if (q < a.groups) {
        a.sbase[q] = bh + ih - h;
        a.tprefix[q] = bt + it - t;
    }
    if (q == a.groups - 1) {
        a.sbase[a.groups] = bh + ih;
        a.tprefix[a.groups] = bt + it;
    }
}

// The (group, tile) of per-tile workgroup b, or false past the last tile:
// the group q with tprefix[q] <= b < tprefix[q + 1] (binary search).
__device__ __forceinline__ bool bucket_tile_of(const BucketArgs &a, uint32_t b, uint32_t &q,
                                               uint32_t &t, uint32_t &nt)
{
    if (b >= a.tprefix[a.groups])
        return false;
    uint32_t lo = 0, hi = a.groups;  // tprefix[lo] <= b < tprefix[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.tprefix[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    q = lo;
    t = b - a.tprefix[q];
    nt = a.tprefix[q + 1] - a.tprefix[q];
    return true;
}

// Index of the count of segment g in tile b (b: the tile's index over all
// groups, tprefix[q] + t) in tcounts: segment-major, so that the flat scan
// puts every segment's hits together, in the order of the tiles (and so of
// the groups) within it.
__device__ __forceinline__ uint64_t bucket_count_at(const BucketArgs &a, uint32_t g, uint32_t b)
{
    return (uint64_t)g * a.max_tiles + b;
}

// Histogram pass: per tile, its hits per segment, stored at their
// (segment, tile) place; workgroups past the last tile store zeros in their
// column, so that the scan reads a fully written array.
__global__ void __launch_bounds__(1024) bucket_hist_kernel(BucketArgs a)
{
    __shared__ uint32_t hist[MAX_BUCKET_SEGS];
    const uint32_t nseg = a.nseg;
    for (uint32_t g = threadIdx.x; g < nseg; g += blockDim.x)
        hist[g] = 0;
    __syncthreads();
    uint32_t q, t, nt;
    if (!bucket_tile_of(a, blockIdx.x, q, t, nt)) {
        for (uint32_t g = threadIdx.x; g < nseg; g += blockDim.x)
            a.tcounts[bucket_count_at(a, g, blockIdx.x)] = 0;
        return;
    }
    const uint64_t t0 = (uint64_t)a.sbase[q] + (uint64_t)t * a.tile;
    const uint64_t t1 = min((uint64_t)a.sbase[q] + a.filled[q], t0 + a.tile);
    // eight entries per thread and round, all read before any is counted
    constexpr int UNROLL = 8;
    for (uint64_t i0 = t0 + threadIdx.x; i0 < t1; i0 += (uint64_t)UNROLL * blockDim.x) {
        uint32_t v[UNROLL];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            const uint64_t i = i0 + (uint64_t)k * blockDim.x;
            v[k] = i < t1 ? a.stream[i] : ~0u;
        }
#pragma unroll
        for (int k = 0; k < UNROLL; ++k)
            if (v[k] != ~0u)
                atomicAdd(&hist[min(v[k] >> HIT_BITS, nseg - 1)], 1u);
    }
    __syncthreads();
    for (uint32_t g = threadIdx.x; g < nseg; g += blockDim.x)
        a.tcounts[bucket_count_at(a, g, blockIdx.x)] = hist[g];
}

// Starts: hs[g] = the scanned count of (segment g, tile 0), the first place
// of segment g's hits, and hs[nseg] = the total.
__global__ void __launch_bounds__(256) bucket_starts_kernel(BucketArgs a)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g <= a.nseg)
        a.hs[g] = a.tcounts[(uint64_t)g * a.max_tiles];  // [nseg * max_tiles]: the total
}

// Scatter pass: per tile, in rounds of BUCKET_SORT_SUB hits: counted by
// segment (LDS atomics), scanned, put in segment order in LDS and written
// out so that consecutive threads write consecutive places of one bucket;
// each segment's cursor starts at the tile's scanned count and moves past
// each round's hits.  The order of hits within a bucket is free (the sieve
// clears each hit's bit).  Launched with 1024 threads (nseg <=
// MAX_BUCKET_SEGS).
__global__ void __launch_bounds__(1024, 8) bucket_scatter_kernel(BucketArgs a)
{
    // Double-buffered per round (b = the round's parity): cnt[b] counts the
    // round's hits per segment, off[b] is its exclusive scan, cur[b] each
    // segment's next place.  Round r touches cnt/off/cur[b] and prepares
    // cnt[b ^ 1] (zeroed) and cur[b ^ 1] (advanced); with the buffers of the
    // next round apart, three barriers per round order every access.
    __shared__ uint32_t cnt[2][MAX_BUCKET_SEGS];
    __shared__ uint32_t off[2][MAX_BUCKET_SEGS];
    __shared__ uint32_t cur[2][MAX_BUCKET_SEGS];
    __shared__ uint32_t sorted[BUCKET_SORT_SUB];
    constexpr int PER = BUCKET_SORT_SUB / 1024;
    constexpr int SCAN_PER = MAX_BUCKET_SEGS / 64;  // segments per lane of the one-wavefront scan
    static_assert(MAX_BUCKET_SEGS % 64 == 0, "the scan's lanes cover the segments");
    uint32_t q, t, nt;
    if (!bucket_tile_of(a, blockIdx.x, q, t, nt))
        return;
    const uint32_t nseg = a.nseg;  // <= MAX_BUCKET_SEGS
    const uint32_t mask = (1u << HIT_BITS) - 1u;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t g = threadIdx.x; g < nseg; g += blockDim.x) {
        cur[0][g] = a.tcounts[bucket_count_at(a, g, blockIdx.x)];
        cnt[0][g] = 0;
        cnt[1][g] = 0;
    }
    const uint64_t b0 = (uint64_t)a.sbase[q] + (uint64_t)t * a.tile;
    const uint64_t b1 = min((uint64_t)a.sbase[q] + a.filled[q], b0 + a.tile);
    // each round's hits are loaded while the round before is sorted, as
    // streaming loads (their last use: with these and the segment kernel's,
    // 2^63: 0.911 -> 0.888 ms for 2^28 numbers)
    uint32_t next[PER];
    auto load = [&](uint64_t r0) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint64_t i = r0 + threadIdx.x + k * blockDim.x;
            next[k] = i < b1 ? __builtin_nontemporal_load(&a.stream[i]) : 0u;
        }
    };
    load(b0);
    __syncthreads();
    uint32_t b = 0;
    for (uint64_t r0 = b0; r0 < b1; r0 += BUCKET_SORT_SUB, b ^= 1u) {
        const uint32_t n = (uint32_t)min((uint64_t)BUCKET_SORT_SUB, b1 - r0);
        uint32_t v[PER], rank[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k)
            v[k] = next[k];
        load(r0 + BUCKET_SORT_SUB);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t i = threadIdx.x + k * blockDim.x;
            rank[k] = 0;
            if (i < n) {
                // (the clamp only keeps LDS indices inside the arrays: every
                // entry was written by the fill pass with its segment)
                v[k] = min(v[k] >> HIT_BITS, nseg - 1) << HIT_BITS | (v[k] & mask);
                rank[k] = atomicAdd(&cnt[b][v[k] >> HIT_BITS], 1u);
            }
        }
        __syncthreads();  // the round's counts are in cnt[b]
        if (wave == 0) {
            // exclusive scan of cnt[b] into off[b], SCAN_PER consecutive
            // segments per lane
            const uint32_t g0 = (uint32_t)lane * SCAN_PER;
            uint32_t c[SCAN_PER], local = 0;
#pragma unroll
            for (int j = 0; j < SCAN_PER; ++j) {
                c[j] = g0 + j < nseg ? cnt[b][g0 + j] : 0u;
                local += c[j];
            }
            uint32_t incl = local;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= o)
                    incl += y;
            }
            uint32_t run = incl - local;
#pragma unroll
            for (int j = 0; j < SCAN_PER; ++j) {
                if (g0 + j < nseg)
                    off[b][g0 + j] = run;
                run += c[j];
            }
        }
        __syncthreads();  // off[b]: each segment's offset in this round
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t i = threadIdx.x + k * blockDim.x;
            if (i < n)
                sorted[off[b][v[k] >> HIT_BITS] + rank[k]] = v[k];
        }
        for (uint32_t g = threadIdx.x; g < nseg; g += blockDim.x)
            cnt[b ^ 1u][g] = 0;  // the next round counts from zero
        __syncthreads();  // the round is in segment order
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint32_t i = threadIdx.x + k * blockDim.x;
            if (i < n) {
                const uint32_t w = sorted[i];
                const uint32_t g = w >> HIT_BITS;
                const uint64_t at = (uint64_t)cur[b][g] + (i - off[b][g]);
                if (at < a.hit_cap)
                    a.hits[at] = w & mask;
            }
        }
        for (uint32_t g = threadIdx.x; g < nseg; g += blockDim.x)
            cur[b ^ 1u][g] = cur[b][g] + cnt[b][g];
    }
}

// Exclusive scan of counts[0 .. n) in place, total at counts[n], in three
// passes over tiles of SCAN_TILE words: tile sums, a scan of the sums (one
// workgroup), then each tile scanned and offset.
constexpr int SCAN_TILE = 8192;  // 1024 threads x 8


__global__ void __launch_bounds__(1024) scan_tile_sums(const uint32_t *counts, uint32_t n,
                                                      uint32_t *sums)
{
    __shared__ uint32_t wsum[16];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t v = 0;
    for (int k = 0; k < SCAN_TILE / 1024; ++k) {
        const uint64_t i = base + (uint64_t)k * blockDim.x + threadIdx.x;
        if (i < n)
            v += counts[i];
    }
    const uint32_t t = block_sum_1024(v, wsum);
    if (threadIdx.x == 0)
        sums[blockIdx.x] = t;
}

// Exclusive scan of up to 1024 values in place (one workgroup); total at [m].
__global__ void __launch_bounds__(1024) scan_small(uint32_t *v, uint32_t m)
{
    __shared__ uint32_t wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t x = threadIdx.x < m ? v[threadIdx.x] : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += y;
    }
    if (lane == 63)
        wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w)
        before += wsum[w];
    if (threadIdx.x < m)
        v[threadIdx.x] = before + incl - x;
    if (threadIdx.x == blockDim.x - 1)
        v[m] = before + incl;
}

__global__ void __launch_bounds__(1024) scan_tiles(uint32_t *counts, uint32_t n,
                                                  const uint32_t *sums)
{
    __shared__ uint32_t wsum[16];
    constexpr int PER = SCAN_TILE / 1024;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // thread t owns the PER consecutive words t*PER .. of the tile
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * PER;
    uint32_t x[PER], local = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        x[k] = base + k < n ? counts[base + k] : 0u;
        local += x[k];
    }
    uint32_t incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += y;
    }
    if (lane == 63)
        wsum[wave] = incl;
    __syncthreads();
    uint32_t run = sums[blockIdx.x] + incl - local;
    for (int w = 0; w < wave; ++w)
        run += wsum[w];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (base + k < n)
            counts[base + k] = run;
        run += x[k];
    }
    const uint32_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (blockIdx.x == ntiles - 1 && threadIdx.x == blockDim.x - 1)
        counts[n] = run;  // the total
}

}  // namespace

namespace {

// Chunk c's odd primes (the popcount of table words 64c .. 64c + 63): one
// wavefront per chunk.
__global__ void __launch_bounds__(256) chunk_popc_kernel(const uint32_t *table, uint32_t *cnt)
{
    const uint64_t c = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    if (c >= TABLE_CHUNKS)
        return;  // (uniform per wavefront)
    uint32_t v = (uint32_t)__popc(table[(c << 6) + lane]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    if (lane == 0)
        cnt[c] = v;
}

constexpr uint32_t CHUNK_SCAN_TILES = (uint32_t)((TABLE_CHUNKS + SCAN_TILE - 1) / SCAN_TILE);
static_assert(CHUNK_SCAN_TILES <= 1024, "one workgroup scans the tile sums");

}  // namespace

size_t chunk_primes_words() { return TABLE_CHUNKS + 1 + CHUNK_SCAN_TILES + 1; }

hipError_t launch_chunk_primes(DeviceState &ds, hipStream_t s)
{
    uint32_t *cnt = ds.chunk_primes, *sums = cnt + TABLE_CHUNKS + 1;
    const uint32_t n = (uint32_t)TABLE_CHUNKS;
    chunk_popc_kernel<<<(unsigned)(TABLE_CHUNKS * 64 / 256), 256, 0, s>>>(ds.table, cnt);
    scan_tile_sums<<<CHUNK_SCAN_TILES, 1024, 0, s>>>(cnt, n, sums);
    scan_small<<<1, 1024, 0, s>>>(sums, CHUNK_SCAN_TILES);
    scan_tiles<<<CHUNK_SCAN_TILES, 1024, 0, s>>>(cnt, n, sums);
    return hipGetLastError();
}

namespace {

// The piece's sieving primes: res[k] = {primes[k], floor(2^32 / primes[k]),
// base mod primes[k]} for k < count.
__global__ void __launch_bounds__(256) range_residue_kernel(uint64_t base,
                                                           const uint32_t *__restrict__ primes,
                                                           const uint64_t *__restrict__ inv,
                                                           uint32_t count, SievePrime *__restrict__ res)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) {
        const uint32_t p = primes[k];
        const uint64_t q = inv[k];
        // the high word of floor((2^64 - 1) / p) is floor(2^32 / p) (p odd)
        res[k] = SievePrime{p, (uint32_t)(q >> 32), (uint32_t)mod_small(base, p, q)};
    }
}

}  // namespace

hipError_t launch_range_residues(uint64_t lo, uint64_t bound, const DeviceState &ds,
                                 SievePrime *res, hipStream_t s)
{
    // at most pi(bound) < 1.25506 bound / ln bound primes (Rosser and
    // Schoenfeld, Illinois J. Math. 6, 1962), all of them below 100
    uint64_t count = bound < 100 ? 25 : (uint64_t)(1.25506 * (double)bound / std::log((double)bound)) + 1;
    count = std::min<uint64_t>(count, (uint64_t)ds.num_range_primes);
    if (!res || count == 0)
        return hipErrorInvalidValue;
    range_residue_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(
        lo | 1, ds.range_primes, ds.range_inv, (uint32_t)count, res);
    return hipGetLastError();
}

hipError_t launch_range_primes(DeviceState &ds, hipStream_t s)
{
    range_count_kernel<<<RANGE_LIST_GROUPS, 256, 0, s>>>(ds.table, ds.range_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    range_list_kernel<<<RANGE_LIST_GROUPS, 256, 0, s>>>(ds.table, ds.range_count,
                                                        ds.range_primes, ds.range_inv);
    return hipGetLastError();
}

hipError_t launch_range_table(uint64_t lo, uint8_t *out, uint64_t len, const DeviceState &ds,
                              hipStream_t s)
{
    const uint64_t threads = (len + 4095) / 4096 * 64;  // one wavefront per 4096 numbers
    const uint64_t blocks = (threads + 255) / 256;
    if (blocks > 0x7fffffffull)
        return hipErrorInvalidValue;
    range_table_kernel<<<(unsigned)blocks, 256, 0, s>>>(lo, out, len, ds.table);
    return hipGetLastError();
}

BucketLayout bucket_layout(uint32_t nseg, unsigned groups, uint64_t hit_cap, uint64_t len,
                           uint64_t root)
{
    BucketLayout L{};
    // Tiles of 8 or 16 rounds (a power-of-two multiple of BUCKET_SORT_SUB):
    // 16 while at least SCATTER_MIN_TILES full tiles of 16 remain, and longer
    // only until the count array fits the three-pass scan (at most 1024 scan
    // tiles).  Longer tiles leave fewer counts and partial lines (measured at
    // 2^63: 2^14-hit tiles 1.46 ms and 866 MiB written per 2^28 numbers,
    // 2^16-hit tiles 1.37 ms and 732 MiB); enough tiles keep the scatter's
    // workgroups balanced (2^28 numbers at 2^50, 30 M hits: 2^15-hit tiles
    // 0.417 ms against 0.455 with 2^16; at 2^63, 61 M hits, 2^16 against 2^15:
    // 0.903 against 0.939 ms; tiles of 2^18 for the 2^30-number piece below
    // 2^64: 3.18 against 3.07 ms with 2^16).
    auto words = [&](uint64_t tile, uint64_t &max_tiles) {
        max_tiles = (hit_cap + tile - 1) / tile + groups;
        return (uint64_t)nseg * max_tiles;
    };
    // (the tiles counted from the expected hits, len / 2 times the sum of 1/p
    // over the primes in (BUCKET_SMALL, root], about len / 2 (ln ln root -
    // ln ln BUCKET_SMALL) by Mertens: hit_cap also bounds one hit per prime)
    const double lr = std::log(std::log((double)std::max<uint64_t>(root, BUCKET_SMALL + 1)));
    const double hits = 0.5 * (double)len * std::max(0.0, lr - std::log(std::log((double)BUCKET_SMALL)));
    uint64_t tile = 8 * BUCKET_SORT_SUB, max_tiles = 0;
    if (hits / (double)(2 * tile) >= (double)SCATTER_MIN_TILES)
        tile *= 2;
    while (tile < ((uint64_t)1 << 24) && words(tile, max_tiles) > (uint64_t)SCAN_TILE * 1024)
        tile *= 2;
    const uint64_t n2 = words(tile, max_tiles);
    if (n2 <= (uint64_t)SCAN_TILE * 1024) {
        L.tile = (uint32_t)tile;
        L.max_tiles = (uint32_t)max_tiles;
        const uint64_t ntiles = (n2 + SCAN_TILE - 1) / SCAN_TILE;
        // starts, wsplit, totals, filled, sbase, tprefix, counts + total,
        // scan sums + total
        L.count_words = (uint64_t)nseg + 1 + 2 * (uint64_t)groups +
                        3 * ((uint64_t)groups + 1) + n2 + 1 + ntiles + 1;
        L.ok = true;
    }
    return L;
}

hipError_t launch_range_buckets(uint64_t lo, uint64_t len, uint64_t root, unsigned groups,
                                uint64_t hit_bound, const DeviceState &ds, const RangeWs &rw,
                                hipStream_t s)
{
    BucketArgs a;
    a.lo = lo;
    a.len = len;
    a.root = root;
    a.table = ds.table;
    a.w_begin = (BUCKET_SMALL + 1) >> 6;
    a.w_end = (root >> 6) + 1;
    // the first word whose numbers all exceed max(BUCKET_SMALL, (len - 1) / 2)
    const uint64_t lo_p = std::max<uint64_t>((len - 1) / 2, BUCKET_SMALL);
    a.w_mid = std::min(a.w_end, std::max(a.w_begin, (lo_p >> 6) + 1));
    a.chunk_primes = ds.chunk_primes;
    a.nseg = (uint32_t)((len + RANGE_SEG - 1) / RANGE_SEG);
    a.groups = groups;
    a.hits = rw.hits;
    a.stream = rw.stream;
    a.hit_cap = hit_bound;  // the layout's room; the buffers may hold more
    if (a.nseg > (uint32_t)MAX_BUCKET_SEGS || a.w_end > (uint64_t)TABLE_WORDS ||
        a.w_end <= a.w_begin || groups == 0 || groups > (unsigned)MAX_BUCKET_GROUPS ||
        hit_bound > rw.hit_cap || hit_bound >= ((uint64_t)1 << 32) || !ds.chunk_primes ||
        lo <= root)
        return hipErrorInvalidValue;
    const BucketLayout L = bucket_layout(a.nseg, groups, hit_bound, len, root);
    if (!L.ok || rw.count_cap < L.count_words)
        return hipErrorInvalidValue;
    a.tile = L.tile;
    a.max_tiles = L.max_tiles;
    const uint64_t n2 = (uint64_t)a.nseg * L.max_tiles;
    const uint32_t ntiles = (uint32_t)((n2 + SCAN_TILE - 1) / SCAN_TILE);
    uint32_t *w = rw.counts;
    a.hs = w;  // first: the segment kernel reads the starts at the workspace's base
    w += (uint64_t)a.nseg + 1;
    a.wsplit = w;
    w += groups + 1;
    a.totals = w;
    w += groups;
    a.filled = w;
    w += groups;
    a.sbase = w;
    w += groups + 1;
    a.tprefix = w;
    w += groups + 1;
    a.tcounts = w;
    w += n2 + 1;
    uint32_t *sums = w;  // ntiles + 1
    hipError_t e = hipSuccess;
    auto step = [&](auto launch) {
        if (e == hipSuccess) {
            launch();
            e = hipGetLastError();
        }
    };
    step([&] { bucket_split_kernel<<<1, 1024, 0, s>>>(a); });
    // the bound pass: the words taken prime by prime at most
    // BUCKET_BOUND_PER per thread, and over at least 1024 workgroups while
    // they allow; then one wavefront per group boundary
    const uint64_t words = a.w_mid - a.w_begin;
    a.bound_per = (uint32_t)std::min<uint64_t>(
        BUCKET_BOUND_PER, std::max<uint64_t>(1, (words + 1024 * 1024 - 1) / (1024 * 1024)));
    const unsigned enum_blocks = (unsigned)((words + 1024 * a.bound_per - 1) / (1024 * a.bound_per));
    const unsigned count_blocks = (groups + 1 + 15) / 16;
    step([&] { bucket_bound_kernel<<<enum_blocks + count_blocks, 1024, 0, s>>>(a, enum_blocks); });
    step([&] { bucket_plan_kernel<<<1, 1024, 0, s>>>(a); });
    step([&] { range_fill_kernel<<<groups, BUCKET_THREADS, 0, s>>>(a); });
    step([&] { bucket_hist_kernel<<<L.max_tiles, 1024, 0, s>>>(a); });
    step([&] { scan_tile_sums<<<ntiles, 1024, 0, s>>>(a.tcounts, (uint32_t)n2, sums); });
    step([&] { scan_small<<<1, 1024, 0, s>>>(sums, ntiles); });
    step([&] { scan_tiles<<<ntiles, 1024, 0, s>>>(a.tcounts, (uint32_t)n2, sums); });
    step([&] { bucket_starts_kernel<<<(a.nseg + 1 + 255) / 256, 256, 0, s>>>(a); });
    step([&] { bucket_scatter_kernel<<<L.max_tiles, 1024, 0, s>>>(a); });
    return e;
}

hipError_t launch_range_sieve(uint64_t lo, uint8_t *out, uint64_t len, unsigned grid,
                              uint64_t chunk, unsigned groups, const DeviceState &ds,
                              const Workspace &ws, const RangeWs &rw, hipStream_t s,
                              int partial_log2, int complete_log2)
{
    // (lo >= 2^32 keeps every sieving prime, below 2^25, out of the piece;
    // an even chunk keeps o0 = (lo | 1) + segment offset)
    if (partial_log2 < 17 || partial_log2 > RANGE_PARTIAL_LOG2 || complete_log2 < partial_log2 ||
        complete_log2 > RANGE_PRIME_LOG2 || lo < TABLE_BOUND || chunk > RANGE_SEG || (chunk & 1) ||
        !rw.res || len > RANGE_PIECE)
        return hipErrorInvalidValue;
    RangeArgs a;
    a.partial_log2 = (uint32_t)partial_log2;
    a.complete_log2 = (uint32_t)complete_log2;
    a.lo = lo;
    a.len = len;
    a.chunk = chunk;
    a.hit_start = rw.counts;
    a.hit_cap = rw.hit_cap;
    a.hits = rw.hits;
    a.groups = groups;
    a.out = out;
    a.primes = ds.range_primes;
    a.res = rw.res;
    a.nprimes = (uint32_t)ds.num_range_primes;
    a.surv = ws.surv;
    a.counts = ws.counts;
    // bucket mode: one workgroup per segment of RANGE_SEG numbers, as the
    // bucket passes counted them
    if (groups != 0 && (chunk != RANGE_SEG || grid != (len + RANGE_SEG - 1) / RANGE_SEG))
        return hipErrorInvalidValue;
    range_sieve_kernel<<<grid, RANGE_THREADS, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace isp
