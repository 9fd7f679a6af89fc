// range.hip -- primality of every integer in a contiguous interval
// [lo, lo + len), without an input array.
//
// Paper: section 6.1.3 sieves all primes up to the maximum once and then
// only tests membership; section 1 describes the sieve of Eratosthenes.
// For an interval that is the natural way to work: the part below 2^32 is
// copied out of the device table, bit by bit; above it, each workgroup sieves
// one segment of the interval in LDS by the odd primes up to
// min(2^20, sqrt(segment end)).  When those primes reach the square root
// (segment end <= 2^40) the survivors are exactly the primes; otherwise the
// survivors (about 4% of the numbers: those with no factor below 2^20) go to
// the same two Miller-Rabin kernels as array inputs, through the same
// per-workgroup regions and counts.
//
// Segment layout: workgroup g covers numbers [lo + g*chunk, lo + (g+1)*chunk)
// with chunk = classify_chunk(len, grid) (a multiple of 64, at most
// RANGE_SEG + 63); bit j of its LDS bitset stands for the odd number o0 + 2j.
// Crossing off: primes below 8192 by whole wavefronts (lane l takes the
// multiples l, l+64, ...), larger primes one per thread.  The first odd
// multiple of p at or above max(o0, p^2) needs o0 mod p, taken with a
// precomputed floor((2^64 - 1) / p) (one 64-bit multiply-high, no division).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace isp {

namespace {

constexpr int RANGE_THREADS = 512;
constexpr uint32_t WAVE_PRIME_LIMIT = 8192;  // primes below this: wavefront per prime

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

// Odd primes below 2^20 from the device table (bits of odd numbers below
// 2^20 are the first 2^14 words), in order, with their reciprocals.  One
// workgroup of 1024 threads, 16 words each.
__global__ void __launch_bounds__(1024) range_primes_kernel(const uint32_t *__restrict__ table,
                                                            uint32_t *__restrict__ primes,
                                                            uint64_t *__restrict__ inv,
                                                            uint32_t *__restrict__ count)
{
    __shared__ uint32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int w0 = tid * 16;
    uint32_t c = 0;
    for (int k = 0; k < 16; ++k)
        c += __popc(table[w0 + k]);
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += y;
    }
    if (lane == 63)
        wsum[wave] = incl;
    __syncthreads();
    uint32_t pos = incl - c;
    for (int w = 0; w < wave; ++w)
        pos += wsum[w];
    for (int k = 0; k < 16; ++k) {
        const uint32_t word = table[w0 + k];
        for (int b = 0; b < 32; ++b) {
            if ((word >> b) & 1) {
                const uint32_t p = 2u * (32u * (uint32_t)(w0 + k) + (uint32_t)b) + 1u;
                primes[pos] = p;
                inv[pos] = ~(uint64_t)0 / p;
                ++pos;
            }
        }
    }
    if (tid == blockDim.x - 1)
        *count = pos;
}

// out[i] = primality of lo + i for lo + len <= 2^32: one table bit per odd number.
__global__ void range_table_kernel(uint64_t lo, uint8_t *__restrict__ out, uint64_t len,
                                   const uint32_t *__restrict__ table)
{
    const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
    if (i0 >= len)
        return;
    const uint64_t i1 = i0 + 16 < len ? i0 + 16 : len;
    uint8_t r[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint64_t v = lo + i0 + j;
        uint8_t b = 0;
        if (i0 + j < i1) {
            if (v == 2)
                b = 1;
            else if ((v & 1) && v > 1)
                b = (uint8_t)((table[v >> 6] >> ((v >> 1) & 31)) & 1u);
        }
        r[j] = b;
    }
    if (i1 - i0 == 16) {
        typedef uint32_t u32u __attribute__((aligned(1)));
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<u32u *>(out + i0 + 4 * q) =
                (uint32_t)r[4 * q] | ((uint32_t)r[4 * q + 1] << 8) |
                ((uint32_t)r[4 * q + 2] << 16) | ((uint32_t)r[4 * q + 3] << 24);
    } else {
        for (uint64_t i = i0; i < i1; ++i)
            out[i] = r[i - i0];
    }
}

struct RangeArgs {
    uint64_t lo;         // first number of this piece (>= 2^32)
    uint64_t len;        // numbers in this piece
    uint8_t *out;        // out[i] <-> lo + i
    const uint32_t *primes;
    const uint64_t *inv;
    uint32_t nprimes;
    Survivor *surv;      // grid regions of classify_chunk(len, grid) entries
    uint32_t *counts;    // [grid]
};

// Integer square root of x < 2^64 (floor), from a double estimate.
__device__ __forceinline__ uint64_t isqrt64(uint64_t x)
{
    uint64_t r = (uint64_t)sqrt((double)x);
    if (r > 0xffffffffull)
        r = 0xffffffffull;
    while (r * r > x)
        --r;
    while (r < 0xffffffffull && (r + 1) * (r + 1) <= x)
        ++r;
    return r;
}

__global__ void __launch_bounds__(RANGE_THREADS) range_sieve_kernel(RangeArgs a)
{
    __shared__ uint32_t bits[(RANGE_SEG + 64) / 64 + 1];  // odd numbers of the segment
    __shared__ uint32_t wsum[RANGE_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const uint64_t chunk = classify_chunk(a.len, gridDim.x);
    const uint64_t r0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t r1 = r0 + chunk < a.len ? r0 + chunk : a.len;
    if (r0 >= r1) {
        if (tid == 0)
            a.counts[blockIdx.x] = 0;
        return;
    }
    const uint64_t s_lo = a.lo + r0;          // first number of the segment
    const uint64_t s_last = a.lo + r1 - 1;    // last number (no overflow: <= 2^64 - 1)
    const uint64_t o0 = s_lo | 1;             // first odd number
    const uint32_t nbits = o0 > s_last ? 0u : (uint32_t)((s_last - o0) / 2 + 1);
    // (o0 <= s_last whenever the segment holds an odd number; o0 = s_lo | 1
    // cannot wrap because s_lo <= s_last <= 2^64 - 1 and a wrap needs s_lo = 2^64 - 1,
    // which is odd)
    const uint32_t nwords = (nbits + 31) / 32;
    for (uint32_t w = tid; w < nwords; w += blockDim.x)
        bits[w] = w + 1 < nwords || (nbits & 31) == 0 ? 0xffffffffu : (1u << (nbits & 31)) - 1u;
    __syncthreads();
    const uint64_t root = isqrt64(s_last);
    // primes up to min(2^20, root); the list is sorted, so stop at the first above
    uint32_t np = a.nprimes;
    {
        uint32_t lo_i = 0, hi_i = np;  // first index with prime > root
        while (lo_i < hi_i) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if ((uint64_t)a.primes[mid] <= root)
                lo_i = mid + 1;
            else
                hi_i = mid;
        }
        np = lo_i;
    }
    // every prime up to the root is in the list when the root is below 2^20
    const bool complete = root < ((uint64_t)1 << 20);
    // first bit index of the odd multiples of p at or above max(o0, p^2), or
    // "none" (all offsets are taken from o0, so nothing wraps near 2^64)
    const uint64_t span = s_last - o0;  // valid only when nbits > 0
    auto first_bit = [&](uint32_t k, uint32_t p) -> uint64_t {
        const uint64_t pp = (uint64_t)p * p;  // < 2^40, odd
        uint64_t off;
        if (pp >= o0) {
            off = pp - o0;
        } else {
            const uint64_t r = mod_small(o0, p, a.inv[k]);
            off = r ? p - r : 0;  // o0 + off: first multiple of p at or above o0
            if (off & 1)
                off += p;         // o0 is odd: an odd offset gives an even multiple
        }
        return off > span ? ~(uint64_t)0 : off >> 1;
    };
    // small primes: one wavefront per prime
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
    for (uint32_t k = wave; k < k_split; k += nwaves) {
        const uint32_t p = a.primes[k];
        const uint64_t j0 = first_bit(k, p);
        if (j0 >= nbits)
            continue;
        for (uint64_t j = j0 + (uint64_t)lane * p; j < nbits; j += 64ull * p)
            atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
    }
    // larger primes: one thread per prime
    for (uint32_t k = k_split + tid; k < np; k += blockDim.x) {
        const uint32_t p = a.primes[k];
        for (uint64_t j = first_bit(k, p); j < nbits; j += p)
            atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
    }
    __syncthreads();
    // outputs: 8 consecutive numbers per thread per pass; survivors of an
    // incomplete sieve go to the Miller-Rabin kernels (out = 0 until then)
    Survivor *region = a.surv + r0;
    uint32_t filled = 0;
    for (uint64_t p0 = r0; p0 < r1; p0 += 8ull * blockDim.x) {
        const uint64_t i0 = p0 + 8ull * tid;
        uint8_t r[8];
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            r[j] = 0;
            const uint64_t i = i0 + j;
            if (i < r1) {
                const uint64_t v = a.lo + i;
                if (v & 1) {
                    const uint64_t b = (v - o0) >> 1;
                    const bool sv = (bits[b >> 5] >> (b & 31)) & 1u;
                    if (sv && complete)
                        r[j] = 1;
                    cnt += sv && !complete;
                }
            }
        }
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
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t i = i0 + j;
            if (i < r1) {
                a.out[i] = r[j];
                const uint64_t v = a.lo + i;
                if (!complete && (v & 1)) {
                    const uint64_t b = (v - o0) >> 1;
                    if ((bits[b >> 5] >> (b & 31)) & 1u) {
                        Survivor s;
                        s.n = v;
                        s.out = a.out + i;
                        region[pos++] = s;
                    }
                }
            }
        }
        filled += all;
        __syncthreads();  // wsum is rewritten next pass
    }
    if (tid == 0)
        a.counts[blockIdx.x] = filled;
}

}  // namespace

hipError_t launch_range_primes(DeviceState &ds, hipStream_t s)
{
    range_primes_kernel<<<1, 1024, 0, s>>>(ds.table, ds.range_primes, ds.range_inv,
                                           ds.range_count);
    return hipGetLastError();
}

hipError_t launch_range_table(uint64_t lo, uint8_t *out, uint64_t len, const DeviceState &ds,
                              hipStream_t s)
{
    const uint64_t threads = (len + 15) / 16;
    const uint64_t blocks = (threads + 255) / 256;
    if (blocks > 0x7fffffffull)
        return hipErrorInvalidValue;
    range_table_kernel<<<(unsigned)blocks, 256, 0, s>>>(lo, out, len, ds.table);
    return hipGetLastError();
}

hipError_t launch_range_sieve(uint64_t lo, uint8_t *out, uint64_t len, unsigned grid,
                              const DeviceState &ds, const Workspace &ws, hipStream_t s)
{
    RangeArgs a;
    a.lo = lo;
    a.len = len;
    a.out = out;
    a.primes = ds.range_primes;
    a.inv = ds.range_inv;
    a.nprimes = (uint32_t)ds.num_range_primes;
    a.surv = ws.surv;
    a.counts = ws.counts;
    range_sieve_kernel<<<grid, RANGE_THREADS, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace isp
