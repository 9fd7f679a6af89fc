// sieve.hip -- the device-resident odd-only sieve table for n < 2^32, and the
// small constant tables derived from it.
//
// Paper: section 1 describes the sieve of Eratosthenes (cross off the
// multiples of each prime); section 4 restricts candidates to odd numbers
// (the 2-wheel); section 6.1.3 sieves once up to the maximum and then only
// tests membership.  Here the sieve runs once per device up to 2^32 and
// membership is a single bit.
//
// Layout: uint32_t table[2^26]; bit (i & 31) of word (i >> 5) is 1 iff the
// odd number 2i+1 is prime.  256 MiB in HBM, read-only after the build.
//
// Kernels:
//   base_primes_kernel  one workgroup sieves the 32768 odd numbers below 2^16
//                       in LDS and writes the 6541 odd primes in order.
//   wheel_table_kernel  the same bits again on the 2*3*5*7 wheel (48 bits per
//                       210 numbers, 122.7 MB): the copy the array path reads,
//                       half the size of the odd-only table, which on a
//                       random lookup also leaves out the multiples of 3, 5
//                       and 7 (54% of the odd numbers).
//   sieve_kernel        one workgroup per 32 KiB segment (2^18 odd numbers).
//                       Multiples of 3..31 come from a periodic word mask
//                       (pre-sieve); each base prime p below 8192 is crossed
//                       off from max(p^2, segment start) by a whole
//                       wavefront, lane l taking the multiples l, l+64,
//                       l+128, ... of the stride p (in bit units), and each
//                       larger one (at most 32 multiples per segment) by one
//                       thread, with LDS atomic ANDs.  The first multiples
//                       come from 32-bit remainders, 64 primes at a time
//                       in a wavefront's lanes.
#include "internal.h"
#include "mont.h"

namespace isp {

namespace {

constexpr int SEG_WORDS = 8192;        // 32 KiB of LDS per workgroup
constexpr int SEG_BITS = SEG_WORDS * 32;
constexpr int SIEVE_THREADS = 1024;
constexpr int FIRST_CROSSED = 10;      // index of 37 in the odd-prime list

// Bits j < 32 with j = 0 (mod p).
__device__ __forceinline__ uint32_t period_mask(uint32_t p)
{
    uint32_t m = 0;
    for (uint32_t j = 0; j < 32; j += p)
        m |= 1u << j;
    return m;
}

// Inclusive scan of one value per lane across a 64-lane wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o)
            x += y;
    }
    return x;
}

__global__ void __launch_bounds__(1024) base_primes_kernel(uint32_t *primes, uint32_t *count)
{
    __shared__ uint32_t bits[1024];  // bit i <-> 2i+1 < 65536
    __shared__ uint32_t wave_sum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    bits[tid] = tid == 0 ? 0xfffffffeu : 0xffffffffu;  // 1 is not prime
    __syncthreads();
    // Crossing off the multiples of composite odd p as well is harmless.
    for (uint32_t p = 3; p * p < 65536; p += 2)
        for (uint32_t m = p * p + 2 * p * tid; m < 65536; m += 2 * p * blockDim.x)
            atomicAnd(&bits[m >> 6], ~(1u << ((m >> 1) & 31)));
    __syncthreads();
    const uint32_t w = bits[tid];
    const uint32_t c = __popc(w);
    const uint32_t incl = wave_inclusive_scan(c, lane);
    if (lane == 63)
        wave_sum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < wave; ++k)
        before += wave_sum[k];
    uint32_t pos = before + incl - c;
    for (uint32_t b = 0; b < 32; ++b)
        if ((w >> b) & 1)
            primes[pos++] = 2 * (32 * tid + b) + 1;
    if (tid == blockDim.x - 1)
        *count = pos;
}

__global__ void __launch_bounds__(SIEVE_THREADS) sieve_kernel(uint32_t *__restrict__ table,
                                                              const uint32_t *__restrict__ primes,
                                                              const uint32_t *__restrict__ pcount)
{
    __shared__ uint32_t seg[SEG_WORDS];
    const uint32_t w0 = blockIdx.x * SEG_WORDS;   // first table word of the segment
    const uint32_t lo = 2u * (w0 * 32u) + 1u;     // smallest odd number in it

    // Pre-sieve 3..31: in word w, bit j stands for 2(32w+j)+1, which p
    // divides iff j = (p-1)/2 - 32w (mod p).
    constexpr uint32_t SMALL[10] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
    for (int k = threadIdx.x; k < SEG_WORDS; k += blockDim.x) {
        const uint32_t w = w0 + k;
        uint32_t word = 0xffffffffu;
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const uint32_t p = SMALL[q];
            const uint32_t r = ((p - 1) / 2 + p - (32u * w) % p) % p;
            word &= ~(period_mask(p) << r);
        }
        seg[k] = word;
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        uint32_t keep = 0;  // the pre-sieved primes themselves stay prime
#pragma unroll
        for (int q = 0; q < 10; ++q)
            keep |= 1u << ((SMALL[q] - 1) / 2);
        seg[0] = (seg[0] | keep) & ~1u;  // and 1 is not prime
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    // the wavefront index as a scalar (the wavefront loop below is uniform)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const int np = (int)*pcount;
    const uint64_t hi = (uint64_t)lo + 2ull * SEG_BITS;  // exclusive
    // bit index of p's first odd multiple at or above max(p^2, lo), or
    // SEG_BITS when none falls in the segment (32-bit remainders: lo < 2^32)
    auto first_bit = [&](uint32_t p) -> uint32_t {
        const uint64_t pp = (uint64_t)p * p;
        if (pp >= hi)
            return (uint32_t)SEG_BITS;
        if (pp >= lo)
            return (uint32_t)((pp - lo) >> 1);  // p^2 is odd
        const uint32_t r = lo % p;
        uint32_t off = r ? p - r : 0u;  // lo + off: the first multiple at or above lo
        if (off & 1u)
            off += p;  // lo is odd: an odd offset gives an even multiple
        return off >> 1;
    };
    // primes 37 .. 8191 (the first 1027 odd primes): one wavefront per
    // prime.  The wavefront's primes are k = FIRST_CROSSED + wave + m nwaves;
    // their first bits are computed 64 at a time, one per lane, and each
    // crossing loop takes its prime and start from a lane (the remainders
    // run on the vector units, not on the compute unit's one scalar unit).
    constexpr int WAVE_PRIMES = 1027;
    const int k_split = np < WAVE_PRIMES ? np : WAVE_PRIMES;
    for (int kb = FIRST_CROSSED + wave; kb < k_split; kb += 64 * nwaves) {
        const int k = kb + lane * nwaves;
        uint32_t pl = 0, jl = (uint32_t)SEG_BITS;
        if (k < k_split) {
            pl = primes[k];
            jl = first_bit(pl);
        }
        const int cnt = min(64, (k_split - kb + nwaves - 1) / nwaves);
        for (int i = 0; i < cnt; ++i) {
            const uint32_t p = __builtin_amdgcn_readlane(pl, i);
            const uint32_t j0 = __builtin_amdgcn_readlane(jl, i);
            for (uint32_t j = j0 + (uint32_t)lane * p; j < (uint32_t)SEG_BITS; j += 64u * p)
                atomicAnd(&seg[j >> 5], ~(1u << (j & 31)));
        }
    }
    // larger primes: at most 32 multiples in the segment, one thread each
    for (int k = k_split + (int)threadIdx.x; k < np; k += blockDim.x) {
        const uint32_t p = primes[k];
        for (uint32_t j = first_bit(p); j < (uint32_t)SEG_BITS; j += p)
            atomicAnd(&seg[j >> 5], ~(1u << (j & 31)));
    }
    __syncthreads();
    for (int k = threadIdx.x; k < SEG_WORDS; k += blockDim.x)
        table[w0 + k] = seg[k];
}

// The wheel table, one thread per 32-bit word: bit b stands for the number
// 210 floor(b / 48) + res[b mod 48], whose bit is read from the odd-only
// table (0 for the numbers of the last block at or above 2^32).  A word's 32
// numbers increase and span at most 142 (the largest distance between a
// residue coprime to 210 and the 31st after it, around the cycle), so their
// table bits lie in four consecutive table words, read once.
__global__ void __launch_bounds__(256) wheel_table_kernel(uint32_t *__restrict__ wtable,
                                                          const uint32_t *__restrict__ table)
{
    __shared__ uint8_t res[WHEEL_RES];
    if (threadIdx.x < WHEEL_RES)
        res[threadIdx.x] = WHEEL.res[threadIdx.x];
    __syncthreads();
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= WHEEL_WORDS)
        return;
    const uint32_t b0 = (uint32_t)(w * 32);  // < 2^30
    uint32_t q = b0 / WHEEL_RES, r = b0 - q * WHEEL_RES;
    const uint64_t t0 = ((uint64_t)q * WHEEL_MOD + res[r]) >> 6;  // the first number's table word
    uint32_t tw[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        tw[i] = t0 + i < TABLE_WORDS ? table[t0 + i] : 0u;
    const uint64_t lo64 = tw[0] | (uint64_t)tw[1] << 32, hi64 = tw[2] | (uint64_t)tw[3] << 32;
    uint32_t word = 0;
    for (uint32_t j = 0; j < 32; ++j) {
        const uint64_t v = (uint64_t)q * WHEEL_MOD + res[r];
        const uint32_t idx = (uint32_t)((v >> 1) - (t0 << 5));  // below 103
        const uint64_t bits = idx < 64 ? lo64 >> idx : hi64 >> (idx - 64);
        if (v < TABLE_BOUND)
            word |= (uint32_t)(bits & 1u) << j;
        if (++r == WHEEL_RES) {
            r = 0;
            ++q;
        }
    }
    wtable[w] = word;
}

}  // namespace

hipError_t launch_wheel_table(DeviceState &ds, hipStream_t s)
{
    wheel_table_kernel<<<(unsigned)((WHEEL_WORDS + 255) / 256), 256, 0, s>>>(ds.wtable, ds.table);
    return hipGetLastError();
}

hipError_t launch_base_primes(DeviceState &ds, hipStream_t s)
{
    base_primes_kernel<<<1, 1024, 0, s>>>(ds.base_primes, ds.base_count);
    return hipGetLastError();
}

hipError_t launch_sieve(DeviceState &ds, hipStream_t s)
{
    static_assert(TABLE_WORDS % SEG_WORDS == 0, "segments tile the table");
    sieve_kernel<<<(unsigned)(TABLE_WORDS / SEG_WORDS), SIEVE_THREADS, 0, s>>>(
        ds.table, ds.base_primes, ds.base_count);
    return hipGetLastError();
}

}  // namespace isp
