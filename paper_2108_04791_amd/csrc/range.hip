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
// bucket mode (below): the primes above 2^20 up to the square root are
// sorted into per-segment buckets first, and the segments are complete
// again.  A short piece is sieved by the odd primes below 2^22 (below 2^18
// when it has fewer than 256 full segments; it is then cut into up to 256
// shorter ones, since so few workgroups would wait on the sieve's latency)
// and the survivors (about 3.4% of the numbers with no factor below 2^22,
// 4.5% below 2^18) go to the same two Miller-Rabin kernels as array inputs,
// through the same per-workgroup regions and counts.
//
// Segment layout: workgroup g covers numbers [lo + g*chunk, lo + (g+1)*chunk)
// with chunk = classify_chunk(len, grid) (a multiple of 64, at most
// RANGE_SEG); bit j of its LDS bitset stands for the odd number o0 + 2j.
// The multiples of 3 .. 31 come from periodic word masks (pre-sieve);
// primes 37 .. 8191 are crossed off by whole wavefronts (lane l takes the
// multiples l, l+64, ... of the stride), larger primes one per thread.  The
// first odd multiple of p at or above max(o0, p^2) needs o0 mod p, taken
// with a precomputed floor((2^64 - 1) / p) (one 64-bit multiply-high, no
// division).
//
// Output: 16 consecutive numbers per thread per pass, consecutive threads on
// consecutive 16-byte pieces.  Their 8 odd members are 8 consecutive bits;
// each group of 4 bits becomes 8 output bytes by one multiply that spreads
// bit i to byte 2i (or 2i + 1), and the piece goes out as one 16-byte store.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace isp {

namespace {

constexpr int RANGE_THREADS = 1024;
constexpr uint32_t WAVE_PRIME_LIMIT = 8192;  // primes below this: wavefront per prime
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
    const uint64_t *inv;
    uint32_t nprimes;
    Survivor *surv;      // grid regions of `chunk` entries
    uint32_t *counts;    // [grid]
    // bucket mode: the primes above BUCKET_SMALL come as precomputed hits
    const uint32_t *hit_start;  // [groups * grid + 1]: the hits of segment g found
                                // by group q are hits[hit_start[q * grid + g] ..
                                // hit_start[q * grid + g + 1])
    const uint32_t *hits;       // bit indices within their segment
    uint64_t hit_cap;           // entries allocated in hits
    uint32_t groups;            // 0: no buckets
    uint32_t partial_log2;      // where the sieve cannot be complete: primes below 2^this
    uint32_t complete_log2;     // segments whose root is below 2^this are complete
};


__global__ void __launch_bounds__(RANGE_THREADS) range_sieve_kernel(RangeArgs a)
{
    constexpr int MAX_WORDS = (int)(RANGE_SEG / 64);  // 2^13 words of odd-number bits
    __shared__ uint32_t bits[MAX_WORDS + 1];          // + one zero word past the end
    __shared__ uint32_t wsum[RANGE_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63;
    // the wavefront index as a scalar, so per-prime work of the wavefront
    // loop below (the prime, its first multiple) runs on the scalar unit
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
    // first bit index of the odd multiples of p at or above max(o0, p^2), or
    // "none" (all offsets are taken from o0, so nothing wraps near 2^64)
    const uint64_t span = s_last - o0;  // valid only when nbits > 0
    auto first_bit = [&](uint32_t p, uint64_t inv) -> uint64_t {
        const uint64_t pp = (uint64_t)p * p;  // < 2^50, odd
        uint64_t off;
        if (pp >= o0) {
            off = pp - o0;
        } else {
            const uint64_t r = mod_small(o0, p, inv);
            off = r ? p - r : 0;  // o0 + off: first multiple of p at or above o0
            if (off & 1)
                off += p;         // o0 is odd: an odd offset gives an even multiple
        }
        return off > span ? ~(uint64_t)0 : off >> 1;
    };
    // primes 37 .. 8191: one wavefront per prime
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
    for (uint32_t k = PRESIEVED + wave; k < k_split; k += nwaves) {
        const uint32_t p = a.primes[k];
        const uint64_t j0 = first_bit(p, a.inv[k]);
        if (j0 >= nbits)
            continue;
        // bit indices below 2^18: 32-bit arithmetic
        const uint32_t stride = 64u * p;
        for (uint32_t j = (uint32_t)j0 + (uint32_t)lane * p; j < nbits; j += stride)
            atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
    }
    // larger primes: one thread per prime; the thread's next prime and its
    // constant are loaded while the current one is crossed off (the loads'
    // latency, not the arithmetic, bounds this loop)
    {
        uint32_t k = k_split + tid;
        uint32_t p = 0;
        uint64_t inv = 0;
        if (k < np) {
            p = a.primes[k];
            inv = a.inv[k];
        }
        while (k < np) {
            const uint32_t kn = k + blockDim.x;
            uint32_t pn = 0;
            uint64_t invn = 0;
            if (kn < np) {
                pn = a.primes[kn];
                invn = a.inv[kn];
            }
            const uint64_t j0 = first_bit(p, inv);
            if (j0 < nbits)
                for (uint32_t j = (uint32_t)j0; j < nbits; j += p)
                    atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
            k = kn;
            p = pn;
            inv = invn;
        }
    }
    // bucket mode: the hits of the primes above BUCKET_SMALL in this segment
    if (buckets) {
        // one run per group, read by one wavefront (the hits fit by
        // construction; the clamp only keeps reads inside the allocation)
        for (uint32_t q = wave; q < a.groups; q += nwaves) {
            const uint64_t at = (uint64_t)q * gridDim.x + blockIdx.x;
            const uint32_t h0 = a.hit_start[at];
            const uint32_t h1 = (uint32_t)min((uint64_t)a.hit_start[at + 1], a.hit_cap);
            for (uint32_t h = h0 + lane; h < h1; h += 64) {
                const uint32_t j = a.hits[h];
                atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
            }
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
// A prime p > 2^19 has at most one odd multiple in a segment of 2^19
// numbers (BUCKET_SMALL is at least that), so visiting every such prime in every segment costs one
// reduction per prime and segment.  Bucket mode inverts the loop (the
// bucket sieve of segmented sieving): the odd primes in (BUCKET_SMALL,
// sqrt(end)] are read from the device table, each prime's odd multiples at
// or above max(lo, p^2) are enumerated once over the whole piece, and each
// becomes a hit (its bit index) in the bucket of its segment.  Two passes
// over the same primes by `groups` workgroups: count the hits per (segment,
// group) in LDS, then after an exclusive scan write them at their places,
// so no global atomic is needed.  The segment kernel then applies its
// bucket.  With every prime up to the square root crossed off, the
// segments are complete at any magnitude below 2^64.

struct BucketArgs {
    uint64_t lo, len;        // the piece
    uint64_t w_begin, w_end; // table words holding the odd primes in (BUCKET_SMALL, root]
    uint64_t root;
    const uint32_t *table;
    uint32_t nseg;           // segments of RANGE_SEG numbers
    uint32_t *counts;        // [groups * nseg + 1], group-major: (group, g)
    uint32_t *hits;
    uint64_t hit_cap;
};

// lo mod p for p < 2^32 from a double-precision quotient estimate (error
// below one unit: lo < 2^64 is rounded to 53 bits and the quotient is below
// 2^45, so the estimate is within 2^-7 of lo / p) and one correction each way.
__device__ __forceinline__ uint64_t mod_u32(uint64_t x, uint32_t p)
{
    const double q = (double)x * (1.0 / (double)p);
    uint64_t qi = q < 1.0 ? 0 : (uint64_t)q;
    int64_t r = (int64_t)(x - qi * (uint64_t)p);
    if (r < 0)
        r += p;
    if (r >= (int64_t)p)
        r -= p;
    return (uint64_t)r;
}

// Offset from lo of p's first odd multiple at or above max(lo, p^2), or an
// offset >= len when there is none.
__device__ __forceinline__ uint64_t bucket_first(const BucketArgs &a, uint32_t p)
{
    const uint64_t pp = (uint64_t)p * p;
    uint64_t off;
    if (pp >= a.lo) {
        off = pp - a.lo;  // odd square: odd when lo is even, and lo + off is odd
    } else {
        const uint64_t r = mod_u32(a.lo, p);
        off = r ? p - r : 0;
        if (((a.lo + off) & 1) == 0)
            off += p;  // the next multiple is odd
    }
    return off;
}

// Cost of the primes below x, up to constants: one first-hit computation per
// prime (x / ln x primes) and one bucket entry per hit (len/2 * sum 1/p, which
// grows like ln ln x).  Group g takes the primes whose cumulative cost falls
// in its equal share, so the low primes with hundreds of hits each and the
// high primes with at most one are spread evenly.
__device__ __forceinline__ double bucket_cost(double x, double len)
{
    const double lx = log(x);
    return 24.0 * x / lx + 4.0 * 0.5 * len * log(lx);
}

// The prime bound where the cumulative cost reaches `target` (bisection).
__device__ double bucket_split(double target, double lo, double hi, double len)
{
    for (int it = 0; it < 80; ++it) {
        const double mid = 0.5 * (lo + hi);
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

// Every odd multiple of p in the piece, each counted in (FILL: written to)
// the bucket of its segment.  The lanes of a wavefront hold consecutive
// primes, whose multiples march through the segments together; each lane
// starts at its own share (lane / 64) of its K multiples and wraps around,
// so at each step the lanes touch different segments instead of queueing on
// the same LDS counter.
template <bool FILL>
__device__ __forceinline__ void bucket_hits(const BucketArgs &a, uint32_t p, uint32_t lane,
                                            uint32_t *cnt)
{
    const uint64_t first = bucket_first(a, p);
    if (first >= a.len)
        return;
    const uint64_t step = 2ull * p;
    const uint64_t span = a.len - 1 - first;  // < 2^30
    // K = floor(span / step) + 1; step > span means a single multiple, and
    // otherwise step < 2^30 fits 32 bits
    uint32_t K = 1;
    if (step <= span)
        K = (uint32_t)span / (uint32_t)step + 1u;
    uint64_t off = first + (uint64_t)((lane * K) >> 6) * step;
    for (uint32_t j = 0; j < K; ++j) {
        const uint32_t g = (uint32_t)(off >> RANGE_SEG_LOG2);
        if (FILL) {
            const uint32_t at = atomicAdd(&cnt[g], 1u);
            if (at < a.hit_cap)
                a.hits[at] = (uint32_t)((off & (RANGE_SEG - 1)) >> 1);
        } else {
            atomicAdd(&cnt[g], 1u);
        }
        off += step;
        if (off >= a.len)
            off = first;
    }
}

// Count pass (FILL false): cnt[g] counts this group's hits in segment g and
// goes to counts[group * nseg + g] (group-major, so that each group's hits
// land in one contiguous stretch of `hits`).  Fill pass: cnt[g] starts at the
// scanned offset of (group, g), so each atomic increment yields the hit's
// place in `hits` directly.  The wavefront-scope fences below order LDS
// accesses between the lanes of one wavefront (whose LDS operations complete
// in order) without waiting for its global stores.
template <bool FILL>
__global__ void __launch_bounds__(BUCKET_THREADS) range_bucket_kernel(BucketArgs a)
{
    __shared__ uint32_t cnt[MAX_BUCKET_SEGS];
    __shared__ uint32_t pbuf[BUCKET_THREADS / 64][BUCKET_PBUF];
    __shared__ uint64_t wrange[2];
    const uint32_t groups = gridDim.x;
    for (uint32_t g = threadIdx.x; g < a.nseg; g += blockDim.x)
        cnt[g] = FILL ? a.counts[(uint64_t)blockIdx.x * a.nseg + g] : 0u;
    if (threadIdx.x == 0) {
        // this group's words: equal shares of the cost between BUCKET_SMALL and root
        const double len = (double)a.len, x0 = (double)BUCKET_SMALL, x1 = (double)a.root + 1.0;
        const double c0 = bucket_cost(x0, len), c1 = bucket_cost(x1, len);
        uint64_t wb = a.w_begin, we = a.w_end;
        if (blockIdx.x > 0)
            wb = (uint64_t)bucket_split(c0 + (c1 - c0) * blockIdx.x / groups, x0, x1, len) >> 6;
        if (blockIdx.x + 1 < groups)
            we = (uint64_t)bucket_split(c0 + (c1 - c0) * (blockIdx.x + 1) / groups, x0, x1, len) >> 6;
        wrange[0] = wb < a.w_begin ? a.w_begin : (wb > a.w_end ? a.w_end : wb);
        wrange[1] = we < a.w_begin ? a.w_begin : (we > a.w_end ? a.w_end : we);
    }
    __syncthreads();
    const uint64_t wb = wrange[0], we = wrange[1];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nwaves = blockDim.x >> 6;
    uint32_t *buf = pbuf[wave];
    auto take = [&](uint32_t p) {
        if (p > BUCKET_SMALL && p <= a.root)
            bucket_hits<FILL>(a, p, lane, cnt);
    };
    // the primes of a chunk of 64 words (w0 .. w0 + 63; lane l holds word
    // w0 + l) are listed densely in LDS (a wavefront prefix sum of the
    // words' popcounts) and then taken one per lane
    auto chunk = [&](uint64_t w0, uint32_t word) {
        const uint64_t w = w0 + lane;
        const uint32_t c = (uint32_t)__popc(word);
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= (uint32_t)o)
                inc += t;
        }
        const uint32_t total = __shfl(inc, 63, 64);
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
    const uint64_t nch = we > wb ? (we - wb + 63) / 64 : 0;
    for (uint64_t ch = wave; ch < nch; ch += nwaves) {
        const uint64_t w = wb + 64 * ch + lane;
        chunk(wb + 64 * ch, w < we ? a.table[w] : 0u);
    }
    if (!FILL) {
        __syncthreads();
        for (uint32_t g = threadIdx.x; g < a.nseg; g += blockDim.x)
            a.counts[(uint64_t)blockIdx.x * a.nseg + g] = cnt[g];
    }
}

// Exclusive scan of counts[0 .. n) in place, total at counts[n], in three
// passes over tiles of SCAN_TILE words: tile sums, a scan of the sums (one
// workgroup), then each tile scanned and offset.
constexpr int SCAN_TILE = 8192;  // 1024 threads x 8

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

hipError_t launch_range_buckets(uint64_t lo, uint64_t len, uint64_t root, unsigned groups,
                                const DeviceState &ds, const RangeWs &rw, hipStream_t s)
{
    BucketArgs a;
    a.lo = lo;
    a.len = len;
    a.root = root;
    a.table = ds.table;
    a.w_begin = (BUCKET_SMALL + 1) >> 6;
    a.w_end = (root >> 6) + 1;
    a.nseg = (uint32_t)((len + RANGE_SEG - 1) / RANGE_SEG);
    a.counts = rw.counts;
    a.hits = rw.hits;
    a.hit_cap = rw.hit_cap;
    if (a.nseg > (uint32_t)MAX_BUCKET_SEGS || a.w_end > (uint64_t)TABLE_WORDS ||
        a.w_end <= a.w_begin)
        return hipErrorInvalidValue;
    const uint32_t n = a.nseg * groups;
    const uint32_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles > 1024 || rw.count_cap < (uint64_t)n + 1 + ntiles + 1)
        return hipErrorInvalidValue;
    uint32_t *sums = rw.counts + n + 1;  // ntiles + 1 words after the counts
    range_bucket_kernel<false><<<groups, BUCKET_THREADS, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        scan_tile_sums<<<ntiles, 1024, 0, s>>>(rw.counts, n, sums);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        scan_small<<<1, 1024, 0, s>>>(sums, ntiles);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        scan_tiles<<<ntiles, 1024, 0, s>>>(rw.counts, n, sums);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        range_bucket_kernel<true><<<groups, BUCKET_THREADS, 0, s>>>(a);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_range_sieve(uint64_t lo, uint8_t *out, uint64_t len, unsigned grid,
                              uint64_t chunk, unsigned groups, const DeviceState &ds,
                              const Workspace &ws, const RangeWs &rw, hipStream_t s,
                              int partial_log2, int complete_log2)
{
    if (partial_log2 < 17 || partial_log2 > RANGE_PARTIAL_LOG2 || complete_log2 < partial_log2 ||
        complete_log2 > RANGE_PRIME_LOG2)
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
    a.inv = ds.range_inv;
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
