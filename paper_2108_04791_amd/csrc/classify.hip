// classify.hip -- dispatch, table lookup, trial filter and survivor
// compaction in one streaming pass.
//
// Per element (paper: the input classes of section 1, the membership test of
// section 6.1.3, the array shrinking of section 6.1.2):
//   n < 2 -> 0, n == 2 -> 1, even -> 0
//   odd n < 2^32 -> its bit in the sieve table: for these arrays the copy
//                   on the 2*3*5*7 wheel (48 bits per 210 numbers), where a
//                   multiple of 3, 5 or 7 needs no read at all
//   odd n >= 2^32 -> 0 if a small odd prime divides it, else a survivor
// Every output byte is written here with coalesced stores (survivors get 0);
// the Miller-Rabin kernels later store a 1 for each prime survivor.
//
// Divisibility without division: a residue of n modulo a product of a few
// consecutive filter primes from two dot-product instructions, then per
// prime p: p | s iff s * p^-1 mod 2^32 <= floor((2^32 - 1) / p) (Granlund
// and Montgomery, PLDI 1994); see divisible_range.
//
// Work split without global atomics: the grid is a fixed number of
// workgroups; workgroup g owns the contiguous element range
// [g * chunk, (g + 1) * chunk) of the (for batched calls, virtual
// concatenated) input, writes its survivors to its own region
// surv[g * chunk ...] and stores its survivor count in counts[g]; the
// Miller-Rabin kernel scans those counts.  (A single hot device-scope
// atomic sustains only about 1e8 operations per second on this part, far
// too few to append survivors one workgroup at a time.)
//
// Also here: filter2_kernel, the second filter stage over each region's
// survivors (the rest of the first 64 odd primes), which also does the
// magnitude binning (survivors ordered by bit length in windows of 2048),
// and small_kernel, which decides a call of at most SMALL_MAX elements in
// one launch.
#include "compact.h"
#include "internal.h"
#include "mr_lane.h"

namespace isp {

namespace {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2), aligned(8)));

// Compile-time table of the first odd primes with their inverses modulo 2^32
// and the bound floor((2^32 - 1) / p), so the unrolled filter below uses
// immediate constants and issues no memory load.
constexpr int DENSE_TO = 64;  // the second stage ends at the 64th odd prime (313)
constexpr int FILTER2_BLOCK = 512;

constexpr bool ce_is_prime(uint64_t p)
{
    for (uint64_t d = 3; d * d <= p; d += 2)
        if (p % d == 0)
            return false;
    return true;
}

constexpr uint64_t ce_inv64(uint64_t p)
{
    uint64_t x = (3 * p) ^ 2;
    for (int k = 0; k < 4; ++k)
        x *= 2 - p * x;
    return x;
}

struct FilterTable {
    uint64_t prime[MAX_FILTER_PRIMES];
    uint32_t inv[MAX_FILTER_PRIMES];  // p^-1 mod 2^32
    uint32_t lim[MAX_FILTER_PRIMES];  // floor((2^32 - 1) / p)
    constexpr FilterTable() : prime(), inv(), lim()
    {
        int k = 0;
        for (uint64_t p = 3; k < MAX_FILTER_PRIMES; p += 2) {
            if (ce_is_prime(p)) {
                prime[k] = p;
                inv[k] = (uint32_t)ce_inv64(p);
                lim[k] = 0xffffffffu / (uint32_t)p;
                ++k;
            }
        }
    }
    // The residue groups: consecutive primes k .. end - 1 (end <= k1) whose
    // product M stays at most RES_M_MAX.
    constexpr int group_end(int k, int k1) const
    {
        uint64_t m = prime[k];
        int e = k + 1;
        while (e < k1 && m * prime[e] <= RES_M_MAX)
            m *= prime[e++];
        return e;
    }
    constexpr uint32_t product(int k, int e) const
    {
        uint64_t m = 1;
        for (int i = k; i < e; ++i)
            m *= prime[i];
        return (uint32_t)m;
    }
    static constexpr uint64_t RES_M_MAX = 16383;
};
constexpr FilterTable FILTER{};
static_assert(FILTER.inv[0] * 3u == 1u && FILTER.lim[0] == 1431655765u, "p = 3");
static_assert(FILTER.prime[MAX_FILTER_PRIMES - 1] == 727, "the 128th odd prime is 727");
static_assert(FILTER.group_end(0, 64) == 5 && FILTER.product(0, 5) == 15015, "3 5 7 11 13");

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Whether one of the odd primes K .. K1 - 1 divides n = h 2^32 + l, one
// residue group at a time.  With n's 16-bit chunks c_0 .. c_3 and a group's
// product M <= 16383, s = sum c_i (2^(16 i) mod M) is congruent to n modulo
// M, hence modulo each prime of the group, and s <= 4 (2^16 - 1) 16382 <
// 2^32: two v_dot2_u32_u16 form it.  Each prime p of the group then divides
// n iff it divides s, i.e. iff s p^-1 mod 2^32 <= floor((2^32 - 1) / p)
// (Granlund and Montgomery, PLDI 1994): one multiply and one compare.
template <int K, int K1>
__device__ __forceinline__ bool divisible_range(uint32_t l, uint32_t h)
{
    if constexpr (K >= K1) {
        return false;
    } else {
        constexpr int E = FILTER.group_end(K, K1);
        constexpr uint32_t M = FILTER.product(K, E);
        constexpr uint32_t W1 = (uint32_t)((1ull << 16) % M), W2 = (uint32_t)((1ull << 32) % M),
                           W3 = (uint32_t)((1ull << 48) % M);
        const uint32_t s0 = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, l),
                                                   u16x2{(unsigned short)1, (unsigned short)W1}, 0u,
                                                   false);
        const uint32_t s = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, h),
                                                  u16x2{(unsigned short)W2, (unsigned short)W3}, s0,
                                                  false);
        bool d = false;
#pragma unroll
        for (int k = K; k < E; ++k)
            d |= s * FILTER.inv[k] <= FILTER.lim[k];
        return d | divisible_range<E, K1>(l, h);
    }
}

__device__ __forceinline__ uint32_t lo_word(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi_word(uint64_t v) { return (uint32_t)(v >> 32); }

// 0 or 1: decided; 2: survivor of the filter (NF odd primes).
template <int NF>
__device__ __forceinline__ int classify_one(uint64_t v, const uint32_t *__restrict__ table)
{
    if (v < 3)
        return v == 2 ? 1 : 0;
    if ((v & 1) == 0)
        return 0;
    if (v < TABLE_BOUND)
        return (int)((table[v >> 6] >> ((v >> 1) & 31)) & 1u);
    return divisible_range<0, NF>(lo_word(v), hi_word(v)) ? 0 : 2;
}

// The same decision split in two, so that a thread issues the table reads
// of all its elements before it waits for any.  The read: for odd
// 3 <= v < 2^32 coprime to 210, the wheel-table word holding bit
// 48 floor(v / 210) + pos[v mod 210] (pos: the residue's index, in LDS);
// returns that bit's place in the word (widx: the word's index), or -1 when
// v needs no read.  An odd v < 2^32 sharing a factor with 210 is then prime
// only as 3, 5 or 7.  Branch-free, so that the caller can issue every
// element's LDS and table reads back to back: for a v that needs no read it
// computes a valid LDS index and returns widx = 0.
__device__ __forceinline__ int wheel_slot(uint64_t v, const uint8_t *wpos, uint32_t &widx)
{
    const bool in = (v & 1) != 0 && v >= 3 && v < TABLE_BOUND;
    const uint32_t n = (uint32_t)v | 1u;  // odd, so its residue indexes pos
    const uint32_t q = div210_odd(n);
    const uint32_t p = wpos[n - q * WHEEL_MOD];
    const bool read = in && p != 0xffu;
    const uint32_t b = q * WHEEL_RES + p;  // below 48 * 20452226 < 2^30 when read
    widx = read ? b >> 5 : 0u;
    return read ? (int)(b & 31u) : -1;
}

template <int NF>
__device__ __forceinline__ int classify_with(uint64_t v, uint32_t word, int bit)
{
    if (v < 3)
        return v == 2 ? 1 : 0;
    if ((v & 1) == 0)
        return 0;
    if (v < TABLE_BOUND)
        return bit >= 0 ? (int)((word >> bit) & 1u) : (v <= 7 ? 1 : 0);
    return divisible_range<0, NF>(lo_word(v), hi_word(v)) ? 0 : 2;
}

struct ClassifyShared {
    uint8_t wpos[WHEEL_MOD + 2];  // residue mod 210 -> its index among the 48 (0xff: none)
    uint32_t wave_cnt[16];
    uint32_t pass_total;
};

// One pass over the blockDim * EPT elements from p0 of one array, those
// below `end`.  Thread t takes the element pairs p0 + k * 2 * blockDim + 2t
// (k < EPT / 2; one element p0 + t when EPT is 1), so each load and store
// instruction of a wavefront covers one contiguous stretch.  Writes the
// output bytes and appends the pass's survivors at region[filled ...].
// Called by every thread of the block.
template <int EPT, int NF>
__device__ __forceinline__ void classify_pass(const uint64_t *__restrict__ n,
                                              uint8_t *__restrict__ out, uint64_t p0,
                                              uint64_t end, const uint32_t *__restrict__ wtable,
                                              Survivor *__restrict__ region, uint32_t &filled,
                                              ClassifyShared &sh)
{
    constexpr int PAIRS = EPT >= 2 ? EPT / 2 : 1;
    constexpr int PER = EPT >= 2 ? 2 : 1;  // consecutive elements per thread and step
    const uint64_t step = (uint64_t)blockDim.x * PER;
    const uint64_t mine = p0 + (uint64_t)threadIdx.x * PER;
    const bool full = p0 + step * PAIRS <= end;
    uint64_t v[EPT];
    if (full) {
#pragma unroll
        for (int k = 0; k < PAIRS; ++k) {
            if constexpr (PER == 2) {
                const u64x2 t = *reinterpret_cast<const u64x2 *>(n + mine + k * step);
                v[2 * k] = t.x;
                v[2 * k + 1] = t.y;
            } else {
                v[k] = n[mine + k * step];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint64_t i = mine + (j / PER) * step + (j % PER);
            v[j] = i < end ? n[i] : 0;
        }
    }
    // every table read first (a wavefront with no odd value below 2^32 in
    // the pass skips them), then the verdicts
    uint32_t word[EPT];
    int bit[EPT];
    bool any = false;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        word[j] = 0;
        bit[j] = -1;
        any |= (v[j] & 1) != 0 && v[j] < TABLE_BOUND;
    }
    if (__ballot(any) != 0) {
        uint32_t wi[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            bit[j] = wheel_slot(v[j], sh.wpos, wi[j]);
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            word[j] = wtable[wi[j]];
    }
    bool sv[EPT];
    uint8_t r[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint64_t i = mine + (j / PER) * step + (j % PER);
        const int c = classify_with<NF>(v[j], word[j], bit[j]);
        sv[j] = c == 2 && i < end;
        r[j] = (uint8_t)(c == 1);
    }
    if (full && PER == 2) {
        typedef uint16_t u16u __attribute__((aligned(1)));
#pragma unroll
        for (int k = 0; k < PAIRS; ++k)
            *reinterpret_cast<u16u *>(out + mine + k * step) =
                (uint16_t)(r[2 * k] | ((uint16_t)r[2 * k + 1] << 8));
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint64_t i = mine + (j / PER) * step + (j % PER);
            if (i < end)
                out[i] = r[j];
        }
    }

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    // compaction in the pass's element order (per slot): ballot per
    // slot, LDS scan over waves
    uint64_t masks[EPT];
    uint32_t wave_total = 0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        masks[j] = __ballot(sv[j]);
        wave_total += __popcll(masks[j]);
    }
    if (lane == 0)
        sh.wave_cnt[wave] = wave_total;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < nwaves; ++w) {
            const uint32_t t = sh.wave_cnt[w];
            sh.wave_cnt[w] = run;
            run += t;
        }
        sh.pass_total = run;
    }
    __syncthreads();
    uint32_t pos = filled + sh.wave_cnt[wave];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (sv[j]) {
            Survivor s;
            s.n = v[j];
            s.out = out + mine + (j / PER) * step + (j % PER);
            region[pos + __popcll(masks[j] & lt)] = s;
        }
        pos += __popcll(masks[j]);
    }
    filled += sh.pass_total;
    __syncthreads();  // sh is reused by the next pass
}

// Workgroup g classifies the element range [g * chunk, (g + 1) * chunk) of
// the input (plain) or of the virtual concatenation of the arrays (batched).
template <int EPT, bool BATCHED, int NF>
__global__ void __launch_bounds__(1024) classify_kernel(ClassifyArgs a)
{
    __shared__ ClassifyShared sh;
    for (uint32_t r = threadIdx.x; r < WHEEL_MOD; r += blockDim.x)
        sh.wpos[r] = WHEEL.pos[r];
    __syncthreads();
    const uint64_t g = blockIdx.x;
    const uint64_t total = BATCHED ? a.desc->total : a.total;
    const uint64_t chunk = classify_chunk(total, gridDim.x);
    const uint64_t r0 = g * chunk;
    const uint64_t r1 = r0 + chunk < total ? r0 + chunk : total;
    Survivor *region = a.surv + r0;
    uint32_t filled = 0;
    const uint64_t per_pass = (uint64_t)blockDim.x * EPT;
    if (r0 < r1) {
        if constexpr (!BATCHED) {
            for (uint64_t p0 = r0; p0 < r1; p0 += per_pass)
                classify_pass<EPT, NF>(a.n, a.out, p0, r1, a.wtable, region, filled, sh);
        } else {
            const BatchDesc *d = a.desc;
            // first array overlapping r0: prefix[lo] <= r0 < prefix[hi]
            uint32_t lo = 0, hi = d->num_arrays;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (d->elem_prefix[mid] <= r0)
                    lo = mid;
                else
                    hi = mid;
            }
            for (uint32_t k = lo; k < d->num_arrays && d->elem_prefix[k] < r1; ++k) {
                const uint64_t s0 = d->elem_prefix[k], s1 = d->elem_prefix[k + 1];
                if (s1 <= r0)
                    continue;  // an empty array at the start of the range
                const uint64_t b0 = (r0 > s0 ? r0 : s0) - s0;  // local range in array k
                const uint64_t b1 = (r1 < s1 ? r1 : s1) - s0;
                const uint64_t *nv = d->n_ptrs[k];
                uint8_t *ov = d->out_ptrs[k];
                for (uint64_t p0 = b0; p0 < b1; p0 += per_pass)
                    classify_pass<EPT, NF>(nv, ov, p0, b1, a.wtable, region, filled, sh);
            }
        }
    }
    if (threadIdx.x == 0)
        a.counts[g] = filled;
}

template <int EPT, bool BATCHED>
hipError_t launch_classify_nf(const ClassifyArgs &a, unsigned grid, int block, hipStream_t s)
{
    switch (a.nfilter) {
    case 0:
        classify_kernel<EPT, BATCHED, 0><<<grid, block, 0, s>>>(a);
        break;
    case 8:
        classify_kernel<EPT, BATCHED, 8><<<grid, block, 0, s>>>(a);
        break;
    case 16:
        classify_kernel<EPT, BATCHED, 16><<<grid, block, 0, s>>>(a);
        break;
    case 24:
        classify_kernel<EPT, BATCHED, 24><<<grid, block, 0, s>>>(a);
        break;
    case 32:
        classify_kernel<EPT, BATCHED, 32><<<grid, block, 0, s>>>(a);
        break;
    case 48:
        classify_kernel<EPT, BATCHED, 48><<<grid, block, 0, s>>>(a);
        break;
    case 64:
        classify_kernel<EPT, BATCHED, 64><<<grid, block, 0, s>>>(a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool BATCHED>
hipError_t launch_classify_t(const ClassifyArgs &a, unsigned grid, int block, int ept,
                             hipStream_t s)
{
    switch (ept) {
    case 1:
        return launch_classify_nf<1, BATCHED>(a, grid, block, s);
    case 2:
        return launch_classify_nf<2, BATCHED>(a, grid, block, s);
    case 4:
        return launch_classify_nf<4, BATCHED>(a, grid, block, s);
    case 8:
        return launch_classify_nf<8, BATCHED>(a, grid, block, s);
    default:
        return hipErrorInvalidValue;
    }
}

// A small array in one launch.  Each element gets a team of 8 consecutive
// lanes (8 teams per wavefront): every lane classifies it as classify_pass
// does (table lookup below 2^32, the trial filter above) and, for a survivor
// of the filter, runs the strong test to base 2; lanes 0..5 of the team then
// take one of the six other bases each.  The element is prime when all
// eight lanes pass (one wavefront ballot).  The call costs one launch and
// about two exponentiations of latency, where the three-kernel path costs
// three launches; throughput is not the concern at these sizes.
template <int NF>
__global__ void __launch_bounds__(SMALL_BLOCK) small_kernel(const uint64_t *__restrict__ n,
                                                         uint8_t *__restrict__ out, uint32_t len,
                                                         const uint32_t *__restrict__ table)
{
    constexpr uint32_t BASES6[6] = {325u, 9375u, 28178u, 450775u, 9780504u, 1795265022u};
    __shared__ uint64_t tbl[8 * SMALL_BLOCK];  // each lane's window table, by column
    const uint32_t gid = blockIdx.x * SMALL_BLOCK + threadIdx.x;
    const uint32_t i = gid / SMALL_TEAM, k = gid % SMALL_TEAM;
    const uint64_t v = i < len ? n[i] : 0;  // 0: decided (not prime) at once
    const int c = classify_one<NF>(v, table);
    bool ok = true;
    if (c == 2) {
        const LaneMr m = lane_mr(v);
        ok = sprp2_lane(m);
        if (ok && k < 6)
            ok = sprp_lane(m, r2_mod_n(m.c), BASES6[k], tbl, threadIdx.x, SMALL_BLOCK);
    }
    const uint64_t pass = __ballot(ok);
    const unsigned first = (threadIdx.x & 63u) & ~(SMALL_TEAM - 1u);
    if (k == 0 && i < len)
        out[i] = (uint8_t)(c == 1 || (c == 2 && ((pass >> first) & 0xffu) == 0xffu));
}

// Second trial-filter stage, between classify and the base-2 round: one
// workgroup per classify region compacts the region's survivors in place to
// those with no factor among the odd primes nf .. DENSE_TO - 1, and
// rewrites its count.  Only the survivors of the first stage (about a fifth
// of the elements) pay for these primes, one thread per survivor, and a
// prime p removes 1/p of them, each of which would otherwise cost a base-2
// exponentiation of ~1,700 instructions: worth it up to p ~ 300.
//
// With SORT (magnitude binning), the kept survivors of each window of
// F2_WINDOW entries are also ordered by decreasing bit length (a counting
// sort over the 32 lengths 64 .. 33, ranks from LDS atomics), so that a
// wavefront of the base-2 round gets values of (nearly) one bit length and
// its lanes run the same number of squarings.  A window is a few thousand
// survivors, i.e. tens of thousands of input elements.  Every entry of a
// window is read into registers before the first barrier, and it is written
// back at most at its own position, so the sort is in place.  Without SORT
// the survivors keep their order.
constexpr int F2_PER_THREAD = 4;
constexpr uint32_t F2_WINDOW = FILTER2_BLOCK * F2_PER_THREAD;

template <int NF>
__device__ __forceinline__ bool filter2_keep(uint64_t n)
{
    return !divisible_range<NF, DENSE_TO>(lo_word(n), hi_word(n));
}

template <int NF, bool SORT>
__global__ void __launch_bounds__(FILTER2_BLOCK) filter2_kernel(Survivor *__restrict__ surv,
                                                               uint32_t *__restrict__ counts,
                                                               uint64_t total,
                                                               const uint64_t *total_dev)
{
    __shared__ uint32_t wave_cnt[FILTER2_BLOCK / 64];
    __shared__ uint32_t hist[NUM_BINS], off[NUM_BINS + 1];
    const uint32_t g = blockIdx.x;
    // the regions of the classify grid (of the same size as this grid)
    const uint64_t chunk = classify_chunk(total_dev ? *total_dev : total, gridDim.x);
    Survivor *region = surv + (uint64_t)g * chunk;
    const uint32_t count = counts[g];
    uint32_t kept = 0;  // entries kept so far (block-uniform)
    if constexpr (!SORT) {
        for (uint32_t r0 = 0; r0 < count; r0 += FILTER2_BLOCK) {
            const uint32_t i = r0 + threadIdx.x;
            Survivor e;
            e.n = 0;
            e.out = nullptr;
            bool keep = false;
            if (i < count) {
                e = region[i];
                keep = filter2_keep<NF>(e.n);
            }
            compact_round<FILTER2_BLOCK>(region, e, keep, kept, wave_cnt);
        }
    } else {
        const int lane = threadIdx.x & 63;
        if (threadIdx.x < NUM_BINS)
            hist[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t w0 = 0; w0 < count; w0 += F2_WINDOW) {
            Survivor e[F2_PER_THREAD];
            uint32_t rank[F2_PER_THREAD];
            int key[F2_PER_THREAD];
            bool keep[F2_PER_THREAD];
#pragma unroll
            for (int k = 0; k < F2_PER_THREAD; ++k) {
                const uint32_t i = w0 + k * FILTER2_BLOCK + threadIdx.x;
                keep[k] = false;
                if (i < count) {
                    e[k] = region[i];
                    keep[k] = filter2_keep<NF>(e[k].n);
                }
            }
#pragma unroll
            for (int k = 0; k < F2_PER_THREAD; ++k) {
                key[k] = keep[k] ? __clzll(e[k].n) : 0;  // 0 (64 bits) .. 31 (33 bits)
                rank[k] = keep[k] ? atomicAdd(&hist[key[k]], 1u) : 0u;
            }
            __syncthreads();  // every entry of the window is read and counted
            if (threadIdx.x < 64) {
                const uint32_t h = lane < NUM_BINS ? hist[lane] : 0u;
                uint32_t incl = h;
#pragma unroll
                for (int o = 1; o < NUM_BINS; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o, 64);
                    if (lane >= o)
                        incl += y;
                }
                if (lane < NUM_BINS) {
                    off[lane] = incl - h;
                    hist[lane] = 0;  // ready for the next window
                }
                if (lane == NUM_BINS - 1)
                    off[NUM_BINS] = incl;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < F2_PER_THREAD; ++k)
                if (keep[k])
                    region[kept + off[key[k]] + rank[k]] = e[k];
            kept += off[NUM_BINS];
        }
    }
    if (threadIdx.x == 0)
        counts[g] = kept;
}

}  // namespace

hipError_t launch_filter2(Survivor *surv, uint32_t *counts, unsigned grid, uint64_t total,
                          const uint64_t *total_dev, int nf, int sorted, hipStream_t s)
{
#define F2(N, S) filter2_kernel<N, S><<<grid, FILTER2_BLOCK, 0, s>>>(surv, counts, total, total_dev)
    switch (nf) {
    case 8:
        sorted ? F2(8, true) : F2(8, false);
        break;
    case 16:
        sorted ? F2(16, true) : F2(16, false);
        break;
    case 24:
        sorted ? F2(24, true) : F2(24, false);
        break;
    case 32:
        sorted ? F2(32, true) : F2(32, false);
        break;
    case 48:
        sorted ? F2(48, true) : F2(48, false);
        break;
    default:
        // no first stage (0) or nothing left to test (64): only the sort
        if (!sorted)
            return hipSuccess;
        F2(DENSE_TO, true);
        break;
    }
#undef F2
    return hipGetLastError();
}

hipError_t launch_small(const uint64_t *n, uint8_t *out, size_t len, const uint32_t *table,
                        int nfilter, hipStream_t s)
{
    if (len == 0 || len > SMALL_MAX)
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)((len * SMALL_TEAM + SMALL_BLOCK - 1) / SMALL_BLOCK);
    const uint32_t m = (uint32_t)len;
    switch (nfilter) {
    case 0:
        small_kernel<0><<<grid, SMALL_BLOCK, 0, s>>>(n, out, m, table);
        break;
    case 8:
        small_kernel<8><<<grid, SMALL_BLOCK, 0, s>>>(n, out, m, table);
        break;
    case 16:
        small_kernel<16><<<grid, SMALL_BLOCK, 0, s>>>(n, out, m, table);
        break;
    case 24:
        small_kernel<24><<<grid, SMALL_BLOCK, 0, s>>>(n, out, m, table);
        break;
    case 32:
        small_kernel<32><<<grid, SMALL_BLOCK, 0, s>>>(n, out, m, table);
        break;
    case 48:
        small_kernel<48><<<grid, SMALL_BLOCK, 0, s>>>(n, out, m, table);
        break;
    case 64:
        small_kernel<64><<<grid, SMALL_BLOCK, 0, s>>>(n, out, m, table);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_classify(const ClassifyArgs &a, unsigned grid, int block, int ept, hipStream_t s)
{
    return a.desc ? launch_classify_t<true>(a, grid, block, ept, s)
                  : launch_classify_t<false>(a, grid, block, ept, s);
}

}  // namespace isp
