// classify.hip -- dispatch, table lookup, trial filter and survivor
// compaction in one streaming pass; then the magnitude-binning pass.
//
// Per element (paper: the input classes of section 1, the membership test of
// section 6.1.3, the array shrinking of section 6.1.2):
//   n < 2 -> 0, n == 2 -> 1, even -> 0
//   odd n < 2^32 -> bit (n >> 1) of the sieve table
//   odd n >= 2^32 -> 0 if a small odd prime divides it, else a survivor
// Every output byte is written here with coalesced stores (survivors get 0);
// the Miller-Rabin kernels later store a 1 for each prime survivor.
//
// Divisibility without division (Granlund and Montgomery, PLDI 1994):
// p | n iff n * p^-1 mod 2^64 <= floor((2^64 - 1) / p), for odd p.
//
// Survivors (value, output address) are appended to a device list: a
// wavefront ballot per element slot gives each lane its rank, the per-wave
// totals are scanned in LDS, and one atomic per workgroup reserves the
// block's range.  The order across workgroups is not deterministic; results
// do not depend on it.  A per-block LDS histogram of survivor bit lengths
// (33..64) feeds the binning pass.
//
// Binning (counting sort by bit length, longest first): each block counts
// its chunk per bin in LDS, reserves per-bin ranges with one atomic per bin,
// and scatters.  Wavefronts of the Miller-Rabin kernels then see values of
// one bit length, so every lane runs the same number of squarings.
#include "internal.h"

namespace isp {

namespace {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2), aligned(8)));

__device__ __forceinline__ uint64_t lanemask_lt(int lane)
{
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// 0 or 1: decided; 2: survivor of the filter.
__device__ __forceinline__ int classify_one(uint64_t v, const uint32_t *__restrict__ table,
                                            const FilterPrime *__restrict__ filt, int nfilt)
{
    if (v < 3)
        return v == 2 ? 1 : 0;
    if ((v & 1) == 0)
        return 0;
    if (v < TABLE_BOUND)
        return (int)((table[v >> 6] >> ((v >> 1) & 31)) & 1u);
    for (int k = 0; k < nfilt; ++k)
        if (v * filt[k].inv <= filt[k].lim)
            return 0;
    return 2;
}

__device__ __forceinline__ int bin_of(uint64_t v)
{
    return (64 - __clzll(v)) - 33;  // v >= 2^32: 0..31
}

// Appends the survivors of a block to ws.surv: slot-major within a wave.
template <int EPT>
__device__ __forceinline__ void append_survivors(const uint64_t (&v)[EPT], const bool (&sv)[EPT],
                                                 uint8_t *out_base, Survivor *__restrict__ surv,
                                                 Counters *__restrict__ ctr, int binning,
                                                 uint32_t *wave_off, uint32_t *hist,
                                                 uint32_t *block_base)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    uint64_t masks[EPT];
    uint32_t wave_total = 0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        masks[j] = __ballot(sv[j]);
        wave_total += __popcll(masks[j]);
    }
    if (lane == 0)
        wave_off[wave] = wave_total;
    if (binning) {
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (sv[j])
                atomicAdd(&hist[bin_of(v[j])], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < nwaves; ++w) {
            uint32_t t = wave_off[w];
            wave_off[w] = run;
            run += t;
        }
        *block_base = run ? atomicAdd(&ctr->survivors, run) : 0u;
    }
    if (binning && threadIdx.x < NUM_BINS) {
        // hist is complete after the barrier above
        uint32_t h = hist[threadIdx.x];
        if (h)
            atomicAdd(&ctr->bin_count[threadIdx.x], h);
    }
    __syncthreads();
    uint32_t pos = *block_base + wave_off[wave];
    const uint64_t lt = lanemask_lt(lane);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (sv[j]) {
            Survivor s;
            s.n = v[j];
            s.out = out_base + j;
            surv[pos + __popcll(masks[j] & lt)] = s;
        }
        pos += __popcll(masks[j]);
    }
}

// Classifies elements [base, base + EPT) of one array (those below `end`),
// writes their output bytes and appends the survivors.  Called by every
// thread of the block (it contains barriers).
template <int EPT>
__device__ __forceinline__ void classify_span(const uint64_t *__restrict__ n,
                                              uint8_t *__restrict__ out, uint64_t base,
                                              uint64_t end, const uint32_t *__restrict__ table,
                                              const FilterPrime *__restrict__ filt, int nfilt,
                                              Survivor *__restrict__ surv,
                                              Counters *__restrict__ ctr, int binning,
                                              uint32_t *wave_off, uint32_t *hist,
                                              uint32_t *block_base)
{
    uint64_t v[EPT];
    const bool full = base + EPT <= end;
    if (full) {
        if constexpr (EPT >= 2) {
#pragma unroll
            for (int j = 0; j < EPT; j += 2) {
                u64x2 t = *reinterpret_cast<const u64x2 *>(n + base + j);
                v[j] = t.x;
                v[j + 1] = t.y;
            }
        } else {
            v[0] = n[base];
        }
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            v[j] = base + j < end ? n[base + j] : 0;
    }
    bool sv[EPT];
    uint8_t r[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        int c = classify_one(v[j], table, filt, nfilt);
        sv[j] = c == 2 && base + j < end;
        r[j] = (uint8_t)(c == 1);
    }
    if (full) {
        if constexpr (EPT == 4) {
            typedef uint32_t u32u __attribute__((aligned(1)));
            *reinterpret_cast<u32u *>(out + base) = (uint32_t)r[0] | ((uint32_t)r[1] << 8) |
                                                    ((uint32_t)r[2] << 16) | ((uint32_t)r[3] << 24);
        } else if constexpr (EPT == 8) {
            typedef uint64_t u64u __attribute__((aligned(1)));
            uint64_t p = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                p |= (uint64_t)r[j] << (8 * j);
            *reinterpret_cast<u64u *>(out + base) = p;
        } else {
#pragma unroll
            for (int j = 0; j < EPT; ++j)
                out[base + j] = r[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (base + j < end)
                out[base + j] = r[j];
    }
    append_survivors<EPT>(v, sv, out + base, surv, ctr, binning, wave_off, hist, block_base);
}

template <int EPT>
__global__ void __launch_bounds__(1024) classify_kernel(const uint64_t *__restrict__ n,
                                                        uint8_t *__restrict__ out, uint64_t len,
                                                        const uint32_t *__restrict__ table,
                                                        const FilterPrime *__restrict__ filt,
                                                        int nfilt, Survivor *__restrict__ surv,
                                                        Counters *__restrict__ ctr, int binning)
{
    __shared__ uint32_t wave_off[16];
    __shared__ uint32_t hist[NUM_BINS];
    __shared__ uint32_t block_base;
    if (binning && threadIdx.x < NUM_BINS)
        hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * EPT;
    classify_span<EPT>(n, out, base, len, table, filt, nfilt, surv, ctr, binning, wave_off, hist,
                       &block_base);
}

// Batched form: a persistent grid walks tiles of many arrays.  Tile t of the
// whole batch belongs to the array a with tile_prefix[a] <= t <
// tile_prefix[a+1] (binary search) and covers elements
// [(t - tile_prefix[a]) * tile, +tile) of it.
template <int EPT>
__global__ void __launch_bounds__(1024) classify_batched_kernel(
    const BatchDesc *__restrict__ desc, const uint32_t *__restrict__ table,
    const FilterPrime *__restrict__ filt, int nfilt, Survivor *__restrict__ surv,
    Counters *__restrict__ ctr, int binning, uint32_t tile)
{
    __shared__ uint32_t wave_off[16];
    __shared__ uint32_t hist[NUM_BINS];
    __shared__ uint32_t block_base;
    __shared__ uint32_t cur_tile;
    const uint32_t num_arrays = desc->num_arrays;
    const uint32_t num_tiles = desc->num_tiles;
    const uint64_t *const *n_ptrs = desc->n_ptrs;
    uint8_t *const *out_ptrs = desc->out_ptrs;
    const uint64_t *lens = desc->lens;
    const uint32_t *tile_prefix = desc->tile_prefix;
    const uint32_t per_pass = blockDim.x * EPT;

    for (;;) {
        if (threadIdx.x == 0)
            cur_tile = atomicAdd(&ctr->tile_cursor, 1u);
        __syncthreads();
        const uint32_t t = cur_tile;
        __syncthreads();
        if (t >= num_tiles)
            break;
        uint32_t lo = 0, hi = num_arrays;  // prefix[lo] <= t < prefix[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tile_prefix[mid] <= t)
                lo = mid;
            else
                hi = mid;
        }
        const uint64_t len = lens[lo];
        const uint64_t t0 = (uint64_t)(t - tile_prefix[lo]) * tile;
        const uint64_t t1 = t0 + tile < len ? t0 + tile : len;
        const uint64_t *nv = n_ptrs[lo];
        uint8_t *ov = out_ptrs[lo];
        for (uint64_t pass0 = t0; pass0 < t1; pass0 += per_pass) {
            if (binning && threadIdx.x < NUM_BINS)
                hist[threadIdx.x] = 0;
            __syncthreads();
            classify_span<EPT>(nv, ov, pass0 + (uint64_t)threadIdx.x * EPT, t1, table, filt, nfilt,
                               surv, ctr, binning, wave_off, hist, &block_base);
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(256) bin_kernel(const Survivor *__restrict__ in,
                                                  Survivor *__restrict__ outl,
                                                  Counters *__restrict__ ctr)
{
    __shared__ uint32_t start[NUM_BINS];
    __shared__ uint32_t lcount[NUM_BINS];
    __shared__ uint32_t lbase[NUM_BINS];
    const uint32_t total = ctr->survivors;
    const int tid = threadIdx.x;
    if (tid < NUM_BINS) {
        // longest values first: bin 31 (64-bit) starts at 0
        uint32_t s = 0;
        for (int b = NUM_BINS - 1; b > tid; --b)
            s += ctr->bin_count[b];
        start[tid] = s;
    }
    for (uint64_t chunk = (uint64_t)blockIdx.x * blockDim.x; chunk < total;
         chunk += (uint64_t)gridDim.x * blockDim.x) {
        if (tid < NUM_BINS)
            lcount[tid] = 0;
        __syncthreads();
        const uint64_t i = chunk + tid;
        const bool active = i < total;
        Survivor s;
        int b = 0;
        uint32_t lpos = 0;
        if (active) {
            s = in[i];
            b = bin_of(s.n);
            lpos = atomicAdd(&lcount[b], 1u);
        }
        __syncthreads();
        if (tid < NUM_BINS && lcount[tid])
            lbase[tid] = start[tid] + atomicAdd(&ctr->bin_cursor[tid], lcount[tid]);
        __syncthreads();
        if (active)
            outl[lbase[b] + lpos] = s;
        __syncthreads();
    }
}

__global__ void reset_kernel(Counters *ctr)
{
    uint32_t *w = reinterpret_cast<uint32_t *>(ctr);
    for (unsigned k = threadIdx.x; k < sizeof(Counters) / 4; k += blockDim.x)
        w[k] = 0;
}

}  // namespace

hipError_t launch_reset(Counters *ctr, hipStream_t s)
{
    reset_kernel<<<1, 128, 0, s>>>(ctr);
    return hipGetLastError();
}

hipError_t launch_classify(const uint64_t *n, uint8_t *out, uint64_t len, const DeviceState &ds,
                           const Workspace &ws, const Tuning &t, hipStream_t s)
{
    const uint64_t per_block = (uint64_t)t.classify_block * t.classify_ept;
    const uint64_t blocks = (len + per_block - 1) / per_block;
    if (blocks > 0x7fffffffull)
        return hipErrorInvalidValue;
    const int bin = t.mr_bins > 0;
    switch (t.classify_ept) {
    case 1:
        classify_kernel<1><<<(unsigned)blocks, t.classify_block, 0, s>>>(
            n, out, len, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin);
        break;
    case 2:
        classify_kernel<2><<<(unsigned)blocks, t.classify_block, 0, s>>>(
            n, out, len, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin);
        break;
    case 4:
        classify_kernel<4><<<(unsigned)blocks, t.classify_block, 0, s>>>(
            n, out, len, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin);
        break;
    case 8:
        classify_kernel<8><<<(unsigned)blocks, t.classify_block, 0, s>>>(
            n, out, len, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_classify_batched(const BatchDesc *desc, uint32_t grid, const DeviceState &ds,
                                   const Workspace &ws, const Tuning &t, hipStream_t s)
{
    const int bin = t.mr_bins > 0;
    const uint32_t tile = (uint32_t)t.batch_tile;
    switch (t.classify_ept) {
    case 1:
        classify_batched_kernel<1><<<grid, t.classify_block, 0, s>>>(
            desc, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin, tile);
        break;
    case 2:
        classify_batched_kernel<2><<<grid, t.classify_block, 0, s>>>(
            desc, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin, tile);
        break;
    case 4:
        classify_batched_kernel<4><<<grid, t.classify_block, 0, s>>>(
            desc, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin, tile);
        break;
    case 8:
        classify_batched_kernel<8><<<grid, t.classify_block, 0, s>>>(
            desc, ds.table, ds.filter, t.filter_primes, ws.surv, ws.ctr, bin, tile);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bin(const Workspace &ws, const Tuning &t, int cus, hipStream_t s)
{
    (void)t;
    bin_kernel<<<(unsigned)(cus * 4), 256, 0, s>>>(ws.surv, ws.sorted, ws.ctr);
    return hipGetLastError();
}

}  // namespace isp
