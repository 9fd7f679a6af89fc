// mr.hip -- deterministic Miller-Rabin over the seven bases, one survivor per
// lane, in two persistent phases.
//
// Paper, section 2.1: write n - 1 = 2^s d with d odd; a prime n satisfies,
// for every base a, a^d = 1 or a^(2^r d) = -1 (mod n) for some 0 <= r < s
// (Eq. 1-3, read as the standard strong test).  Eq. 4 lists the seven bases
// 2, 325, 9375, 28178, 450775, 9780504, 1795265022 that make the test exact
// for every 64-bit n; n is prime iff it passes all seven.  Section 2.4
// computes a^d by square-and-multiply.  Every n reaching this file is odd
// and >= 2^32, so every base is already reduced (all are below 2^31).
//
// Phase 1 (all survivors): base 2 only.  The exponent is processed over the
// bits of n - 1 from the top, so every lane with the same bit length L runs
// exactly L - 2 squarings; the multiply by 2 is a modular doubling (the
// ModAdd of section 2.2) selected without a branch.  About 4 in 5 survivors
// of random inputs fail here.  Passers go to the workgroup's own region.
//
// Phase 2 (base-2 passers, almost all prime): the six remaining bases, one
// base per lane: a wavefront takes 10 candidates on 60 lanes (lanes 6c ..
// 6c+5 hold the six bases of candidate c) and a ballot ANDs the six
// verdicts.  a^d uses a fixed window of W bits with a per-lane table of
// a^0..a^(2^W - 1) selected by a tree of selects (no dynamic register
// indexing), so all lanes multiply at the same steps; then up to s - 1
// squarings look for -1.  A prime stores out = 1 (classify wrote 0).
//
// Work split without global atomics (a single hot device-scope atomic
// sustains only about 1e8 operations per second on this part): each
// workgroup scans the producer's per-workgroup counts in LDS, takes an
// equal slice of the resulting dense index space, and finds each element's
// producer region by binary search in LDS.
#include "internal.h"
#include "mont.h"

namespace isp {

namespace {

// Strong probable-prime test to base 2 for odd n >= 2^32.
__device__ __forceinline__ bool sprp_base2(uint64_t n)
{
    const int L = 64 - __clzll(n);
    const MontCtx c = make_ctx(n, L);
    const uint64_t e = n - 1;
    const int s = __ffsll((long long)e) - 1;
    uint64_t x = dbl_mod(c.one, n);  // top bit of e (bit L-1): x = 2
    bool pass = (s == L - 1) && (x == c.one || x == c.mone);
    for (int t = L - 2; t >= 1; --t) {
        x = montsqr(x, n, c.ninv);
        const uint64_t x2 = dbl_mod(x, n);
        x = ((e >> t) & 1) ? x2 : x;
        pass |= (t == s) & ((x == c.one) | (x == c.mone));
        pass |= (t < s) & (x == c.mone);
    }
    return pass;
}

// T[w] for a per-lane w < 2^W, as a tree of selects on the bits of w with
// constant register indices (dynamic indexing would go through scratch).
template <int W>
__device__ __forceinline__ uint64_t select_pow(const uint64_t (&T)[1 << W], unsigned w)
{
    uint64_t v[1 << W];
#pragma unroll
    for (int k = 0; k < (1 << W); ++k)
        v[k] = T[k];
#pragma unroll
    for (int level = 0; level < W; ++level) {
        const bool bit = (w >> level) & 1;
        const int step = 1 << level;
#pragma unroll
        for (int k = 0; k < (1 << W); k += 2 * step)
            v[k] = bit ? v[k + step] : v[k];
    }
    return v[0];
}

// Strong test for one base a (in Montgomery form am) given d, s.
template <int W>
__device__ __forceinline__ bool sprp_window(uint64_t am, uint64_t d, int s, const MontCtx &c)
{
    constexpr int TS = 1 << W;
    uint64_t T[TS];
    T[0] = c.one;
    T[1] = am;
#pragma unroll
    for (int k = 2; k < TS; ++k)
        T[k] = montmul(T[k - 1], am, c.n, c.ninv);
    const int Ld = 64 - __clzll(d);
    const int nwin = (Ld + W - 1) / W;
    int pos = (nwin - 1) * W;
    uint64_t x = select_pow<W>(T, (unsigned)(d >> pos) & (TS - 1));
    for (pos -= W; pos >= 0; pos -= W) {
#pragma unroll
        for (int k = 0; k < W; ++k)
            x = montsqr(x, c.n, c.ninv);
        x = montmul(x, select_pow<W>(T, (unsigned)(d >> pos) & (TS - 1)), c.n, c.ninv);
    }
    if (x == c.one || x == c.mone)
        return true;
    for (int r = 1; r < s; ++r) {
        x = montsqr(x, c.n, c.ninv);
        if (x == c.mone)
            return true;
    }
    return false;
}

// Strong test of odd n >= 2^32 to one base a < 2^32.
template <int W>
__device__ __forceinline__ bool sprp_one_base(uint64_t n, uint32_t a)
{
    const int L = 64 - __clzll(n);
    const MontCtx c = make_ctx(n, L);
    const uint64_t r2 = r2_mod_n(c);
    const uint64_t e = n - 1;
    const int s = __ffsll((long long)e) - 1;
    return sprp_window<W>(to_mont(a, r2, c), e >> s, s, c);
}

// Exclusive prefix of counts[0..nc) into pre[0..nc] (pre[nc] = total), in
// LDS.  nc <= MAX_GRID; blockDim is a multiple of 64, at most 256.
__device__ __forceinline__ void lds_prefix(const uint32_t *__restrict__ counts, uint32_t nc,
                                           uint32_t *pre, uint32_t *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    const uint32_t per = (nc + blockDim.x - 1) / blockDim.x;
    const uint32_t i0 = tid * per;
    uint32_t local = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (i0 + k < nc)
            local += counts[i0 + k];
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
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w)
        before += wsum[w];
    uint32_t run = before + incl - local;
    for (uint32_t k = 0; k < per; ++k) {
        if (i0 + k < nc) {
            pre[i0 + k] = run;
            run += counts[i0 + k];
        }
    }
    if (tid == blockDim.x - 1) {
        uint32_t tot = 0;
        for (int w = 0; w < nwaves; ++w)
            tot += wsum[w];
        pre[nc] = tot;
    }
    __syncthreads();
}

// Region of dense index i: the largest k < nc with pre[k] <= i.
__device__ __forceinline__ uint32_t find_region(const uint32_t *pre, uint32_t nc, uint32_t i)
{
    uint32_t lo = 0, hi = nc;  // pre[lo] <= i < pre[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t call_total(const MrArgs &a)
{
    return a.total_dev ? *a.total_dev : a.total;
}

__global__ void __launch_bounds__(MR_MAX_BLOCK) mr_phase1_kernel(MrArgs a)
{
    __shared__ uint32_t pre[MAX_GRID + 1];
    __shared__ uint32_t wsum[MR_MAX_BLOCK / 64];
    __shared__ uint32_t wave_cnt[MR_MAX_BLOCK / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const uint64_t total = call_total(a);
    const uint64_t chunk_c = classify_chunk(total, a.grid_c);
    const uint64_t chunk_1 = cand_chunk(total, a.grid1);
    lds_prefix(a.counts_c, a.grid_c, pre, wsum);
    const uint32_t n1 = pre[a.grid_c];
    const uint32_t g = blockIdx.x;
    const uint32_t s0 = (uint32_t)((uint64_t)n1 * g / a.grid1);
    const uint32_t s1 = (uint32_t)((uint64_t)n1 * (g + 1) / a.grid1);
    Survivor *region = a.cand + (uint64_t)g * chunk_1;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t filled = 0;
    for (uint32_t r0 = s0; r0 < s1; r0 += blockDim.x) {
        const uint32_t i = r0 + threadIdx.x;
        bool pass = false;
        Survivor sv;
        sv.n = 0;
        sv.out = nullptr;
        if (i < s1) {
            const uint32_t k = find_region(pre, a.grid_c, i);
            sv = a.surv[(uint64_t)k * chunk_c + (i - pre[k])];
            pass = sprp_base2(sv.n);
        }
        const uint64_t m = __ballot(pass);
        if (lane == 0)
            wave_cnt[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < nwaves; ++w) {
            const uint32_t c = wave_cnt[w];
            before += w < wave ? c : 0u;
            all += c;
        }
        if (pass)
            region[filled + before + __popcll(m & lt)] = sv;
        filled += all;
        __syncthreads();  // wave_cnt is rewritten next round
    }
    if (threadIdx.x == 0)
        a.counts1[g] = filled;
}

template <int W>
__global__ void __launch_bounds__(MR_MAX_BLOCK) mr_phase2_kernel(MrArgs a)
{
    __shared__ uint32_t pre[MAX_GRID + 1];
    __shared__ uint32_t wsum[MR_MAX_BLOCK / 64];
    constexpr uint32_t BASES[6] = {325u, 9375u, 28178u, 450775u, 9780504u, 1795265022u};
    constexpr int PER_WAVE = 10;  // candidates per wavefront, 6 lanes each
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const uint64_t total = call_total(a);
    const uint64_t chunk_1 = cand_chunk(total, a.grid1);
    lds_prefix(a.counts1, a.grid1, pre, wsum);
    const uint32_t n2 = pre[a.grid1];
    const uint32_t g = blockIdx.x;
    const uint32_t s0 = (uint32_t)((uint64_t)n2 * g / gridDim.x);
    const uint32_t s1 = (uint32_t)((uint64_t)n2 * (g + 1) / gridDim.x);
    const uint32_t per_round = PER_WAVE * nwaves;
    const int c_in_wave = lane / 6, b = lane - 6 * (lane / 6);
    for (uint32_t r0 = s0; r0 < s1; r0 += per_round) {
        const uint32_t j = r0 + wave * PER_WAVE + c_in_wave;
        const bool active = lane < 6 * PER_WAVE && j < s1;
        bool ok = false;
        uint8_t *out = nullptr;
        if (active) {
            const uint32_t k = find_region(pre, a.grid1, j);
            const Survivor sv = a.cand[(uint64_t)k * chunk_1 + (j - pre[k])];
            out = sv.out;
            ok = sprp_one_base<W>(sv.n, BASES[b]);
        }
        const uint64_t m = __ballot(ok);
        if (active && b == 0 && ((m >> lane) & 0x3full) == 0x3full)
            *out = 1;
    }
}

__global__ void montmul_test_kernel(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b,
                                    const uint64_t *__restrict__ n, uint64_t *__restrict__ out,
                                    uint64_t len)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len)
        return;
    const uint64_t m = n[i];
    const MontCtx c = make_ctx(m, 64 - __clzll(m));
    const uint64_t r2 = r2_mod_n(c);
    const uint64_t am = montmul(a[i], r2, m, c.ninv);
    const uint64_t bm = montmul(b[i], r2, m, c.ninv);
    const uint64_t pm = montmul(am, bm, m, c.ninv);
    out[i] = montmul(pm, 1, m, c.ninv);
}

}  // namespace

hipError_t launch_mr1(const MrArgs &a, int block, hipStream_t s)
{
    mr_phase1_kernel<<<a.grid1, block, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_mr2(const MrArgs &a, unsigned grid2, int block, int window, hipStream_t s)
{
    switch (window) {
    case 1:
        mr_phase2_kernel<1><<<grid2, block, 0, s>>>(a);
        break;
    case 2:
        mr_phase2_kernel<2><<<grid2, block, 0, s>>>(a);
        break;
    case 3:
        mr_phase2_kernel<3><<<grid2, block, 0, s>>>(a);
        break;
    case 4:
        mr_phase2_kernel<4><<<grid2, block, 0, s>>>(a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_montmul_test(const uint64_t *a, const uint64_t *b, const uint64_t *n,
                               uint64_t *out, uint64_t len, hipStream_t s)
{
    const uint64_t blocks = (len + 255) / 256;
    if (blocks > 0x7fffffffull)
        return hipErrorInvalidValue;
    montmul_test_kernel<<<(unsigned)blocks, 256, 0, s>>>(a, b, n, out, len);
    return hipGetLastError();
}

}  // namespace isp
