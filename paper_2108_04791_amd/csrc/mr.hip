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
// of random inputs fail here.  Passers are appended (ballot + one atomic
// per wavefront) to the candidate list.
//
// Phase 2 (base-2 passers, almost all prime): the six remaining bases.  a^d
// uses a fixed window of W bits with a table of a^0..a^(2^W - 1) per lane,
// selected by a compare tree (no dynamic register indexing), so all lanes
// multiply at the same steps.  Then up to s - 1 squarings look for -1.  A
// lane that passes all six stores out = 1 (the classify pass wrote 0).
//
// Both phases are persistent: each wavefront takes 64 list entries at a
// time from an atomic cursor until the list is exhausted, so every wave
// exits once the list is drained.
#include "internal.h"
#include "mont.h"

namespace isp {

namespace {

__device__ __forceinline__ uint64_t lanemask_lt(int lane)
{
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

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

template <int W>
__device__ __forceinline__ bool mr_remaining_bases(uint64_t n)
{
    const int L = 64 - __clzll(n);
    const MontCtx c = make_ctx(n, L);
    const uint64_t r2 = r2_mod_n(c);
    const uint64_t e = n - 1;
    const int s = __ffsll((long long)e) - 1;
    const uint64_t d = e >> s;
    constexpr uint32_t BASES[6] = {325u, 9375u, 28178u, 450775u, 9780504u, 1795265022u};
#pragma unroll 1
    for (int b = 0; b < 6; ++b) {
        const uint64_t am = to_mont(BASES[b], r2, c);
        if (!sprp_window<W>(am, d, s, c))
            return false;
    }
    return true;
}

__global__ void __launch_bounds__(MR_MAX_BLOCK) mr_phase1_kernel(const Survivor *__restrict__ list,
                                                        Survivor *__restrict__ cand,
                                                        Counters *__restrict__ ctr)
{
    const uint32_t total = ctr->survivors;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lanemask_lt(lane);
    for (;;) {
        uint32_t chunk = 0;
        if (lane == 0)
            chunk = atomicAdd(&ctr->work1, 64u);
        chunk = __shfl(chunk, 0, 64);
        if (chunk >= total)
            break;
        const uint32_t i = chunk + lane;
        const bool active = i < total;
        Survivor sv;
        sv.n = 0;
        sv.out = nullptr;
        bool pass = false;
        if (active) {
            sv = list[i];
            pass = sprp_base2(sv.n);
        }
        const uint64_t m = __ballot(pass);
        uint32_t base = 0;
        if (lane == 0 && m)
            base = atomicAdd(&ctr->candidates, (uint32_t)__popcll(m));
        base = __shfl(base, 0, 64);
        if (pass)
            cand[base + __popcll(m & lt)] = sv;
    }
}

template <int W>
__global__ void __launch_bounds__(MR_MAX_BLOCK) mr_phase2_kernel(const Survivor *__restrict__ cand,
                                                        Counters *__restrict__ ctr)
{
    const uint32_t total = ctr->candidates;
    const int lane = threadIdx.x & 63;
    for (;;) {
        uint32_t chunk = 0;
        if (lane == 0)
            chunk = atomicAdd(&ctr->work2, 64u);
        chunk = __shfl(chunk, 0, 64);
        if (chunk >= total)
            break;
        const uint32_t i = chunk + lane;
        if (i < total) {
            const Survivor sv = cand[i];
            if (mr_remaining_bases<W>(sv.n))
                *sv.out = 1;
        }
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

hipError_t launch_mr1(const Workspace &ws, const Tuning &t, int cus, hipStream_t s)
{
    const unsigned grid = (unsigned)(cus * t.mr_blocks_per_cu);
    const Survivor *list = t.mr_bins > 0 ? ws.sorted : ws.surv;
    Survivor *cand = t.mr_bins > 0 ? ws.surv : ws.sorted;
    mr_phase1_kernel<<<grid, t.mr_block, 0, s>>>(list, cand, ws.ctr);
    return hipGetLastError();
}

hipError_t launch_mr2(const Workspace &ws, const Tuning &t, int cus, hipStream_t s)
{
    const unsigned grid = (unsigned)(cus * t.mr_blocks_per_cu);
    const Survivor *cand = t.mr_bins > 0 ? ws.surv : ws.sorted;
    switch (t.mr_window) {
    case 1:
        mr_phase2_kernel<1><<<grid, t.mr_block, 0, s>>>(cand, ws.ctr);
        break;
    case 2:
        mr_phase2_kernel<2><<<grid, t.mr_block, 0, s>>>(cand, ws.ctr);
        break;
    case 3:
        mr_phase2_kernel<3><<<grid, t.mr_block, 0, s>>>(cand, ws.ctr);
        break;
    case 4:
        mr_phase2_kernel<4><<<grid, t.mr_block, 0, s>>>(cand, ws.ctr);
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
