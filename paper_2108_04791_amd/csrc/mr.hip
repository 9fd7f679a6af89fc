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
// bits of n - 1 from the top in a loop whose count is the same on every lane
// of a wavefront (L - 2 steps for the longest n in it); the multiply by 2 is
// a modular doubling (the ModAdd of section 2.2) selected without a branch.
// About 4 in 5 survivors of random inputs fail here (their output byte keeps
// the 0 that classify wrote).  Passers go to the workgroup's own region, and
// the workgroup then computes each passer's Montgomery constants once for
// phase 2.
//
// Phase 2 (base-2 passers): in two rounds per workgroup over its slice of
// the candidates.  Round 1 tests base 325, one candidate per lane, and
// lists the passers; round 2 runs the five other bases of those as five
// independent tasks per candidate, laid out densely over the lanes.  A
// composite that passes base 2 (a strong pseudoprime, e.g. a Carmichael
// number) almost always fails 325, so it costs one base instead of six.  A
// candidate that passes 325 stores out = 1 in round 1, and a lane whose base
// fails in round 2 stores out = 0 after the workgroup barrier between the
// rounds, so the verdict is the AND of the bases without any cross-lane step
// (several lanes may store the same 0).  Only about as many bytes as there
// are primes are written, scattered, by this phase, and none by phase 1.
// a^d uses a fixed window of W bits with the lane's table of
// a^0..a^(2^W - 1) in LDS, so all lanes multiply at the same steps; then up
// to s - 1 squarings look for -1.
//
// Work split without global atomics (a single hot device-scope atomic
// sustains only about 1e8 operations per second on this part): each
// workgroup scans the producer's per-workgroup counts in LDS and takes an
// equal slice of the resulting dense index space; inside the workgroup each
// wavefront takes the next 64 items of the slice from an LDS counter, so the
// wavefronts the issue arbiter favours (older ones first) simply do more of
// the slice.  An item's producer region is found by a search in LDS that
// starts from the wavefront's previous region.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"
#include "mont.h"

namespace isp {

namespace {

// Largest value of v over the wavefront for 0 <= v < 2^BITS, as a
// wavefront-uniform (scalar) value, built from the top bit down with one
// ballot per bit; every lane must be active.
template <int BITS>
__device__ __forceinline__ int wave_max(int v)
{
    int acc = 0;
#pragma unroll
    for (int b = 1 << (BITS - 1); b > 0; b >>= 1)
        if (__ballot(v >= acc + b) != 0)
            acc += b;
    return acc;
}

// The largest bit length L in [33, 64] of a wavefront's values.
__device__ __forceinline__ int wave_max_len(int L) { return 33 + wave_max<5>(L - 33); }

// Strong probable-prime test to base 2 for odd n >= 2^32, n - 1 = 2^s d.
// Called with all 64 lanes of the wavefront active.
//
// x runs over x_t = 2^(floor((n-1) / 2^t)) (Montgomery form) for t from the
// top down to 1: one squaring per bit and a modular doubling when the bit
// is set.  x_s = 2^d, and below s the bits are zero, so x_t = 2^(2^(s-t) d)
// for t <= s: n passes iff x_s = 1 or x_t = -1 for some 1 <= t <= s.
//
// Every lane runs the same steps: bits Lmax - 2 down to 1, Lmax being the
// largest bit length in the wavefront.  A lane with a shorter n starts from
// x = 1 and squares it through its leading zero bits, so its first set bit
// makes x = 2 exactly where its own exponent starts.  The loop count is the
// same on all lanes (a scalar loop), and only the last smax steps (smax: the
// largest s in the wavefront) compare.  The bit of each step is read from
// the 32-bit half of n - 1 that holds it, one bit-field extract.
//
// SQ (wavefront-uniform) by the largest n of the wavefront: 0 below 2^60,
// 1 below 2^62, 2 below 2^63, 3 otherwise.  Below 2^63 the squares take the
// carry-free form (montsqr63).  Below 2^60 the steps before the comparisons
// keep x in (0, 4n) (lazy squares, whose input may be below 4n there, and a
// plain shift for the doubling); below 2^62 they keep it in [0, 2n)
// (reduced squares of inputs below 2n, and the shift).
template <int SQ>
__device__ __forceinline__ bool sprp_base2_run(uint64_t n, const MontCtx &c, uint64_t e, int s,
                                               int L, int Lmax, int smax)
{
    auto sqr = [&](uint64_t y) {
        return SQ == 3 ? montsqr(y, n, c.ninv) : montsqr63(y, n, c.ninv);
    };
    // bit Lmax - 1: the leading one of the longest lanes (x = 2), a leading
    // zero of the others (x = 1)
    uint64_t x = L == Lmax ? dbl_mod(c.one, n) : c.one;
    // 2x mod n for x < n: 2x >= n exactly when x >= (n + 1) / 2 (n is odd),
    // and then 2x - n = 2x + (2^64 - n) modulo 2^64, carry or not.
    const uint64_t half = (n >> 1) + 1, neg_n = 0 - n;
    auto step = [&](uint32_t bit) {
        x = sqr(x);
        // x <- 2^bit x mod n in one instruction: (x << bit) + (2^64 - n) when
        // the bit is set and 2x wraps past n, (x << bit) + 0 otherwise
        const uint64_t sub = (bit != 0 && x >= half) ? neg_n : 0;
        x = shl_add(x, bit, sub);
    };
    // steps for bits hi_t down to lo_t of n - 1, held in `word` at t - base
    auto steps = [&](uint32_t word, int base, int hi_t, int lo_t) {
        for (int t = hi_t; t >= lo_t; --t) {
            const uint32_t bit = __builtin_amdgcn_ubfe(word, (uint32_t)(t - base), 1u);
            if constexpr (SQ == 0)
                x = montsqr63_lazy(x, n, c.ninv) << bit;
            else if constexpr (SQ == 1)
                x = montsqr63(x, n, c.ninv) << bit;
            else
                step(bit);
        }
    };
    // bits Lmax - 2 .. smax + 1, those above 31 first
    const int top = Lmax - 2, low = smax + 1;
    steps(hi32(e), 32, top, low > 32 ? low : 32);
    steps(lo32(e), 0, top < 31 ? top : 31, low);
    // bits min(smax, Lmax - 2) .. 1, comparing (the first square reduces x)
    bool pass = false;
    for (int t = smax < top ? smax : top; t >= 1; --t) {
        step((uint32_t)(e >> t) & 1u);
        pass |= (t <= s && x == c.mone) || (t == s && x == c.one);
    }
    return pass;
}

// c receives n's Montgomery context (kept for the passers' constants).
__device__ __forceinline__ bool sprp_base2(uint64_t n, MontCtx &c)
{
    const int L = 64 - __clzll(n);
    const uint64_t e = n - 1;
    const int s = __ffsll((long long)e) - 1;  // 1 .. 63
    const int Lmax = wave_max_len(L), smax = wave_max<6>(s);
    c.n = n;
    c.ninv = inv64(n);
    c.one = r_mod_n_wide(n);
    c.mone = n - c.one;
    if (Lmax <= 60)
        return sprp_base2_run<0>(n, c, e, s, L, Lmax, smax);
    if (Lmax <= 62)
        return sprp_base2_run<1>(n, c, e, s, L, Lmax, smax);
    if (Lmax == 63)
        return sprp_base2_run<2>(n, c, e, s, L, Lmax, smax);
    return sprp_base2_run<3>(n, c, e, s, L, Lmax, smax);
}

// Strong test for one base (am: its Montgomery form) with n - 1 = 2^s d.
// a^d by a fixed window of W bits: the lane's table a^0 .. a^(2^W - 1) sits
// in LDS, column threadIdx.x of tbl[2^W][blockDim] (each lane reads only
// its own column, so no barrier is needed and the rows are bank-aligned).
// SQ as for sprp_base2_run.  SQ 0 (every n of the wavefront below 2^62):
// products stay in (0, 2n) and are reduced once before the comparisons.
template <int W, int SQ>
__device__ __forceinline__ bool sprp_window(uint64_t am, uint64_t d, int s, const MontCtx &c,
                                            uint64_t *tbl)
{
    constexpr int TS = 1 << W;
    auto mul = [&](uint64_t x, uint64_t y) {
        return SQ == 0 ? montmul_lazy(x, y, c.n, c.ninv) : montmul(x, y, c.n, c.ninv);
    };
    // (the lazy square keeps the general form: with the carry-free square
    // the compiler needs one more register move per step)
    auto sqr = [&](uint64_t x) {
        return SQ == 0 ? montmul_lazy(x, x, c.n, c.ninv)
                       : SQ == 1 ? montsqr63(x, c.n, c.ninv) : montsqr(x, c.n, c.ninv);
    };
    const unsigned col = threadIdx.x, stride = blockDim.x;
    uint64_t p = c.one;
    tbl[col] = p;
#pragma unroll
    for (int k = 1; k < TS; ++k) {
        p = k == 1 ? am : mul(p, am);
        tbl[k * stride + col] = p;
    }
    // windows from the wavefront's longest d down: a lane with a shorter d
    // reads window value 0 (table entry 1) until its own top window, so every
    // lane runs the same scalar loop (all lanes must be active)
    const int Ld = 64 - __clzll(d);
    const int nwin = wave_max<6>((Ld + W - 1) / W);  // <= 63
    int pos = (nwin - 1) * W;  // at most 63 - W: d < 2^63
    uint64_t x = tbl[((unsigned)(d >> pos) & (TS - 1)) * stride + col];
    for (pos -= W; pos >= 0; pos -= W) {
#pragma unroll
        for (int k = 0; k < W; ++k)
            x = sqr(x);
        x = mul(x, tbl[((unsigned)(d >> pos) & (TS - 1)) * stride + col]);
    }
    if (SQ == 0 && x >= c.n)
        x -= c.n;
    if (x == c.one || x == c.mone)
        return true;
    for (int r = 1; r < s; ++r) {
        x = SQ == 2 ? montsqr(x, c.n, c.ninv) : montsqr63(x, c.n, c.ninv);
        if (x == c.mone)
            return true;
    }
    return false;
}

// Strong test of odd n >= 2^32 to one base a < 2^32, given n's Montgomery
// constants.  Called with all 64 lanes of the wavefront active.
template <int W>
__device__ __forceinline__ bool sprp_one_base(uint64_t n, const MontPrep &pr, uint32_t a,
                                              uint64_t *tbl)
{
    MontCtx c;
    c.n = n;
    c.ninv = pr.ninv;
    c.one = pr.one;
    c.mone = n - pr.one;
    const uint64_t e = n - 1;
    const int s = __ffsll((long long)e) - 1;
    const uint64_t am = to_mont(a, pr.r2, c);
    const int Lmax = wave_max_len(64 - __clzll(n));
    if (Lmax <= 62)
        return sprp_window<W, 0>(am, e >> s, s, c, tbl);
    if (Lmax == 63)
        return sprp_window<W, 1>(am, e >> s, s, c, tbl);
    return sprp_window<W, 2>(am, e >> s, s, c, tbl);
}

// R^2 mod n from n's n^-1 and R mod n (the other two constants).
__device__ __forceinline__ uint64_t r2_of(uint64_t n, const MontPrep &p)
{
    MontCtx c;
    c.n = n;
    c.ninv = p.ninv;
    c.one = p.one;
    c.mone = n - p.one;
    return r2_mod_n(c);
}

// The Montgomery constants of odd n >= 2^32.
__device__ __forceinline__ MontPrep mont_prep(uint64_t n)
{
    const MontCtx c = make_ctx(n, 64 - __clzll(n));
    MontPrep pr;
    pr.ninv = c.ninv;
    pr.one = c.one;
    pr.r2 = r2_mod_n(c);
    return pr;
}

// ------------------------------------------------------------------ Lucas
// Strong Lucas probable-prime test with Selfridge's parameters (Baillie and
// Wagstaff, Math. Comp. 35, 1980): D is the first of 5, -7, 9, -11, ... with
// Jacobi symbol (D/n) = -1, P = 1, Q = (1 - D) / 4.  With n + 1 = 2^s d, n
// is a strong Lucas probable prime iff U_d = 0 or V_(d 2^r) = 0 (mod n) for
// some 0 <= r < s.  Together with the base-2 strong test this is the
// Baillie-PSW test, the alternative the paper names as future work (section
// 10.1); it selects the same primes below 2^64.

// Jacobi symbol (a/m) for odd m > 0, by quadratic reciprocity.
__device__ __forceinline__ int jacobi32(uint32_t a, uint32_t m, int t)
{
    while (a != 0) {
        while ((a & 1) == 0) {
            a >>= 1;
            const uint32_t r = m & 7;
            if (r == 3 || r == 5)
                t = -t;
        }
        const uint32_t x = a;
        a = m;
        m = x;
        if ((a & 3) == 3 && (m & 3) == 3)
            t = -t;
        a %= m;
    }
    return m == 1 ? t : 0;
}

// (D/n) for odd n > |D|, |D| odd and < 2^31.
__device__ __forceinline__ int jacobi_d_n(int32_t D, uint64_t n)
{
    int t = 1;
    const uint32_t a = (uint32_t)(D < 0 ? -D : D);
    if (D < 0 && (n & 3) == 3)
        t = -t;  // (-1/n)
    if ((a & 3) == 3 && (n & 3) == 3)
        t = -t;  // reciprocity, both odd
    return jacobi32((uint32_t)(n % a), a, t);
}

__device__ __forceinline__ uint32_t gcd32(uint32_t a, uint32_t b)
{
    while (b) {
        const uint32_t r = a % b;
        a = b;
        b = r;
    }
    return a;
}

__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t n)
{
    return a >= b ? a - b : a - b + n;
}

// 1: strong Lucas probable prime; 0: composite; -1: no D found (the caller
// falls back to the remaining Miller-Rabin bases).
__device__ __forceinline__ int strong_lucas(uint64_t n)
{
    if (n == ~(uint64_t)0)
        return 0;  // 3 divides 2^64 - 1 (and n + 1 would wrap)
    // a perfect square has no D with (D/n) = -1
    const uint64_t r = isqrt_u64(n);
    if (r * r == n)
        return 0;
    int32_t D = 5;
    int k = 0;
    for (;; ++k) {
        if (k >= 4096)
            return -1;
        const int j = jacobi_d_n(D, n);
        if (j == -1)
            break;
        if (j == 0)
            return 0;  // gcd(|D|, n) > 1 and |D| < n
        D = D > 0 ? -(D + 2) : -D + 2;
    }
    const int32_t Q = (1 - D) / 4;
    const uint32_t aq = (uint32_t)(Q < 0 ? -Q : Q);
    if (aq > 1 && gcd32((uint32_t)(n % aq), aq) > 1)
        return 0;
    const int L = 64 - __clzll(n);
    const MontCtx c = make_ctx(n, L);
    const uint64_t r2 = r2_mod_n(c);
    const uint64_t qm = to_mont(Q < 0 ? n - aq : (uint64_t)aq, r2, c);
    const uint64_t e = n + 1;
    const int s = __ffsll((long long)e) - 1;
    const uint64_t d = e >> s;
    const int Ld = 64 - __clzll(d);
    // ladder over the bits of d: (V_k, V_(k+1), Q^k) -> k' = 2k + bit
    uint64_t vk = dbl_mod(c.one, n);  // V_0 = 2
    uint64_t vk1 = c.one;             // V_1 = P = 1
    uint64_t qk = c.one;              // Q^0
    for (int i = Ld - 1; i >= 0; --i) {
        const bool bit = (d >> i) & 1;
        const uint64_t w = sub_mod(montmul(vk, vk1, n, c.ninv), qk, n);  // V_(2k+1)
        const uint64_t qkq = montmul(qk, qm, n, c.ninv);                // Q^(k+1)
        const uint64_t a = bit ? vk1 : vk;
        const uint64_t qb = bit ? qkq : qk;                              // Q^(k+bit)
        const uint64_t sq = sub_mod(montsqr(a, n, c.ninv), dbl_mod(qb, n), n);  // V_(2k+2bit)
        qk = montmul(qb, qk, n, c.ninv);                                 // Q^(2k+bit)
        vk = bit ? w : sq;
        vk1 = bit ? sq : w;
    }
    // U_d = (2 V_(d+1) - P V_d) / D, and D is invertible mod n
    if (dbl_mod(vk1, n) == vk || vk == 0)
        return 1;
    for (int rr = 1; rr < s; ++rr) {
        vk = sub_mod(montsqr(vk, n, c.ninv), dbl_mod(qk, n), n);  // V_(2m) = V_m^2 - 2 Q^m
        if (vk == 0)
            return 1;
        qk = montsqr(qk, n, c.ninv);
    }
    return 0;
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

// Region of dense index i: the largest k < nc with pre[k] <= i, given a k
// with pre[k] <= i to start from.  A lane's indices only grow, so its
// previous region is such a start: one LDS read while i stays in it, else a
// binary search above it.  pre[nc] is the total, so pre[k + 1] is readable.
__device__ __forceinline__ uint32_t find_region(const uint32_t *pre, uint32_t nc, uint32_t k,
                                                uint32_t i)
{
    if (pre[k + 1] > i)
        return k;
    uint32_t lo = k + 1, hi = nc;  // pre[lo] <= i < pre[hi]
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

// Passers of one phase-1 workgroup, grouped before their constants are
// written (when there are at most PASS_PER_THREAD per thread): by bit
// length (64 down to 33) and then by s (1 .. 4, >= 5), so that a phase-2
// wavefront's tasks share the window count of their d, the length of their
// -1 chain and the form of their products.
constexpr int PASS_PER_THREAD = 4;
constexpr int PASS_S_KEYS = 5;
constexpr int PASS_BINS = 32 * PASS_S_KEYS;

__device__ __forceinline__ int pass_key(uint64_t n)
{
    const int s = __ffsll((long long)(n - 1)) - 1;  // >= 1: n is odd
    return __clzll(n) * PASS_S_KEYS + (s < PASS_S_KEYS ? s : PASS_S_KEYS) - 1;
}

__global__ void __launch_bounds__(MR_MAX_BLOCK) mr_phase1_kernel(MrArgs a)
{
    extern __shared__ uint64_t dyn[];
    uint32_t *pre = reinterpret_cast<uint32_t *>(dyn);  // grid_c + 1 entries
    __shared__ uint32_t wsum[MR_MAX_BLOCK / 64];
    __shared__ uint32_t next, fill;
    const int lane = threadIdx.x & 63;
    const uint64_t total = call_total(a);
    const uint64_t chunk_c = classify_chunk(total, a.grid_c);
    const uint64_t chunk_1 = cand_chunk(total, a.grid1);
    lds_prefix(a.counts_c, a.grid_c, pre, wsum);
    const uint32_t n1 = pre[a.grid_c];
    const uint32_t g = blockIdx.x;
    const uint32_t s0 = (uint32_t)((uint64_t)n1 * g / a.grid1);
    const uint32_t s1 = (uint32_t)((uint64_t)n1 * (g + 1) / a.grid1);
    if (threadIdx.x == 0) {
        next = s0;
        fill = 0;
    }
    __syncthreads();
    Survivor *region = a.cand + (uint64_t)g * chunk_1;
    MontPrep *prep = a.prep ? a.prep + (uint64_t)g * chunk_1 : nullptr;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t k = 0;
    for (;;) {
        // the wavefront takes the next 64 survivors of the workgroup's slice
        uint32_t i0 = 0;
        if (lane == 0)
            i0 = atomicAdd(&next, 64u);
        i0 = __shfl(i0, 0, 64);
        if (i0 >= s1)
            break;
        const uint32_t i = i0 + lane;
        Survivor sv;
        sv.n = 0;
        sv.out = nullptr;
        if (i < s1) {
            k = find_region(pre, a.grid_c, k, i);
            sv = a.surv[(uint64_t)k * chunk_c + (i - pre[k])];
        }
        // idle lanes test a copy of an active lane's value, so the whole
        // wavefront runs sprp_base2 together
        const uint64_t act = __ballot(i < s1);
        const uint64_t nv = __shfl(sv.n, __ffsll((long long)act) - 1, 64);
        MontCtx c;
        const bool pass = sprp_base2(i < s1 ? sv.n : nv, c) && i < s1;
        const uint64_t m = __ballot(pass);
        if (m != 0) {
            uint32_t at = 0;
            if (lane == 0)
                at = atomicAdd(&fill, (uint32_t)__popcll(m));
            at = __shfl(at, 0, 64);
            if (pass) {
                const uint32_t pos = at + __popcll(m & lt);
                region[pos] = sv;
                if (prep) {
                    // n^-1 and R mod n now; R^2 mod n below, once sorted
                    prep[pos].ninv = c.ninv;
                    prep[pos].one = c.one;
                }
            }
        }
    }
    __syncthreads();
    // the Montgomery constants of this workgroup's passers, once each, for
    // all the later tasks of each (dense over the workgroup's threads)
    const uint32_t npass = fill;
    if (prep) {
        if (npass <= PASS_PER_THREAD * blockDim.x) {
            // counting sort by pass_key (block-uniform branch): the sorted
            // order as indices in LDS, then every thread reads its (at most
            // PASS_PER_THREAD) entries into registers before any is rewritten
            __shared__ uint16_t perm[PASS_PER_THREAD * MR_MAX_BLOCK];
            __shared__ uint32_t bins[PASS_BINS];
            for (int b = threadIdx.x; b < PASS_BINS; b += blockDim.x)
                bins[b] = 0;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < npass; i += blockDim.x)
                atomicAdd(&bins[pass_key(region[i].n)], 1u);
            __syncthreads();
            if (threadIdx.x < 64) {
                // exclusive scan of the bins by the first wavefront, each
                // lane summing a run of consecutive bins
                constexpr int PER = (PASS_BINS + 63) / 64;
                const int b0 = lane * PER;
                uint32_t local = 0;
#pragma unroll
                for (int q = 0; q < PER; ++q)
                    local += b0 + q < PASS_BINS ? bins[b0 + q] : 0u;
                uint32_t incl = local;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o, 64);
                    if (lane >= o)
                        incl += y;
                }
                uint32_t run = incl - local;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    if (b0 + q < PASS_BINS) {
                        const uint32_t c = bins[b0 + q];
                        bins[b0 + q] = run;
                        run += c;
                    }
                }
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < npass; i += blockDim.x)
                perm[atomicAdd(&bins[pass_key(region[i].n)], 1u)] = (uint16_t)i;
            __syncthreads();
            Survivor mine[PASS_PER_THREAD];
            MontPrep mp[PASS_PER_THREAD];
#pragma unroll
            for (int k = 0; k < PASS_PER_THREAD; ++k) {
                const uint32_t i = threadIdx.x + k * blockDim.x;
                if (i < npass) {
                    mine[k] = region[perm[i]];
                    mp[k] = prep[perm[i]];
                }
            }
            __syncthreads();  // every entry is read before any is rewritten
#pragma unroll
            for (int k = 0; k < PASS_PER_THREAD; ++k) {
                const uint32_t i = threadIdx.x + k * blockDim.x;
                if (i < npass) {
                    region[i] = mine[k];
                    mp[k].r2 = r2_of(mine[k].n, mp[k]);
                    prep[i] = mp[k];
                }
            }
        } else {
            for (uint32_t i = threadIdx.x; i < npass; i += blockDim.x)
                prep[i].r2 = r2_of(region[i].n, prep[i]);
        }
    }
    if (threadIdx.x == 0)
        a.counts1[g] = npass;
}

template <int W>
__global__ void __launch_bounds__(MR_MAX_BLOCK) mr_phase2_kernel(MrArgs a)
{
    // dynamic LDS: the window tables (2^W x blockDim values), then the
    // prefix of the base-2 counts (grid1 + 1 entries)
    extern __shared__ uint64_t dyn[];
    uint64_t *tbl = dyn;
    uint32_t *pre = reinterpret_cast<uint32_t *>(dyn + (1u << W) * blockDim.x);
    __shared__ uint32_t wsum[MR_MAX_BLOCK / 64];
    __shared__ uint32_t next, kept, next2;
    constexpr uint32_t BASES[6] = {325u, 9375u, 28178u, 450775u, 9780504u, 1795265022u};
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t total = call_total(a);
    const uint64_t chunk_1 = cand_chunk(total, a.grid1);
    lds_prefix(a.counts1, a.grid1, pre, wsum);
    // the workgroup's slice of the candidates (dense over all base-2 regions)
    const uint32_t ncand = pre[a.grid1];
    const uint32_t g = blockIdx.x;
    const uint32_t c0 = (uint32_t)((uint64_t)ncand * g / gridDim.x);
    const uint32_t c1 = (uint32_t)((uint64_t)ncand * (g + 1) / gridDim.x);
    // round 2's list: the slots of the slice's candidates that pass base
    // 325, at keep[c0 ...] (the survivor regions are free by now)
    uint32_t *keep = a.keep + c0;
    if (threadIdx.x == 0) {
        next = c0;
        kept = 0;
        next2 = 0;
    }
    __syncthreads();
    // round 1: base 325, one candidate per lane
    uint32_t k = 0;
    for (;;) {
        uint32_t j0 = 0;
        if (lane == 0)
            j0 = atomicAdd(&next, 64u);
        j0 = __shfl(j0, 0, 64);
        if (j0 >= c1)
            break;
        // idle lanes at the end of the slice repeat candidate j0 (lane 0's),
        // so the whole wavefront runs the test together; only real ones count
        const bool real = j0 + lane < c1;
        const uint32_t j = real ? j0 + lane : j0;
        k = find_region(pre, a.grid1, k, j);
        const uint32_t slot = (uint32_t)((uint64_t)k * chunk_1 + (j - pre[k]));
        const Survivor sv = a.cand[slot];
        const MontPrep pr = a.prep[slot];
        const bool ok = sprp_one_base<W>(sv.n, pr, BASES[0], tbl);
        if (ok && real)
            *sv.out = 1;  // provisional: a failing base of round 2 clears it
        const uint64_t m = __ballot(ok && real);
        if (m != 0) {
            uint32_t at = 0;
            if (lane == 0)
                at = atomicAdd(&kept, (uint32_t)__popcll(m));
            at = __shfl(at, 0, 64);
            if (ok && real)
                keep[at + __popcll(m & lt)] = slot;
        }
    }
    __syncthreads();  // the slice's list is complete (and visible to the workgroup)
    // round 2: the five other bases of the kept candidates, five independent
    // tasks each, dense over the lanes (task 5i + b: base b + 1 of kept i)
    const uint32_t tasks = 5u * kept;
    for (;;) {
        uint32_t t0 = 0;
        if (lane == 0)
            t0 = atomicAdd(&next2, 64u);
        t0 = __shfl(t0, 0, 64);
        if (t0 >= tasks)
            break;
        const bool real = t0 + lane < tasks;
        const uint32_t t = real ? t0 + lane : t0;
        const uint32_t i = t / 5u;
        const uint32_t b = t - 5u * i + 1u;
        const uint32_t slot = keep[i];
        const Survivor sv = a.cand[slot];
        const MontPrep pr = a.prep[slot];
        if (!sprp_one_base<W>(sv.n, pr, BASES[b], tbl) && real)
            *sv.out = 0;
    }
}

// Remaining test of every base-2 passer by the strong Lucas test (one task
// per candidate; see strong_lucas).  A prime stores out = 1.
template <int W>
__global__ void __launch_bounds__(MR_MAX_BLOCK) lucas_kernel(MrArgs a)
{
    extern __shared__ uint64_t dyn[];
    uint64_t *tbl = dyn;  // used only by the rare fallback to the Miller-Rabin bases
    uint32_t *pre = reinterpret_cast<uint32_t *>(dyn + (1u << W) * blockDim.x);
    __shared__ uint32_t wsum[MR_MAX_BLOCK / 64];
    __shared__ uint32_t next;
    constexpr uint32_t BASES[6] = {325u, 9375u, 28178u, 450775u, 9780504u, 1795265022u};
    const int lane = threadIdx.x & 63;
    const uint64_t total = call_total(a);
    const uint64_t chunk_1 = cand_chunk(total, a.grid1);
    lds_prefix(a.counts1, a.grid1, pre, wsum);
    const uint32_t n2 = pre[a.grid1];
    const uint32_t g = blockIdx.x;
    const uint32_t s0 = (uint32_t)((uint64_t)n2 * g / gridDim.x);
    const uint32_t s1 = (uint32_t)((uint64_t)n2 * (g + 1) / gridDim.x);
    if (threadIdx.x == 0)
        next = s0;
    __syncthreads();
    uint32_t k = 0;
    for (;;) {
        uint32_t j0 = 0;
        if (lane == 0)
            j0 = atomicAdd(&next, 64u);
        j0 = __shfl(j0, 0, 64);
        if (j0 >= s1)
            break;
        // idle lanes at the end of the slice repeat candidate j0 (lane 0's),
        // so the whole wavefront runs the tests together
        const bool real = j0 + lane < s1;
        const uint32_t j = real ? j0 + lane : j0;
        k = find_region(pre, a.grid1, k, j);
        const uint64_t slot = (uint64_t)k * chunk_1 + (j - pre[k]);
        const Survivor sv = a.cand[slot];
        int v = strong_lucas(sv.n);
        const bool need = v < 0;
        if (__ballot(need) != 0) {
            // the Miller-Rabin bases run on every lane (they need the whole
            // wavefront); only the lanes without a Lucas verdict use them
            const MontPrep pr = mont_prep(sv.n);
            bool w = true;
            for (int b = 0; b < 6; ++b)
                w = sprp_one_base<W>(sv.n, pr, BASES[b], tbl) && w;
            if (need)
                v = w ? 1 : 0;
        }
        if (v && real)
            *sv.out = 1;
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

size_t mr1_lds(const MrArgs &a) { return ((size_t)a.grid_c + 1) * sizeof(uint32_t); }

size_t mr2_lds(const MrArgs &a, int block, int window)
{
    return ((size_t)block << window) * sizeof(uint64_t) + ((size_t)a.grid1 + 1) * sizeof(uint32_t);
}

hipError_t launch_mr1(const MrArgs &a, int block, hipStream_t s)
{
    mr_phase1_kernel<<<a.grid1, block, mr1_lds(a), s>>>(a);
    return hipGetLastError();
}

// Workgroups of phase 2 that fit on one CU at once (LDS or registers
// permitting): its grid is all resident, since each workgroup takes one
// static slice.
int mr2_resident_per_cu(int block, int window, size_t lds)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, size_t>, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_tuple(block, window, lds);
    auto it = cache.find(key);
    if (it != cache.end())
        return it->second;
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (window) {
    case 1:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mr_phase2_kernel<1>, block, lds);
        break;
    case 2:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mr_phase2_kernel<2>, block, lds);
        break;
    case 3:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mr_phase2_kernel<3>, block, lds);
        break;
    case 4:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mr_phase2_kernel<4>, block, lds);
        break;
    }
    if (e != hipSuccess || nb < 1)
        nb = 1;
    cache[key] = nb;
    return nb;
}

hipError_t launch_lucas(const MrArgs &a, int cus, int per_cu, unsigned max_grid, int block,
                        hipStream_t s)
{
    constexpr int W = 3;
    const size_t lds = mr2_lds(a, block, W);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lucas_kernel<W>, block, lds) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    const unsigned grid = std::max(
        1u, std::min({(unsigned)MAX_GRID, max_grid, (unsigned)(cus * std::min(per_cu, nb))}));
    lucas_kernel<W><<<grid, block, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_mr2(const MrArgs &a, int cus, int per_cu, unsigned max_grid, int block,
                      int window, hipStream_t s)
{
    const size_t lds = mr2_lds(a, block, window);
    const int fit = mr2_resident_per_cu(block, window, lds);
    const unsigned grid = std::max(
        1u, std::min({(unsigned)MAX_GRID, max_grid, (unsigned)(cus * std::min(per_cu, fit))}));
    switch (window) {
    case 1:
        mr_phase2_kernel<1><<<grid, block, lds, s>>>(a);
        break;
    case 2:
        mr_phase2_kernel<2><<<grid, block, lds, s>>>(a);
        break;
    case 3:
        mr_phase2_kernel<3><<<grid, block, lds, s>>>(a);
        break;
    case 4:
        mr_phase2_kernel<4><<<grid, block, lds, s>>>(a);
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
