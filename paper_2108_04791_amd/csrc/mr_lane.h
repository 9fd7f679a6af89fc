// mr_lane.h -- strong tests in a single lane, with each lane running its own
// loop counts (no cross-lane step), for the fused kernel that decides a
// small array in one launch.
//
// Paper, section 2.1: with n - 1 = 2^s d (d odd), a prime n has, for every
// base a, a^d = 1 or a^(2^r d) = -1 (mod n) for some 0 <= r < s (Eq. 1-3,
// read as the standard strong test); Eq. 4's seven bases make the test
// exact below 2^64.  Every n here is odd and >= 2^32, above every base, so
// no base needs reducing.
#pragma once
#include "mont.h"

namespace isp {

struct LaneMr {
    MontCtx c;
    uint64_t d;  // n - 1 = 2^s d
    int s;
    int top;     // index of d's leading one
};

__device__ __forceinline__ LaneMr lane_mr(uint64_t n)
{
    LaneMr m;
    m.c = make_ctx(n, 64 - __clzll(n));
    const uint64_t e = n - 1;
    m.s = __ffsll((long long)e) - 1;
    m.d = e >> m.s;
    m.top = 63 - __clzll(m.d);
    return m;
}

// x = 1 or x = -1 at r = 0, or x = -1 after r squarings, 1 <= r < s.
__device__ __forceinline__ bool strong_tail(uint64_t x, const LaneMr &m)
{
    if (x == m.c.one || x == m.c.mone)
        return true;
    for (int r = 1; r < m.s; ++r) {
        x = montsqr(x, m.c.n, m.c.ninv);
        if (x == m.c.mone)
            return true;
    }
    return false;
}

// Base 2: 2^d left to right, squaring and, where the bit is set, doubling
// (the ModAdd of x and x) in place of a product.
__device__ __forceinline__ bool sprp2_lane(const LaneMr &m)
{
    const uint64_t n = m.c.n;
    uint64_t x = dbl_mod(m.c.one, n);  // the leading one: 2 in Montgomery form
    for (int i = m.top - 1; i >= 0; --i) {
        x = montsqr(x, n, m.c.ninv);
        if ((m.d >> i) & 1)
            x = dbl_mod(x, n);
    }
    return strong_tail(x, m);
}

// Base a < 2^32: a^d by fixed 3-bit windows over the lane's table of
// a^0 .. a^7 in LDS (rows of tbl[8][stride], column col).
__device__ __forceinline__ bool sprp_lane(const LaneMr &m, uint64_t r2, uint32_t a, uint64_t *tbl,
                                          unsigned col, unsigned stride)
{
    const uint64_t n = m.c.n, ninv = m.c.ninv;
    const uint64_t am = to_mont(a, r2, m.c);
    uint64_t p = m.c.one;
    tbl[col] = p;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        p = k == 1 ? am : montmul(p, am, n, ninv);
        tbl[k * stride + col] = p;
    }
    int pos = 3 * (m.top / 3);  // windows cover bits top .. 0
    uint64_t x = tbl[((unsigned)(m.d >> pos) & 7u) * stride + col];
    for (pos -= 3; pos >= 0; pos -= 3) {
        x = montsqr(x, n, ninv);
        x = montsqr(x, n, ninv);
        x = montsqr(x, n, ninv);
        x = montmul(x, tbl[((unsigned)(m.d >> pos) & 7u) * stride + col], n, ninv);
    }
    return strong_tail(x, m);
}

}  // namespace isp
