// mont.h -- 64-bit Montgomery arithmetic for one odd modulus per lane.
//
// The paper (sections 2.2-2.4) keeps every intermediate of a^b mod m below
// 2^64 with ModAdd and a double-and-add ModMultiply, because MATLAB has no
// 128-bit products.  A gfx950 lane has 32x32->64 multiply-adds, so the
// product a*b is formed exactly in 128 bits and reduced with Montgomery's
// REDC (P. L. Montgomery, "Modular multiplication without trial division",
// Math. Comp. 44, 1985) in the subtractive form:
//
//     T = a*b,  m = (T mod 2^64) * n^-1 mod 2^64,  t = floor(T/2^64) - floor(m*n/2^64)
//
// Because m*n = T (mod 2^64), the low halves cancel exactly and t lies in
// (-n, n); one conditional add of n gives T * 2^-64 mod n.  This needs no
// carry out of a 64-bit add, so it is valid for every odd n < 2^64,
// including n > 2^63 where the additive form overflows.  Requires a*b < n*2^64
// (true whenever a < n).
//
// The only additions are the modular doublings of section 2.2's ModAdd
// (c = a - (m - b) when a + b >= m): here x + x with the carry kept.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isp {

// n^-1 mod 2^64 for odd n by Newton-Hensel lifting x <- x (2 - n x); the seed
// (3n) xor 2 is correct to 5 bits, and each step doubles the correct bits.
__device__ __forceinline__ uint64_t inv64(uint64_t n)
{
    uint64_t x = (3 * n) ^ 2;  // 5 bits
    x *= 2 - n * x;            // 10
    x *= 2 - n * x;            // 20
    x *= 2 - n * x;            // 40
    x *= 2 - n * x;            // 80
    return x;
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b)
{
    return __umul64hi(a, b);
}

// a * b * 2^-64 mod n, for a*b < n*2^64.
__device__ __forceinline__ uint64_t montmul(uint64_t a, uint64_t b, uint64_t n, uint64_t ninv)
{
    unsigned __int128 T = (unsigned __int128)a * b;
    uint64_t lo = (uint64_t)T, hi = (uint64_t)(T >> 64);
    uint64_t m = lo * ninv;
    uint64_t mh = mulhi64(m, n);
    uint64_t t = hi - mh;
    return hi < mh ? t + n : t;
}

__device__ __forceinline__ uint64_t montsqr(uint64_t a, uint64_t n, uint64_t ninv)
{
    return montmul(a, a, n, ninv);
}

// 2x mod n for x < n (ModAdd of x and x: the carry out of x + x is kept).
__device__ __forceinline__ uint64_t dbl_mod(uint64_t x, uint64_t n)
{
    uint64_t y = x + x;
    bool carry = y < x;
    return (carry || y >= n) ? y - n : y;
}

// Per-lane Montgomery context for an odd modulus n >= 3 with bit length L.
struct MontCtx {
    uint64_t n, ninv;
    uint64_t one;   // 2^64 mod n  (1 in Montgomery form)
    uint64_t mone;  // n - one     (-1 in Montgomery form)
};

// 2^64 mod n: start from 2^(L-1) < n (n odd, so n != 2^(L-1)) and double
// 65 - L times.  For L >= 33 that is at most 32 doublings and no division.
__device__ __forceinline__ uint64_t r_mod_n(uint64_t n, int L)
{
    uint64_t x = (uint64_t)1 << (L - 1);
    for (int k = L - 1; k < 64; ++k)
        x = dbl_mod(x, n);
    return x;
}

__device__ __forceinline__ MontCtx make_ctx(uint64_t n, int L)
{
    MontCtx c;
    c.n = n;
    c.ninv = inv64(n);
    c.one = r_mod_n(n, L);
    c.mone = n - c.one;
    return c;
}

// Montgomery form of a small value v (v < 2^32 <= n) from R^2 mod n:
// montmul(v, R^2) = v * R mod n.
__device__ __forceinline__ uint64_t to_mont(uint64_t v, uint64_t r2, const MontCtx &c)
{
    return montmul(v, r2, c.n, c.ninv);
}

// R^2 mod n from one = R mod n: 2R = dbl(one), then six squarings give
// (2^(2^6)) R = 2^64 R = R^2 mod n.
__device__ __forceinline__ uint64_t r2_mod_n(const MontCtx &c)
{
    uint64_t x = dbl_mod(c.one, c.n);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        x = montsqr(x, c.n, c.ninv);
    return x;
}

}  // namespace isp
