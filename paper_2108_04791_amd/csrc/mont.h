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

// n^-1 mod 2^64 for odd n by Newton-Hensel lifting x <- x (2 - n x): the
// seed (3n) xor 2 is correct to 5 bits and each step doubles the correct
// bits.  The first three steps (to 10, 20, 40 bits) need only n mod 2^32 and
// run on 32-bit words; one 64-bit step finishes.
__device__ __forceinline__ uint64_t inv64(uint64_t n)
{
    const uint32_t n0 = (uint32_t)n;
    uint32_t y = (3u * n0) ^ 2u;  // 5 bits
    y *= 2u - n0 * y;             // 10
    y *= 2u - n0 * y;             // 20
    y *= 2u - n0 * y;             // 40 >= 32
    const uint64_t x = y;
    return x * (2 - n * x);       // 64
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b)
{
    return __umul64hi(a, b);
}

__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint64_t pair32(uint32_t lo, uint32_t hi)
{
    return ((uint64_t)hi << 32) | lo;
}

// a*b + c for 32-bit a, b and 64-bit c, as one v_mad_u64_u32, with the
// carry out of the 64-bit sum returned as 0 or 1 (the instruction's own
// carry-out lane mask, turned into a value by v_cndmask).  A VALU write of
// an SGPR followed by a VALU read of it needs two wait states on this
// target, hence the s_nop.  Pure register arithmetic.
__device__ __forceinline__ uint64_t mad_carry(uint32_t a, uint32_t b, uint64_t c, uint32_t &k)
{
    uint64_t r, cc;
    asm("v_mad_u64_u32 %0, %1, %3, %4, %5\n\t"
        "s_nop 1\n\t"
        "v_cndmask_b32_e64 %2, 0, 1, %1"
        : "=v"(r), "=&s"(cc), "=v"(k)
        : "v"(a), "v"(b), "v"(c));
    return r;
}

// h = floor(m n / 2^64) for m = (t1 2^32 + t0) * n^-1 mod 2^64, the REDC
// correction of a product whose low word is t1:t0.  m = T ninv mod 2^64
// needs only the low product and two low-half cross products; floor(m n /
// 2^64) is assembled from m0 n0, m1 n0, m0 n1 (with its carry) and m1 n1.
__device__ __forceinline__ uint64_t redc_h(uint32_t t0, uint32_t t1, uint64_t n, uint64_t ninv)
{
    const uint32_t n0 = lo32(n), n1 = hi32(n), i0 = lo32(ninv), i1 = hi32(ninv);
    const uint64_t X = (uint64_t)t0 * i0;
    const uint32_t m0 = lo32(X);
    const uint32_t m1 = hi32(X) + t0 * i1 + t1 * i0;
    const uint64_t Z = (uint64_t)m1 * n0 + __umulhi(m0, n0);
    uint32_t k2;
    const uint64_t Z2 = mad_carry(m0, n1, Z, k2);
    return (uint64_t)m1 * n1 + pair32(hi32(Z2), k2);
}

// T = a*b (as hi:lo) and h = floor(m n / 2^64) with m = lo * n^-1 mod 2^64,
// on 32-bit halves (x = x1 2^32 + x0).
//
// T = a*b: with c = floor(a0 b0 / 2^32), M1 = a1 b0 + c < 2^64 and
// M2 = a0 b1 + M1 < 2^65 (carry k), T = (a1 b1 + floor(M2 / 2^32) + k 2^32) 2^64
// + (M2 mod 2^32) 2^32 + (a0 b0 mod 2^32).  Every 32x32+64 step is one
// v_mad_u64_u32: 17 VALU instructions with redc_h.
__device__ __forceinline__ void redc_parts(uint64_t a, uint64_t b, uint64_t n, uint64_t ninv,
                                           uint64_t &hi, uint64_t &h)
{
    const uint32_t a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
    const uint32_t t0 = a0 * b0;
    const uint64_t M1 = (uint64_t)a1 * b0 + __umulhi(a0, b0);
    uint32_t k;
    const uint64_t M2 = mad_carry(a0, b1, M1, k);
    hi = (uint64_t)a1 * b1 + pair32(hi32(M2), k);
    h = redc_h(t0, lo32(M2), n, ninv);
}

// The same for a*a with a < 2^63: a1 < 2^31, so the doubled cross term
// 2 a0 a1 is the single product a0 (2 a1), and M = a0 (2 a1) + floor(a0^2 /
// 2^32) <= (2^32 - 1)(2^32 - 2) + 2^32 - 2 = 2^64 - 2^33 needs no carry:
// a^2 = (a1^2 + floor(M / 2^32)) 2^64 + (M mod 2^32) 2^32 + (a0^2 mod 2^32).
// One instruction fewer than redc_parts, and no carry-out.
__device__ __forceinline__ void redc_sqr_parts(uint64_t a, uint64_t n, uint64_t ninv,
                                               uint64_t &hi, uint64_t &h)
{
    const uint32_t a0 = lo32(a), a1 = hi32(a);
    const uint32_t t0 = a0 * a0;
    // 2 a1 as one shift of the high half (left to itself the compiler forms
    // it from the 64-bit value with two instructions)
    uint32_t a1x2;
    asm("v_lshlrev_b32 %0, 1, %1" : "=v"(a1x2) : "v"(a1));
    const uint64_t M = (uint64_t)a0 * a1x2 + __umulhi(a0, a0);
    hi = (uint64_t)a1 * a1 + hi32(M);
    h = redc_h(t0, lo32(M), n, ninv);
}

// a * b * 2^-64 mod n, for a*b < n*2^64.  Because m n = T (mod 2^64), the low
// halves cancel exactly and hi - h lies in (-n, n); one conditional add of n
// reduces it: 22 VALU instructions plus one compare that the compiler adds
// for the final select.
__device__ __forceinline__ uint64_t montmul(uint64_t a, uint64_t b, uint64_t n, uint64_t ninv)
{
    uint64_t hi, h;
    redc_parts(a, b, n, ninv, hi, h);
    const uint64_t t = hi - h;
    return hi < h ? t + n : t;
}

// The same product for n < 2^62 and a, b < 2n, returned in (0, 2n) without
// the final select: a*b < 4 n^2 < n 2^64, so hi < n and (hi + n) - h lies in
// (0, 2n) with no overflow.  20 VALU instructions.
__device__ __forceinline__ uint64_t montmul_lazy(uint64_t a, uint64_t b, uint64_t n,
                                                 uint64_t ninv)
{
    uint64_t hi, h;
    redc_parts(a, b, n, ninv, hi, h);
    return (hi + n) - h;
}

__device__ __forceinline__ uint64_t montsqr(uint64_t a, uint64_t n, uint64_t ninv)
{
    return montmul(a, a, n, ninv);
}

// a * a * 2^-64 mod n for a < 2^63 and a*a < n*2^64 (a < n, or a < 2n with
// n < 2^62), reduced.
__device__ __forceinline__ uint64_t montsqr63(uint64_t a, uint64_t n, uint64_t ninv)
{
    uint64_t hi, h;
    redc_sqr_parts(a, n, ninv, hi, h);
    const uint64_t t = hi - h;
    return hi < h ? t + n : t;
}

// The square in (0, 2n) like montmul_lazy, for a < 2^63 with a*a < n 2^64
// (so that hi < n): a < 2n with n < 2^62, or a < 4n with n < 2^60.
__device__ __forceinline__ uint64_t montsqr63_lazy(uint64_t a, uint64_t n, uint64_t ninv)
{
    uint64_t hi, h;
    redc_sqr_parts(a, n, ninv, hi, h);
    return (hi + n) - h;
}

// (x << b) + a modulo 2^64 for a per-lane shift b in {0, 1}, as the single
// gfx950 instruction v_lshl_add_u64 (its shift operand takes 0 to 4).  Pure
// VALU arithmetic, no memory access.
__device__ __forceinline__ uint64_t shl_add(uint64_t x, uint32_t b, uint64_t a)
{
    uint64_t r;
    asm("v_lshl_add_u64 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(b), "v"(a));
    return r;
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

// 2^64 mod n for odd n >= 2^32 in a fixed number of instructions.  For n >=
// 2^63 it is 2^64 - n.  Below, the quotient q = floor(2^64 / n) < 2^32 comes
// from a double-precision estimate: n rounded to 53 bits, its reciprocal
// from the hardware estimate refined by two Newton steps, and 2^64 times it
// (an exact scaling) are within 2^-18 of 2^64 / n, so floor(2^64 (1/n) -
// 1/2) is q or q - 1, and r = 2^64 - q n, formed modulo 2^64, lies in [0,
// 2n) with 2n < 2^64: one conditional subtraction ends it.
__device__ __forceinline__ uint64_t r_mod_n_wide(uint64_t n)
{
    const double d = (double)n;
    double inv = __builtin_amdgcn_rcp(d);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    const uint32_t q = (uint32_t)floor(fma(0x1p64, inv, -0.5));
    uint64_t r = 0 - (uint64_t)q * n;
    r = r >= n ? r - n : r;
    return (int64_t)n < 0 ? 0 - n : r;
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
