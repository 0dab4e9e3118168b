// dk_rng.h -- device-side noise generator for gfx950.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 products
// of words 0 and 2 with the round multipliers, whose high halves are XORed with words 1, 3
// and the round key; the key advances by the two Weyl increments between rounds.
//
// Gaussian transform (Box & Muller 1958) as a fixed sequence of correctly rounded binary32
// operations, so its bits are reproducible on any IEEE-754 machine that performs the same
// sequence (no contraction inside; every fused multiply-add is written explicitly):
//   radius word a -> odd integer w = 2 (a >> 9) + 1, u = w 2^-24;
//     w = 2^e m, m in [1, 2), folded into [sqrt(1/2), sqrt(2)];
//     ln u = (e - 24) ln 2 + x g(x), x = m - 1 (exact), g(x) = ln(1 + x)/x by the degree-10
//     polynomial interpolating g at the 11 Chebyshev nodes of [sqrt(1/2) - 1, sqrt(2) - 1]
//     (coefficients rounded to binary32; error below the rounding of the result; no division);
//     R = sqrt(-2 ln u)   (|R| <= sqrt(48 ln 2), a tail cut at probability ~1e-8)
//   angle word b -> quadrant b >> 30 and fraction f = (2 ((b >> 7) & 0x7fffff) + 1) 2^-24;
//     the angle inside the quadrant is reduced to at most pi/4 by the complement, and its
//     sine and cosine come from their Taylor series to degree 9 and 10 (next terms < 2e-9);
//   (z0, z1) = R (cos, sin)(pi/2 (q + f)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dk {

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;   // the three-way XORs are single gfx950 bitop3 instructions (truth table 0x96)
        n.x = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96);
        n.y = (uint32_t)p1;
        n.z = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96);
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Correctly rounded square root of a positive normal binary32 x.  The hardware estimate s is
// within one ulp of sqrt(x), so the rounded root is s or a neighbour s-, s+ of it.  sqrt(x) lies
// below the midpoint of two adjacent floats c < c+ exactly when x <= c c+: x - c c+ is a whole
// multiple of ulp(c)^2, while the squared midpoint exceeds c c+ by ulp(c)^2 / 4, so no float x
// lies in between; and a single-rounding fma gives the sign of x - c c+ exactly.  Hence the
// result is s- if fma(-s-, s, x) <= 0, s+ if fma(-s+, s, x) > 0, and s otherwise.  The radius
// argument -2 ln u lies in [1.1e-7, 33.3], so the scaling of subnormal inputs and the zero and
// infinity cases of a general square root are not needed.
__device__ __forceinline__ float sqrt_rn_normal(float x)
{
    const float s = __builtin_amdgcn_sqrtf(x);
    const float sm = __uint_as_float(__float_as_uint(s) - 1u);
    const float sp = __uint_as_float(__float_as_uint(s) + 1u);
    const float rm = __builtin_fmaf(-sm, s, x);
    const float rp = __builtin_fmaf(-sp, s, x);
    const float r = rm <= 0.0f ? sm : s;
    return rp > 0.0f ? sp : r;
}

// The sequence below is that definition written with integer bit operations where the
// definition selects or negates (the same values, bit for bit, without lane-mask hazards):
//   the fold:  m > binary32(1.41421356) = 0x1.6a09e6p+0 iff the frexp significand of (float)w,
//              which is half of m, exceeds 0x1.6a09e6p-1 (its significand field exceeds 0x3504f3);
//   the complement angle:  1 - f = (2 (j ^ 0x7fffff) + 1) 2^-24 exactly, and f > 1/2 iff bit 22 of j;
//   the quadrant turn:  (c, s) -> (-s, c) twice folds into one swap and two sign-bit flips.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1)
{
#pragma clang fp contract(off)
    const uint32_t w = ((a >> 9) << 1) | 1u;                 // odd, < 2^24, so (float)w is exact
    // w = 2^e m1 with m1 in [1, 2) is m0 2^(e + 1) with m0 = m1 / 2 (frexp); the fold (m1 above
    // binary32(1.41421356), i.e. m0 above half of it) takes m = m0, else m = m1 = 2 m0, and
    // x = m - 1 is exact either way
    const float wf = (float)w;
    const float m0 = __builtin_amdgcn_frexp_mantf(wf);
    const int fold = m0 > 0x1.6a09e6p-1f ? 1 : 0;
    const float ne = (float)(__builtin_amdgcn_frexp_expf(wf) - 25 + fold);   // e - 24 of the folded m
    const float xm = __builtin_fmaf(m0, fold ? 1.0f : 2.0f, -1.0f);        // m - 1, exact
    // -2 ln u, evaluated as -2 (hi + lo) of the definition: every coefficient and constant below
    // carries the factor -2, which is exact (a power of two, no underflow or overflow in this
    // range), so each rounded step yields exactly -2 times the defined step and the sum is
    // exactly -2 (hi + lo), without a multiplication of its own.
    float gx = __builtin_fmaf(-0x1.0d33dap-3f, xm, 0x1.dbfb56p-3f);
    gx = __builtin_fmaf(gx, xm, -0x1.e94d9cp-3f);
    gx = __builtin_fmaf(gx, xm, 0x1.fcc1c0p-3f);
    gx = __builtin_fmaf(gx, xm, -0x1.231156p-2f);
    gx = __builtin_fmaf(gx, xm, 0x1.5554c0p-2f);
    gx = __builtin_fmaf(gx, xm, -0x1.99a6e4p-2f);
    gx = __builtin_fmaf(gx, xm, 0x1.00002ap-1f);
    gx = __builtin_fmaf(gx, xm, -0x1.555540p-1f);
    gx = __builtin_fmaf(gx, xm, 1.0f);
    gx = __builtin_fmaf(gx, xm, -2.0f);
    const float lnm = xm * gx;                                          // -2 x g(x)
    const float hi = ne * -0x1.62ep+0f;                                 // -2 (e - 24) ln2_hi
    const float lo = __builtin_fmaf(ne, -2.0f * (float)(0.69314718055994530942 - 0.693115234375), lnm);
    const float R = sqrt_rn_normal(hi + lo);                            // correctly rounded

    // quadrant q = b >> 30
    const uint32_t flip = (b >> 29) & 1u;                    // f > 1/2
    const uint32_t j = ((b >> 7) & 0x7FFFFFu) ^ ((0u - flip) & 0x7FFFFFu);
    // x = binary32(pi/2) g with g = f or 1 - f (when f > 1/2) = (2 j + 1) 2^-24.  The scaling by
    // 2^-24 is exact, and fma(j, 2 C, C) with C = binary32(pi/2) 2^-24 rounds the same real
    // number (2 j + 1) C once, so x is the defined product.
    constexpr float C = 0x1.921fb6p+0f * 0x1p-24f;
    const float x = __builtin_fmaf((float)j, 2.0f * C, C);
    const float x2 = x * x;
    float ps = __builtin_fmaf(1.0f / 362880.0f, x2, -1.0f / 5040.0f);
    ps = __builtin_fmaf(ps, x2, 1.0f / 120.0f);
    ps = __builtin_fmaf(ps, x2, -1.0f / 6.0f);
    const float sn = __builtin_fmaf(x * x2, ps, x);
    float pc = __builtin_fmaf(-1.0f / 3628800.0f, x2, 1.0f / 40320.0f);
    pc = __builtin_fmaf(pc, x2, -1.0f / 720.0f);
    pc = __builtin_fmaf(pc, x2, 1.0f / 24.0f);
    pc = __builtin_fmaf(pc, x2, -0.5f);
    const float cs = __builtin_fmaf(x2, pc, 1.0f);
    // cos and sin of the quadrant's angle; each odd quarter turn swaps them, and the signs of
    // cos and sin flip in quadrants (1, 2) and (2, 3).  With t = b ^ (b << 1): bit 30 of t is
    // flip ^ (q & 1), the swap, and bit 31 of t is the parity of q's two bits, the cosine's sign;
    // the sine's sign is q's high bit, bit 31 of b.
    const uint32_t t = b ^ (b << 1);
    const uint32_t swap = (uint32_t)((int32_t)(t << 1) >> 31);      // all ones iff bit 30 of t
    const uint32_t sb = __float_as_uint(sn), cb = __float_as_uint(cs);
    const uint32_t c = __builtin_amdgcn_bitop3_b32(swap, sb, cb, 0xCA);  // swap ? sn : cs, bitwise
    const uint32_t s = __builtin_amdgcn_bitop3_b32(swap, cb, sb, 0xCA);  // swap ? cs : sn
    z0 = R * __uint_as_float(c ^ (t & 0x80000000u));
    z1 = R * __uint_as_float(s ^ (b & 0x80000000u));
}

// Normals of the horizontal site pair (2a, y), (2a+1, y) at fine step m.
struct NoiseKey {
    uint32_t k0, k1;     // seed
    uint32_t c2, c3;     // sample bits and tag|level|sample_hi
};

__device__ __forceinline__ NoiseKey make_key(uint64_t seed, uint32_t tag, int level, uint64_t sample)
{
    NoiseKey k;
    k.k0 = (uint32_t)seed;
    k.k1 = (uint32_t)(seed >> 32);
    k.c2 = (uint32_t)sample;
    k.c3 = (tag << 24) | ((uint32_t)level << 16) | (uint32_t)((sample >> 32) & 0xFFFFu);
    return k;
}

__device__ __forceinline__ void site_pair_normals(const NoiseKey& k, uint32_t pair_index, uint32_t step,
                                                  float& a0, float& a1, float& b0, float& b1)
{
    const U4 o = philox10(U4{pair_index, step, k.c2, k.c3}, k.k0, k.k1);
    box_muller(o.x, o.y, a0, a1);
    box_muller(o.z, o.w, b0, b1);
}

}  // namespace dk
