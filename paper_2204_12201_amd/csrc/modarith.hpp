// Modular arithmetic on 64-bit residues for gfx950 (and the host, for tables).
//
// All primes are below 2^61, so lazy values up to 8q fit a 64-bit word.
//  * Shoup multiplication by a constant w (Harvey, "Faster arithmetic for
//    number-theoretic transforms", 2014): with w' = floor(w 2^64 / q),
//    a w - floor(a w' / 2^64) q lies in [0, 2q) for every a < 2^64.  The
//    transforms use a cheaper quotient estimate that is low by at most 2,
//    leaving the remainder in [0, 4q) (mul_shoup_lazy4).
//  * Montgomery multiplication (R = 2^64): REDC(T) = T 2^-64 mod q in [0, 2q)
//    for T < q 2^64, with qinv_neg = -q^-1 mod 2^64.
// The 64 x 64 -> 128-bit products lower to v_mad_u64_u32 / v_mul_hi_u32
// sequences on the 32-bit VALU.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define FHE_HD __host__ __device__ __forceinline__
#else
#define FHE_HD inline
#endif

typedef unsigned __int128 u128;

// Full 64 x 64 -> 128-bit product from four 32 x 32 -> 64-bit multiply-adds
// (each one v_mad_u64_u32 on the device; no partial sum overflows 64 bits).
FHE_HD void mul128(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t p01 = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t p10 = (uint64_t)a1 * b0 + (uint32_t)p01;
    hi = (uint64_t)a1 * b1 + (p01 >> 32) + (p10 >> 32);
    lo = (uint32_t)p00 | (p10 << 32);
}

FHE_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
    uint64_t lo, hi;
    mul128(a, b, lo, hi);
    return hi;
}

// a * w mod q in [0, 2q), any a < 2^64; wp = floor(w * 2^64 / q), w < q.
FHE_HD uint64_t mul_shoup_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t qh = mulhi64(a, wp);
    return a * w - qh * q;
}

// 32 x 32 -> upper 32 bits of the product (v_mul_hi_u32 on the device).
FHE_HD uint32_t mulhi32(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }

// a * w mod q in [0, 4q) for any a < 2^64, w < q, wp = floor(w 2^64 / q).
// floor(a wp / 2^64) = a1 wp1 + floor((a1 wp0 + a0 wp1 + floor(a0 wp0 / 2^32)) / 2^32)
// (32-bit halves); keeping a1 wp1 and the upper halves of the two cross
// products drops three terms below 2^32 each, so the estimate h is low by at
// most 2 and a w - h q (exact modulo 2^64, as it is below 2^64) by at most 2q
// above the [0, 2q) of the exact quotient.  Three 32-bit multiplies for the
// estimate instead of four, and no carry propagation.
FHE_HD uint64_t mul_shoup_lazy4(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t p0 = (uint32_t)wp, p1 = (uint32_t)(wp >> 32);
    uint64_t h = (uint64_t)a1 * p1 + mulhi32(a1, p0);
    h += mulhi32(a0, p1);
    return a * w - h * q;
}

// The same value with nq = 2^64 - q: a w - h q = a w + h nq modulo 2^64.  A
// caller that hides nq from the compiler gets a sum of two products, which
// the device builds from multiply-adds without a borrow chain.
FHE_HD uint64_t mul_shoup_lazy4n(uint64_t a, uint64_t w, uint64_t wp, uint64_t nq) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t p0 = (uint32_t)wp, p1 = (uint32_t)(wp >> 32);
    uint64_t h = (uint64_t)a1 * p1 + mulhi32(a1, p0);
    h += mulhi32(a0, p1);
    return a * w + h * nq;
}

FHE_HD uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

FHE_HD uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    return csub(mul_shoup_lazy(a, w, wp, q), q);
}

// REDC(hi:lo) for hi:lo < q 2^64: returns (hi:lo) 2^-64 mod q in [0, 2q).
FHE_HD uint64_t redc_lazy(uint64_t hi, uint64_t lo, uint64_t q, uint64_t qinv_neg) {
    uint64_t m = lo * qinv_neg;
    uint64_t mh = mulhi64(m, q);
    return hi + mh + (lo != 0 ? 1u : 0u);
}

// a b 2^-64 mod q in [0, 2q) for a b < q 2^64 (e.g. a < 4q, b < q, q < 2^62).
FHE_HD uint64_t mont_mul_lazy(uint64_t a, uint64_t b, uint64_t q, uint64_t qinv_neg) {
    uint64_t lo, hi;
    mul128(a, b, lo, hi);
    return redc_lazy(hi, lo, q, qinv_neg);
}

FHE_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {  // a, b < q
    uint64_t s = a + b;
    return csub(s, q);
}

FHE_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) {  // a, b < q
    return a >= b ? a - b : a + q - b;
}

// 128-bit accumulator helpers.
struct Acc128 {
    uint64_t lo, hi;
};

FHE_HD void acc_init(Acc128 &a) { a.lo = 0; a.hi = 0; }

FHE_HD void acc_mac(Acc128 &a, uint64_t x, uint64_t y) {
    uint64_t lo, hi;
    mul128(x, y, lo, hi);
    a.lo += lo;
    a.hi += hi + (a.lo < lo ? 1u : 0u);
}

#if defined(__HIPCC__)
// Sum of 64 x 64-bit products kept as three 64-bit partial sums (of the
// products of 32-bit halves lo*lo, lo*hi + hi*lo, hi*hi) plus carry counts of
// the first two, so that a term costs four v_mad_u64_u32 and three
// carry additions and nothing is propagated until the end:
//   sum = lo + mid 2^32 + (hi + clo) 2^64 + cmid 2^96.
// The carry-out of each multiply-add (an SGPR lane mask) is added into the
// counts with v_addc; every such read comes at least two instructions after
// the write that produced it.
struct Acc3 {
    uint64_t lo, mid, hi;
    uint32_t clo, cmid;
};

__device__ __forceinline__ void acc3_init(Acc3 &A) {
    A.lo = 0;
    A.mid = 0;
    A.hi = 0;
    A.clo = 0;
    A.cmid = 0;
}

// A += a b for a < 2^64 (vector) and b < 2^64 (wave-uniform).
__device__ __forceinline__ void acc3_mac(Acc3 &A, uint64_t a, uint64_t b) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    uint64_t c1, c2, c3, c4;
    asm("v_mad_u64_u32 %[lo], %[c1], %[a0], %[b0], %[lo]\n\t"
        "v_mad_u64_u32 %[mid], %[c2], %[a0], %[b1], %[mid]\n\t"
        "v_mad_u64_u32 %[hi], %[c4], %[a1], %[b1], %[hi]\n\t"
        "v_addc_co_u32_e64 %[clo], %[c1], 0, %[clo], %[c1]\n\t"
        "v_mad_u64_u32 %[mid], %[c3], %[a1], %[b0], %[mid]\n\t"
        "v_addc_co_u32_e64 %[cmid], %[c2], 0, %[cmid], %[c2]\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32_e64 %[cmid], %[c3], 0, %[cmid], %[c3]"
        : [lo] "+v"(A.lo), [mid] "+v"(A.mid), [hi] "+v"(A.hi), [clo] "+v"(A.clo), [cmid] "+v"(A.cmid),
          [c1] "=&s"(c1), [c2] "=&s"(c2), [c3] "=&s"(c3), [c4] "=&s"(c4)
        : [a0] "v"(a0), [a1] "v"(a1), [b0] "s"(b0), [b1] "s"(b1));
}

// a b 2^-64 mod q in [0, 2q) (the value of mont_mul_lazy) for a wave-uniform
// q, when a b < q 2^64 and hi(a) + hi(b) + hi(q) < 2^32 (32-bit halves).  The
// product T = a b and m q (m = T (-q^-1) mod 2^64) are summed by columns of
// 32-bit halves with multiply-adds whose 64-bit addends are the previous
// partial sums: L = lo(a) lo(b) + m0 q0 (carry cL), Mid = lo(a) hi(b) +
// hi(a) lo(b) + m0 hi(q) + m1 lo(q) (below 2^64 until the last term, whose
// carry is cM; the bound on the high halves keeps the first three below
// 2^64) and H = hi(a) hi(b) + m1 hi(q).  T + m q vanishes modulo 2^64, so its
// bits 32..63 are zero: lo(Mid) + hi(L) is 0 or 2^32, the latter exactly when
// lo(Mid) is nonzero, and (T + m q) / 2^64 = H + hi(Mid) + cL + [lo(Mid) != 0]
// + cM 2^32.  No partial product is zero-extended into a 64-bit addend, which
// would cost register moves.  The carry masks written by the multiply-adds
// are read as carry-ins only two or more instructions later.
__device__ __forceinline__ uint64_t mont_mul_lazy_u(uint64_t a, uint64_t b, uint64_t q, uint64_t qinv_neg) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
    const uint32_t qi0 = (uint32_t)qinv_neg, qi1 = (uint32_t)(qinv_neg >> 32);
    uint64_t P00, Mid, P11, j0;
    asm("v_mad_u64_u32 %[p00], %[j], %[a0], %[b0], 0\n\t"
        "v_mad_u64_u32 %[mid], %[j], %[a0], %[b1], 0\n\t"
        "v_mad_u64_u32 %[p11], %[j], %[a1], %[b1], 0\n\t"
        "v_mad_u64_u32 %[mid], %[j], %[a1], %[b0], %[mid]"
        : [p00] "=&v"(P00), [mid] "=&v"(Mid), [p11] "=&v"(P11), [j] "=&s"(j0)
        : [a0] "v"(a0), [a1] "v"(a1), [b0] "v"(b0), [b1] "v"(b1));
    // m = lo(T) (-q^-1) mod 2^64, lo(T) = (lo P00, hi P00 + lo Mid)
    const uint32_t t0 = (uint32_t)P00, t1 = (uint32_t)(P00 >> 32) + (uint32_t)Mid;
    const uint64_t M = (uint64_t)t0 * qi0;
    const uint32_t m0 = (uint32_t)M, m1 = (uint32_t)(M >> 32) + t0 * qi1 + t1 * qi0;
    uint64_t L, H, cL, cM, j1;
    asm("v_mad_u64_u32 %[l], %[cl], %[m0], %[q0], %[p00]\n\t"
        "v_mad_u64_u32 %[mid], %[j], %[m0], %[q1], %[mid]\n\t"
        "v_mad_u64_u32 %[h], %[j], %[m1], %[q1], %[p11]\n\t"
        "v_mad_u64_u32 %[mid], %[cm], %[m1], %[q0], %[mid]"
        : [l] "=&v"(L), [h] "=&v"(H), [mid] "+v"(Mid), [cl] "=&s"(cL), [cm] "=&s"(cM), [j] "=&s"(j1)
        : [m0] "v"(m0), [m1] "v"(m1), [q0] "s"(q0), [q1] "s"(q1), [p00] "v"(P00), [p11] "v"(P11));
    (void)L;
    const uint32_t h0 = (uint32_t)H, h1 = (uint32_t)(H >> 32), ml = (uint32_t)Mid, mh = (uint32_t)(Mid >> 32);
    uint32_t r0, r1;
    uint64_t e1, e2, e3, nz;
    asm("v_add_co_u32_e64 %[r0], %[e1], %[h0], %[mh]\n\t"
        "v_cmp_ne_u32_e64 %[nz], 0, %[ml]\n\t"
        "v_addc_co_u32_e64 %[r0], %[e2], %[r0], 0, %[cl]\n\t"
        "v_addc_co_u32_e64 %[r1], %[e1], %[h1], 0, %[e1]\n\t"
        "v_addc_co_u32_e64 %[r0], %[e3], %[r0], 0, %[nz]\n\t"
        "v_addc_co_u32_e64 %[r1], %[e2], %[r1], 0, %[e2]\n\t"
        "v_addc_co_u32_e64 %[r1], %[e1], %[r1], 0, %[cm]\n\t"
        "v_addc_co_u32_e64 %[r1], %[e1], %[r1], 0, %[e3]"
        : [r0] "=&v"(r0), [r1] "=&v"(r1), [e1] "=&s"(e1), [e2] "=&s"(e2), [e3] "=&s"(e3), [nz] "=&s"(nz)
        : [h0] "v"(h0), [h1] "v"(h1), [ml] "v"(ml), [mh] "v"(mh), [cl] "s"(cL), [cm] "s"(cM));
    return ((uint64_t)r1 << 32) | r0;
}

// A += c for a constant c < 2^64.
__device__ __forceinline__ void acc3_add(Acc3 &A, uint64_t c) {
    const uint64_t s = A.lo + c;
    A.clo += s < c ? 1u : 0u;
    A.lo = s;
}

// The 128-bit value of A (its sums of products stay below 2^127).
__device__ __forceinline__ Acc128 acc3_value(const Acc3 &A) {
    const uint64_t m = A.mid << 32;
    Acc128 r;
    r.lo = A.lo + m;
    r.hi = A.hi + (A.mid >> 32) + A.clo + ((uint64_t)A.cmid << 32) + (r.lo < m ? 1u : 0u);
    return r;
}
#endif

// (acc) 2^-64 mod q in [0, q) when acc.hi <= 2q - 2: REDC gives hi + mulhi(m, q)
// + [lo != 0] < hi + q + 1 <= 3q - 1, then two conditional subtractions.
FHE_HD uint64_t acc_reduce_mont_small(const Acc128 &a, uint64_t q, uint64_t qinv_neg) {
    uint64_t r = redc_lazy(a.hi, a.lo, q, qinv_neg);
    r = csub(r, q << 1);
    return csub(r, q);
}

// (acc) 2^-64 mod q in [0, q) for any 128-bit acc: the high word is first
// reduced below 2q by a Shoup multiplication by 1 (one_p = floor(2^64 / q)),
// which keeps the REDC input below 2q 2^64; REDC then lands in [0, 3q).
FHE_HD uint64_t acc_reduce_mont(const Acc128 &a, uint64_t q, uint64_t qinv_neg, uint64_t one_p) {
    uint64_t h = mul_shoup_lazy(a.hi, 1, one_p, q);  // [0, 2q)
    uint64_t r = redc_lazy(h, a.lo, q, qinv_neg);    // < (2q 2^64 + q 2^64) / 2^64 = 3q
    r = csub(r, q << 1);
    return csub(r, q);
}
