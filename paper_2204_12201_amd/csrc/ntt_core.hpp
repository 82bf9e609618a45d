// Negacyclic NTT core for gfx950: one workgroup per row of n = 2^L residues.
//
// Transform: forward Cooley-Tukey with the psi twist merged into the twiddles
// (twiddle table entry i holds psi^bitrev(i)), inverse Gentleman-Sande with
// psi^-bitrev(i).  The forward output position bitrev(j) receives
// sum_i a_i psi^(i(2j+1)); the inverse undoes it up to the factor n, which the
// caller folds into a final scaling.
//
// Work decomposition: T = n/E threads, each holding E = 2^LE residues in
// registers (E = 16 or 32).  The L butterfly levels are split into passes of
// LE levels (radix E) plus one shorter pass when LE does not divide L.  In pass p
// a thread owns groups of R = 2^r elements that differ only in the pass's r
// index bits; between passes the row is exchanged through LDS, stored at
// position idx + idx/16 (the padding keeps 16 consecutive lanes on distinct
// bank pairs for every pass's access pattern).  Pass 0 reads the natural
// order with lanes on consecutive addresses; the last pass leaves each lane
// with runs of R consecutive positions of the bit-reversed output.  Only the
// exchange next to pass 0 crosses waves (fixed_bits below): the others are
// wave-local, so waves run the later passes without workgroup barriers.
//
// Butterflies are Harvey's lazy ones with the quotient estimate of
// mul_shoup_lazy4 (twiddle products in [0, 4q)): forward values live in
// [0, 8q), inverse values in [0, 4q), so primes must stay below 2^61.  For
// primes below 2^64 / (4 (L + 1)) the forward transform can also drop the
// conditional subtraction (REDUCE = false): a stage then raises the bound by at
// most 4q, and a row entering below 4q leaves below 4 (L + 1) q.  For primes
// below 2^60 the inverse can skip half of its conditional subtractions (SEMI):
// a sum output may stay below 8q, and is only reduced when both of its inputs
// were sums themselves (see gs_bfly_semi).  Twiddles are (w, floor(w 2^64 / q))
// pairs.
#pragma once
#include <hip/hip_runtime.h>
#include "modarith.hpp"

struct Tw {
    uint64_t w, wp;
};

template <int L, int LE = 4>
struct Geo {
    static_assert(L >= LE, "row shorter than one thread's elements");
    static constexpr int N = 1 << L;
    static constexpr int E = 1 << LE;
    static constexpr int LT = L - LE;
    static constexpr int T = 1 << LT;
    static constexpr int NPASS = (L + LE - 1) / LE;
    static constexpr int lds_words = N + N / 16;
    static constexpr int R(int p) { return p < L / LE ? LE : L % LE; }
    static constexpr int LO(int p) { return L - LE * p - R(p); }
};

__device__ __forceinline__ uint32_t lds_pos(uint32_t idx) { return idx + (idx >> 4); }

// Opaque copy of a value: index math derived from it is recomputed where it is
// used instead of being kept live (as 16 addresses per row) across stages.
__device__ __forceinline__ uint32_t fresh(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

// The (L - r) index bits a thread keeps fixed in pass P, from (tid, group g).
// With whole waves (T >= 64) the wave id goes to the top, the group next and
// the lane at the bottom, so that from pass 1 on every wave owns one closed
// block of 64 * E consecutive indices: the exchanges between passes >= 1 never
// leave the wave and need no workgroup barrier.
template <int L, int LE, int P>
__device__ __forceinline__ uint32_t fixed_bits(uint32_t tid, uint32_t g) {
    constexpr int r = Geo<L, LE>::R(P), LT = Geo<L, LE>::LT;
    constexpr int lgG = LE - r;
    if constexpr (LT >= 6 && lgG > 0)
        return ((tid >> 6) << (6 + lgG)) | (g << 6) | (tid & 63u);
    else
        return (g << LT) | tid;
}

// Global index of element e of group g of thread tid in pass P.
// (Unsigned so that row + index addressing can use a scalar base with a
// 32-bit vector offset.)
template <int L, int LE, int P>
__device__ __forceinline__ uint32_t elem_index(uint32_t tid, uint32_t g, uint32_t e) {
    constexpr int r = Geo<L, LE>::R(P), lo = Geo<L, LE>::LO(P);
    const uint32_t F = fixed_bits<L, LE, P>(tid, g);
    return ((F >> lo) << (lo + r)) | (e << lo) | (F & ((1u << lo) - 1u));
}

// 2^64 - q for mul_shoup_lazy4n, opaque to the compiler (which would
// otherwise fold the sum back into a subtraction).  q is uniform.
__device__ __forceinline__ uint64_t neg_opaque(uint64_t q) {
    const uint64_t n = 0 - q;
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)n);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(n >> 32));
    asm("" : "+s"(lo), "+s"(hi));
    return ((uint64_t)hi << 32) | lo;
}

// q4 = 4q.  REDUCE: X, Y in [0, 8q) -> [0, 8q); otherwise bounds grow by 4q.
template <bool REDUCE>
__device__ __forceinline__ void ct_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp,
                                        uint64_t nq, uint64_t q4) {
    uint64_t x = REDUCE ? csub(X, q4) : X;       // [0, 4q)
    uint64_t t = mul_shoup_lazy4n(Y, w, wp, nq); // [0, 4q)
    X = x + t;                                   // [0, 8q)
    Y = x - t + q4;                              // (0, 8q)
}

// X, Y in [0, 4q) -> [0, 4q).
__device__ __forceinline__ void gs_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp,
                                        uint64_t nq, uint64_t q4) {
    uint64_t x = X, y = Y;
    X = csub(x + y, q4);
    Y = mul_shoup_lazy4n(x - y + q4, w, wp, nq);
}

// Inverse butterfly with a two-class bound (16q < 2^64): X, Y below b, where b
// = 8q if they are sum outputs of the previous level (BIG) and b = 4q
// otherwise.  The sum x + y is below 2b: reduced by 8q only when BIG, so every
// sum output stays below 8q; the difference x - y + b is below 2b and its
// product lands in [0, 4q).
template <bool BIG>
__device__ __forceinline__ void gs_bfly_semi(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp,
                                             uint64_t nq, uint64_t b) {
    uint64_t x = X, y = Y;
    const uint64_t s = x + y;
    X = BIG ? csub(s, b) : s;
    Y = mul_shoup_lazy4n(x - y + b, w, wp, nq);
}

// Twiddle i.  UNIFORM: the index is the same in every lane of the wave; the
// table is then read through the constant address space, which lets the
// compiler use scalar loads (merged into wide ones, one wait per pass) instead
// of per-lane vector loads waited one at a time.
template <bool UNIFORM>
__device__ __forceinline__ Tw load_tw(const Tw *__restrict__ tw, uint32_t i) {
    if constexpr (UNIFORM) {
        typedef const __attribute__((address_space(4))) uint64_t *cptr;
        const cptr p = (cptr)tw + 2u * i;
        return Tw{p[0], p[1]};
    } else {
        return tw[i];
    }
}

template <int L, int LE, int P, bool REDUCE>
__device__ __forceinline__ void fwd_pass(uint64_t (&x)[1 << LE], int tid, const Tw *__restrict__ tw,
                                         uint64_t q) {
    constexpr int r = Geo<L, LE>::R(P), lo = Geo<L, LE>::LO(P), LT = Geo<L, LE>::LT;
    constexpr int R = 1 << r, G = (1 << LE) >> r, l0 = LE * P;
    const uint64_t q4 = q << 2, nq = neg_opaque(q);
#pragma unroll
    for (int g = 0; g < G; g++) {
        const uint32_t F = fixed_bits<L, LE, P>((uint32_t)tid, (uint32_t)g);
        uint32_t H = F >> lo;
        if constexpr (lo >= 6 || LT <= lo) H = __builtin_amdgcn_readfirstlane(H);
#pragma unroll
        for (int u = 0; u < r; u++) {
            const int half = R >> (u + 1);
#pragma unroll
            for (int v = 0; v < (1 << u); v++) {
                const Tw W = load_tw<(lo >= 6 || LT <= lo)>(tw, (1u << (l0 + u)) + (H << u) + v);
#pragma unroll
                for (int w = 0; w < half; w++) {
                    const int e0 = (v << (r - u)) | w;
                    ct_bfly<REDUCE>(x[g * R + e0], x[g * R + e0 + half], W.w, W.wp, nq, q4);
                }
            }
        }
    }
}

// SEMI: the level of bit b (b = r - 1 - u) pairs elements whose lower bits
// agree, so both were sum outputs of the previous level exactly when bit b - 1
// of their slot is 0.  The first level of a pass takes the bound its input
// had: below 4q for the transform's input, below 8q after an exchange.
template <int L, int LE, int P, bool SEMI>
__device__ __forceinline__ void inv_pass(uint64_t (&x)[1 << LE], int tid, const Tw *__restrict__ tw,
                                         uint64_t q) {
    constexpr int r = Geo<L, LE>::R(P), lo = Geo<L, LE>::LO(P), LT = Geo<L, LE>::LT;
    constexpr int R = 1 << r, G = (1 << LE) >> r, l0 = LE * P;
    constexpr bool FIRST = P == Geo<L, LE>::NPASS - 1;
    const uint64_t q4 = q << 2, q8 = q << 3, nq = neg_opaque(q);
#pragma unroll
    for (int g = 0; g < G; g++) {
        const uint32_t F = fixed_bits<L, LE, P>((uint32_t)tid, (uint32_t)g);
        uint32_t H = F >> lo;
        if constexpr (lo >= 6 || LT <= lo) H = __builtin_amdgcn_readfirstlane(H);
#pragma unroll
        for (int u = r - 1; u >= 0; u--) {
            const int half = R >> (u + 1);
#pragma unroll
            for (int v = 0; v < (1 << u); v++) {
                const Tw W = load_tw<(lo >= 6 || LT <= lo)>(tw, (1u << (l0 + u)) + (H << u) + v);
#pragma unroll
                for (int w = 0; w < half; w++) {
                    const int e0 = (v << (r - u)) | w;
                    uint64_t &X = x[g * R + e0], &Y = x[g * R + e0 + half];
                    if constexpr (SEMI) {
                        const bool big = u == r - 1 ? !FIRST : ((w >> (r - 2 - u)) & 1) == 0;
                        if (big) gs_bfly_semi<true>(X, Y, W.w, W.wp, nq, q8);
                        else gs_bfly_semi<false>(X, Y, W.w, W.wp, nq, q4);
                    } else {
                        gs_bfly(X, Y, W.w, W.wp, nq, q4);
                    }
                }
            }
        }
    }
}

template <int L, int LE, int P>
__device__ __forceinline__ void lds_store(uint64_t *lds, const uint64_t (&x)[1 << LE], int tid) {
    constexpr int R = 1 << Geo<L, LE>::R(P), G = (1 << LE) / R;
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int e = 0; e < R; e++) lds[lds_pos(elem_index<L, LE, P>(tid, g, e))] = x[g * R + e];
}

template <int L, int LE, int P>
__device__ __forceinline__ void lds_load(const uint64_t *lds, uint64_t (&x)[1 << LE], int tid) {
    constexpr int R = 1 << Geo<L, LE>::R(P), G = (1 << LE) / R;
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int e = 0; e < R; e++) x[g * R + e] = lds[lds_pos(elem_index<L, LE, P>(tid, g, e))];
}

// Re-layout of a row from pass A to pass B through LDS.  When pass 0 is one
// of the two and the row spans several waves, every wave exchanges with every
// other: workgroup barriers before (the buffer may still be read by the
// previous exchange) and between the store and the load.  Otherwise the
// exchange stays inside the wave, whose LDS operations execute in order, so
// only the compiler is kept from reordering them.
template <int L, int LE, int A, int B>
__device__ __forceinline__ void exchange(uint64_t *lds, uint64_t (&x)[1 << LE], int tid) {
    constexpr bool block = (A == 0 || B == 0) && Geo<L, LE>::T > 64;
    if constexpr (block) {
        __syncthreads();
        lds_store<L, LE, A>(lds, x, tid);
        __syncthreads();
        lds_load<L, LE, B>(lds, x, tid);
    } else {
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
        lds_store<L, LE, A>(lds, x, tid);
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
        lds_load<L, LE, B>(lds, x, tid);
    }
}

struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// Passes P.. of the forward transform.  hook() runs once, right after the
// exchange into the last pass (when the wave's LDS block is no longer read by
// this transform).
template <int L, int LE, int P, bool REDUCE, class Hook>
__device__ __forceinline__ void fwd_from(uint64_t (&x)[1 << LE], uint64_t *lds, int tid,
                                         const Tw *__restrict__ tw, uint64_t q, const Hook &hook) {
    fwd_pass<L, LE, P, REDUCE>(x, tid, tw, q);
    if constexpr (P + 1 < Geo<L, LE>::NPASS) {
        exchange<L, LE, P, P + 1>(lds, x, tid);
        if constexpr (P + 2 == Geo<L, LE>::NPASS) hook();
        fwd_from<L, LE, P + 1, REDUCE>(x, lds, tid, tw, q, hook);
    }
}

// Passes P..0 of the inverse transform.  hook() runs once, right after the
// exchange into pass 1 (from there on, at n = 2^14, every twiddle is
// wave-uniform: no vector-memory wait follows until the transform ends).
template <int L, int LE, int P, bool SEMI, class Hook>
__device__ __forceinline__ void inv_from(uint64_t (&x)[1 << LE], uint64_t *lds, int tid,
                                         const Tw *__restrict__ tw, uint64_t q, const Hook &hook) {
    inv_pass<L, LE, P, SEMI>(x, tid, tw, q);
    if constexpr (P > 0) {
        exchange<L, LE, P, P - 1>(lds, x, tid);
        if constexpr (P == 2) hook();
        inv_from<L, LE, P - 1, SEMI>(x, lds, tid, tw, q, hook);
    }
}

// Forward transform of a row held in registers in pass-0 (natural) layout.
// Leaves the transform in last-pass layout.  REDUCE: values < 8q in and out.
// Otherwise values < 4q in and < 4 (L + 1) q out, for q < 2^64 / (4 (L + 1)).
template <int L, int LE = 4, bool REDUCE = true, class Hook = NoHook>
__device__ __forceinline__ void ntt_fwd_regs(uint64_t (&x)[1 << LE], uint64_t *lds, int tid,
                                             const Tw *__restrict__ tw, uint64_t q,
                                             const Hook &hook = Hook()) {
    fwd_from<L, LE, 0, REDUCE>(x, lds, (int)fresh(tid), tw, q, hook);
}

// Inverse transform (without the 1/n factor) of a row held in last-pass
// layout, values < 4q.  Leaves natural order in pass-0 layout, values < 4q,
// or < 8q with SEMI (for q < 2^60).
template <int L, int LE = 4, bool SEMI = false, class Hook = NoHook>
__device__ __forceinline__ void ntt_inv_regs(uint64_t (&x)[1 << LE], uint64_t *lds, int tid,
                                             const Tw *__restrict__ tw, uint64_t q,
                                             const Hook &hook = Hook()) {
    inv_from<L, LE, Geo<L, LE>::NPASS - 1, SEMI>(x, lds, (int)fresh(tid), tw, q, hook);
}

// ---- two rows of the same prime at once --------------------------------
// The passes below transform two rows held in registers side by side: every
// twiddle is loaded once for both, and the two rows' butterflies give the
// scheduler independent work.  The exchanges stay one row at a time (the LDS
// holds one row).

template <int L, int LE, int P, bool REDUCE>
__device__ __forceinline__ void fwd_pass2(uint64_t (&x)[1 << LE], uint64_t (&y)[1 << LE], int tid,
                                          const Tw *__restrict__ tw, uint64_t q) {
    constexpr int r = Geo<L, LE>::R(P), lo = Geo<L, LE>::LO(P), LT = Geo<L, LE>::LT;
    constexpr int R = 1 << r, G = (1 << LE) >> r, l0 = LE * P;
    const uint64_t q4 = q << 2, nq = neg_opaque(q);
#pragma unroll
    for (int g = 0; g < G; g++) {
        const uint32_t F = fixed_bits<L, LE, P>((uint32_t)tid, (uint32_t)g);
        uint32_t H = F >> lo;
        if constexpr (lo >= 6 || LT <= lo) H = __builtin_amdgcn_readfirstlane(H);
#pragma unroll
        for (int u = 0; u < r; u++) {
            const int half = R >> (u + 1);
#pragma unroll
            for (int v = 0; v < (1 << u); v++) {
                const Tw W = load_tw<(lo >= 6 || LT <= lo)>(tw, (1u << (l0 + u)) + (H << u) + v);
#pragma unroll
                for (int w = 0; w < half; w++) {
                    const int e0 = (v << (r - u)) | w;
                    ct_bfly<REDUCE>(x[g * R + e0], x[g * R + e0 + half], W.w, W.wp, nq, q4);
                    ct_bfly<REDUCE>(y[g * R + e0], y[g * R + e0 + half], W.w, W.wp, nq, q4);
                }
            }
        }
    }
}

template <int L, int LE, int P, bool SEMI>
__device__ __forceinline__ void inv_pass2(uint64_t (&x)[1 << LE], uint64_t (&y)[1 << LE], int tid,
                                          const Tw *__restrict__ tw, uint64_t q) {
    constexpr int r = Geo<L, LE>::R(P), lo = Geo<L, LE>::LO(P), LT = Geo<L, LE>::LT;
    constexpr int R = 1 << r, G = (1 << LE) >> r, l0 = LE * P;
    constexpr bool FIRST = P == Geo<L, LE>::NPASS - 1;
    const uint64_t q4 = q << 2, q8 = q << 3, nq = neg_opaque(q);
#pragma unroll
    for (int g = 0; g < G; g++) {
        const uint32_t F = fixed_bits<L, LE, P>((uint32_t)tid, (uint32_t)g);
        uint32_t H = F >> lo;
        if constexpr (lo >= 6 || LT <= lo) H = __builtin_amdgcn_readfirstlane(H);
#pragma unroll
        for (int u = r - 1; u >= 0; u--) {
            const int half = R >> (u + 1);
#pragma unroll
            for (int v = 0; v < (1 << u); v++) {
                const Tw W = load_tw<(lo >= 6 || LT <= lo)>(tw, (1u << (l0 + u)) + (H << u) + v);
#pragma unroll
                for (int w = 0; w < half; w++) {
                    const int e0 = (v << (r - u)) | w;
                    uint64_t &X0 = x[g * R + e0], &Y0 = x[g * R + e0 + half];
                    uint64_t &X1 = y[g * R + e0], &Y1 = y[g * R + e0 + half];
                    if constexpr (SEMI) {
                        const bool big = u == r - 1 ? !FIRST : ((w >> (r - 2 - u)) & 1) == 0;
                        if (big) {
                            gs_bfly_semi<true>(X0, Y0, W.w, W.wp, nq, q8);
                            gs_bfly_semi<true>(X1, Y1, W.w, W.wp, nq, q8);
                        } else {
                            gs_bfly_semi<false>(X0, Y0, W.w, W.wp, nq, q4);
                            gs_bfly_semi<false>(X1, Y1, W.w, W.wp, nq, q4);
                        }
                    } else {
                        gs_bfly(X0, Y0, W.w, W.wp, nq, q4);
                        gs_bfly(X1, Y1, W.w, W.wp, nq, q4);
                    }
                }
            }
        }
    }
}

template <int L, int LE, int P, bool REDUCE>
__device__ __forceinline__ void fwd_from2(uint64_t (&x)[1 << LE], uint64_t (&y)[1 << LE], uint64_t *lds,
                                          int tid, const Tw *__restrict__ tw, uint64_t q) {
    fwd_pass2<L, LE, P, REDUCE>(x, y, tid, tw, q);
    if constexpr (P + 1 < Geo<L, LE>::NPASS) {
        exchange<L, LE, P, P + 1>(lds, x, tid);
        exchange<L, LE, P, P + 1>(lds, y, tid);
        fwd_from2<L, LE, P + 1, REDUCE>(x, y, lds, tid, tw, q);
    }
}

template <int L, int LE, int P, bool SEMI>
__device__ __forceinline__ void inv_from2(uint64_t (&x)[1 << LE], uint64_t (&y)[1 << LE], uint64_t *lds,
                                          int tid, const Tw *__restrict__ tw, uint64_t q) {
    inv_pass2<L, LE, P, SEMI>(x, y, tid, tw, q);
    if constexpr (P > 0) {
        exchange<L, LE, P, P - 1>(lds, x, tid);
        exchange<L, LE, P, P - 1>(lds, y, tid);
        inv_from2<L, LE, P - 1, SEMI>(x, y, lds, tid, tw, q);
    }
}

// ntt_fwd_regs / ntt_inv_regs of two rows of one prime.
template <int L, int LE = 4, bool REDUCE = true>
__device__ __forceinline__ void ntt_fwd_regs2(uint64_t (&x)[1 << LE], uint64_t (&y)[1 << LE], uint64_t *lds,
                                              int tid, const Tw *__restrict__ tw, uint64_t q) {
    fwd_from2<L, LE, 0, REDUCE>(x, y, lds, (int)fresh(tid), tw, q);
}

template <int L, int LE = 4, bool SEMI = false>
__device__ __forceinline__ void ntt_inv_regs2(uint64_t (&x)[1 << LE], uint64_t (&y)[1 << LE], uint64_t *lds,
                                              int tid, const Tw *__restrict__ tw, uint64_t q) {
    inv_from2<L, LE, Geo<L, LE>::NPASS - 1, SEMI>(x, y, lds, (int)fresh(tid), tw, q);
}

// Global index helpers for the two register layouts.
template <int L, int LE = 4>
__device__ __forceinline__ uint32_t natural_index(uint32_t tid, int s) {  // pass-0 layout, slot s
    return elem_index<L, LE, 0>(tid, 0, s);
}

template <int L, int LE = 4>
__device__ __forceinline__ uint32_t bitrev_layout_index(uint32_t tid, int s) {  // last-pass layout
    constexpr int P = Geo<L, LE>::NPASS - 1;
    constexpr int R = 1 << Geo<L, LE>::R(P);
    return elem_index<L, LE, P>(tid, s / R, s % R);
}

// Prefetch of a row's pass-0 elements through LDS (E = 16, T >= 64).  From
// pass 1 on, wave w keeps its exchanges inside the LDS block of positions
// lds_pos([1024 w, 1024 w + 1024)), which starts at word 1088 w.  Once the
// last exchange of a transform has been read, that block is free until the
// next transform's first (workgroup-wide) exchange; it can then receive the
// wave's pass-0 elements of the next row (16 runs of 64 consecutive residues,
// run s holding elements s T + 64 w + [0, 64)) by the LDS-DMA path, 16 bytes
// per lane and no registers, while the wave keeps computing.  Run s lands at
// word 1088 w + 64 s.  The caller waits for the copies (vmcnt) before reading.
typedef __attribute__((address_space(3))) void *lds_void_ptr;

template <int L>
__device__ __forceinline__ void prefetch_row_lds(uint64_t *lds, const uint64_t *__restrict__ src,
                                                 uint32_t tid) {
    constexpr uint32_t T = Geo<L>::T;
    static_assert(T >= 64, "whole waves only");
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the block's last reads are done
    const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63u;
    uint64_t *blk = lds + 1088u * w;
#pragma unroll
    for (uint32_t m = 0; m < 8; m++) {
        const uint32_t s = 2u * m + (l >> 5);
        const uint64_t *g = src + s * T + 64u * w + 2u * (l & 31u);
        __builtin_amdgcn_global_load_lds((const void *)g, (lds_void_ptr)(blk + 128u * m), 16, 0, 0);
    }
}

// Waits for the copies of prefetch_row_lds (and every other outstanding
// vector-memory load of the wave).
__device__ __forceinline__ void prefetch_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Slot s of the pass-0 layout of the prefetched row.
__device__ __forceinline__ uint64_t prefetched(const uint64_t *lds, uint32_t tid, int s) {
    return lds[1088u * (tid >> 6) + 64u * (uint32_t)s + (tid & 63u)];
}
