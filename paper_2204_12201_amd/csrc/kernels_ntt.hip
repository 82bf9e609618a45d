// Transform kernels: one workgroup of n/16 threads per row (ntt_core.hpp).
//
//  k_ntt_rows      generic batched forward / inverse transform of rows
//  k_fwd_ext       forward transform of the extended inputs of a product
//  k_tensor_intt   tensor component (Montgomery products of transformed
//                  inputs, computed on load) followed by the inverse transform
//                  (the product path for small batches: more workgroups)
//  k_mul_tensor    product of two ciphertexts: forward transforms of the four
//                  input polynomials and the three inverse-transformed tensor
//                  components in one pass
//  k_square_tensor squaring: forward transforms of both input polynomials and
//                  the three inverse-transformed tensor components in one pass
//  k_relin_fused   key switching: digit transforms, inner product with the key
//                  and inverse transforms for one output limb
#include "kernels.hpp"
#include "modarith.hpp"
#include "ntt_core.hpp"

namespace {

__device__ __forceinline__ uint64_t canon8(uint64_t x, uint64_t q) {  // [0, 8q) -> [0, q)
    return csub(csub(csub(x, q << 2), q << 1), q);
}

template <int L>
__device__ __forceinline__ void load_natural(uint64_t (&x)[16], const uint64_t *__restrict__ src,
                                             int tid) {
#pragma unroll
    for (int s = 0; s < 16; s++) x[s] = src[natural_index<L>(tid, s)];
}

template <int L>
__device__ __forceinline__ void load_bitrev(uint64_t (&x)[16], const uint64_t *__restrict__ src,
                                            int tid) {
#pragma unroll
    for (int s = 0; s < 16; s++) x[s] = src[bitrev_layout_index<L>(tid, s)];
}

// Shoup products whose remainder a w - h q is formed as a w + h (2^64 - q)
// (equal modulo 2^64, no borrow chain; see neg_opaque).
__device__ __forceinline__ uint64_t mul_shoup_s(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    return csub(a * w + mulhi64(a, wp) * neg_opaque(q), q);
}
__device__ __forceinline__ uint64_t mul_shoup_lazy4_s(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    return mul_shoup_lazy4n(a, w, wp, neg_opaque(q));
}

// Canonical residue of any 64-bit value: Shoup multiplication by 1.
__device__ __forceinline__ uint64_t canon_any(uint64_t x, uint64_t q, uint64_t one_p) {
    return mul_shoup_s(x, 1, one_p, q);
}

// mode: NttMode (kernels.hpp).  Rows row0, row0 + gridDim.x, ... of data:
// the workgroups stay resident and fetch their next row while the current one
// is transformed (forward with whole waves: into LDS by prefetch_row_lds;
// otherwise into registers).  LZ: every prime below 2^64 / (4 (L + 1)): the
// forward transform skips its conditional subtractions and the inverse half of
// them.
template <int L, bool FWD, bool LZ>
__global__ __launch_bounds__(Geo<L>::T) void k_ntt_rows(DevCtx c, uint64_t *__restrict__ data,
                                                       size_t nrows, int kmod, int limb_off, int mode) {
    __shared__ uint64_t lds[Geo<L>::lds_words];
    constexpr int n = Geo<L>::N;
    constexpr bool DMA = FWD && Geo<L>::T >= 64;
    const uint32_t tid = threadIdx.x;
    size_t row = blockIdx.x;
    uint64_t x[16];
    if constexpr (FWD) load_natural<L>(x, data + row * n, tid);
    else load_bitrev<L>(x, data + row * n, tid);
    for (; row < nrows; row += gridDim.x) {
        const int limb = (int)(row % kmod) + limb_off;
        const PrimeConst &P = c.pc[limb];
        const uint64_t q = P.q;
        uint64_t *ptr = data + row * n;
        const size_t next = row + gridDim.x;
        uint64_t nx[16];
        if constexpr (DMA) {
            auto hook = [&]() {
                if (next < nrows) prefetch_row_lds<L>(lds, data + next * n, fresh(tid));
            };
            ntt_fwd_regs<L, 4, !LZ>(x, lds, tid, c.tw + (size_t)limb * n, q, hook);
        } else {
            if (next < nrows) {
                if constexpr (FWD) load_natural<L>(nx, data + next * n, fresh(tid));
                else load_bitrev<L>(nx, data + next * n, fresh(tid));
            }
            if constexpr (FWD) ntt_fwd_regs<L, 4, !LZ>(x, lds, tid, c.tw + (size_t)limb * n, q);
            else ntt_inv_regs<L, 4, LZ>(x, lds, tid, c.itw + (size_t)limb * n, q);
        }
        const uint32_t t1 = fresh(tid);
        if constexpr (FWD) {
            // the prefetch is waited for before this row's stores are issued
            // (the wait counter covers stores too), so that they drain while
            // the next row is transformed
            if constexpr (DMA)
                if (next < nrows) prefetch_wait();
#pragma unroll
            for (int s = 0; s < 16; s++) {
                uint64_t v;
                if (mode == NTT_FWD_NINVM) v = mul_shoup_s(x[s], P.ninvm, P.ninvm_p, q);
                else v = LZ ? canon_any(x[s], q, P.one_p) : canon8(x[s], q);
                ptr[bitrev_layout_index<L>(t1, s)] = v;
            }
        } else {
            const uint64_t w = mode == NTT_INV ? P.ninv : P.ninvm;
            const uint64_t wp = mode == NTT_INV ? P.ninv_p : P.ninvm_p;
#pragma unroll
            for (int s = 0; s < 16; s++) ptr[natural_index<L>(t1, s)] = mul_shoup_s(x[s], w, wp, q);
            // the inverse ends on the workgroup-wide exchange and the next row
            // starts with a wave-local one in the same buffer
            __syncthreads();
        }
        if (next < nrows) {
            if constexpr (DMA) {
                const uint32_t t0 = fresh(tid);
#pragma unroll
                for (int s = 0; s < 16; s++) x[s] = prefetched(lds, t0, s);
            } else {
#pragma unroll
                for (int s = 0; s < 16; s++) x[s] = nx[s];
            }
        }
    }
}

// Rows (item, poly, limb), grid (K, npoly, items).  Q limbs come from the
// input ciphertexts, P limbs from E (written there by the lift); the forward
// transforms land in E[item][poly][limb], canonical.
template <int L, bool LZ>
__global__ __launch_bounds__(Geo<L>::T) void k_fwd_ext(DevCtx c, const uint64_t *__restrict__ a,
                                                      const uint64_t *__restrict__ b,
                                                      uint64_t *__restrict__ E, int npoly) {
    __shared__ uint64_t lds[Geo<L>::lds_words];
    constexpr int n = Geo<L>::N;
    const uint32_t tid = threadIdx.x;
    const int limb = blockIdx.x, poly = blockIdx.y;
    const size_t item = blockIdx.z;
    const int k = c.k, K = c.K;
    const uint64_t q = c.pc[limb].q, one_p = c.pc[limb].one_p;
    uint64_t *dst = E + ((item * npoly + poly) * K + limb) * (size_t)n;
    const uint64_t *src;
    if (limb < k)
        src = (poly < 2 ? a + ((item * 2 + poly) * k + limb) * (size_t)n
                        : b + ((item * 2 + poly - 2) * k + limb) * (size_t)n);
    else
        src = dst;
    uint64_t x[16];
    load_natural<L>(x, src, tid);
    ntt_fwd_regs<L, 4, !LZ>(x, lds, tid, c.tw + (size_t)limb * n, q);
#pragma unroll
    for (int s = 0; s < 16; s++)
        dst[bitrev_layout_index<L>(tid, s)] = LZ ? canon_any(x[s], q, one_p) : canon8(x[s], q);
}

// grid (K, 3, items): component comp of the tensor of item, limb `limb`.
// Montgomery products carry a factor 2^-64, removed with n^-1 by the final
// multiplication by n^-1 2^64.
template <int L, bool SQ, bool LZ>
__global__ __launch_bounds__(Geo<L>::T) void k_tensor_intt(DevCtx c, const uint64_t *__restrict__ E,
                                                          uint64_t *__restrict__ Dt) {
    __shared__ uint64_t lds[Geo<L>::lds_words];
    constexpr int n = Geo<L>::N;
    constexpr int npoly = SQ ? 2 : 4;
    const uint32_t tid = threadIdx.x;
    const int limb = blockIdx.x, comp = blockIdx.y;
    const size_t item = blockIdx.z;
    const int K = c.K;
    const PrimeConst &P = c.pc[limb];
    const uint64_t q = P.q, qi = P.qinv_neg, q2 = q << 1;
    const size_t rs = (size_t)K * n;  // stride between polys of one item
    const uint64_t *base = E + (item * npoly * K + limb) * (size_t)n;
    uint64_t x[16];
#pragma unroll
    for (int s = 0; s < 16; s++) {
        const uint32_t idx = bitrev_layout_index<L>(tid, s);
        uint64_t v;
        if (SQ) {
            const uint64_t a0 = base[idx], a1 = base[rs + idx];
            if (comp == 0) {
                v = mont_mul_lazy_u(a0, a0, q, qi);
            } else if (comp == 1) {
                const uint64_t m = mont_mul_lazy_u(a0, a1, q, qi);  // d1 = 2 a0 a1
                v = csub(m + m, q2);
            } else {
                v = mont_mul_lazy_u(a1, a1, q, qi);
            }
        } else {
            const uint64_t a0 = base[idx], a1 = base[rs + idx];
            const uint64_t b0 = base[2 * rs + idx], b1 = base[3 * rs + idx];
            if (comp == 0) v = mont_mul_lazy_u(a0, b0, q, qi);
            else if (comp == 1)
                v = csub(mont_mul_lazy_u(a0, b1, q, qi) + mont_mul_lazy_u(a1, b0, q, qi), q2);
            else v = mont_mul_lazy_u(a1, b1, q, qi);
        }
        x[s] = csub(v, q2);  // [0, 2q)
    }
    ntt_inv_regs<L, 4, LZ>(x, lds, tid, c.itw + (size_t)limb * n, q);
    uint64_t *dst = Dt + ((item * 3 + comp) * K + limb) * (size_t)n;
#pragma unroll
    for (int s = 0; s < 16; s++) dst[natural_index<L>(tid, s)] = mul_shoup_s(x[s], P.ninvm, P.ninvm_p, q);
}

// A forward transform output as a Montgomery operand: below 4q (LZ: from
// below 4 (L + 1) q by a Shoup multiplication by 1) or below 2q (from below 8q
// by two conditional subtractions).  Two such operands multiply to less than
// q 2^64 for q < 2^60.
template <bool LZ>
__device__ __forceinline__ uint64_t fwd_operand(uint64_t v, uint64_t q, uint64_t one_p) {
    if constexpr (LZ) return mul_shoup_lazy4_s(v, 1, one_p, q);
    else return csub(csub(v, q << 2), q << 1);
}

// Product of two ciphertexts, transform phase fused: one task per (item,
// limb l), task = l + K item.  For limb l of item it transforms a0, a1, b0, b1
// (Q limbs from the inputs, P limbs from the lift in E), forms d0 = a0 b0, d1 =
// a0 b1 + a1 b0, d2 = a1 b1 (Montgomery products) and inverse transforms each
// into Dt[item][comp][l].  Two rows live in registers; A1, a1 b1 and a0 b1 are
// parked (transform domain) in the item's own output rows, which this task
// alone touches.  With whole waves, each of a0 and b0 is copied into LDS while
// the transform before it finishes (prefetch_row_lds).  PERSIST: a resident
// grid takes the tasks blockIdx.x, blockIdx.x + gridDim.x, ... and loads the
// next task's b1 row into the free registers of y during the last inverse
// transform (after its last vector-memory twiddle load), its a1 row right
// after the last store.  Otherwise grid (K, items), one task per workgroup.
template <int L, bool LZ, bool PERSIST>
__global__ __launch_bounds__(Geo<L>::T) void k_mul_tensor(DevCtx c, const uint64_t *__restrict__ a,
                                                         const uint64_t *__restrict__ b,
                                                         const uint64_t *__restrict__ E,
                                                         uint64_t *__restrict__ Dt, uint32_t tasks) {
    static_assert(!PERSIST || Geo<L>::NPASS >= 3, "the next task's rows load from the pass-2 exchange hook");
    __shared__ uint64_t lds[Geo<L>::lds_words];
    constexpr int n = Geo<L>::N;
    constexpr bool PREFETCH = Geo<L>::T >= 64;
    const uint32_t tid = threadIdx.x;
    const int k = c.k, K = c.K;
    uint32_t task = PERSIST ? blockIdx.x : blockIdx.x + blockIdx.y * (uint32_t)K;
    // row poly of a task: a0, a1 (Q limbs from a), b0, b1 (from b); P limbs from E
    auto row_of = [&](uint32_t t, int poly) {
        const int limb = (int)(t % (uint32_t)K);
        const size_t item = t / (uint32_t)K;
        return limb < k ? (poly < 2 ? a + ((item * 2 + poly) * k + limb) * (size_t)n
                                    : b + ((item * 2 + poly - 2) * k + limb) * (size_t)n)
                        : E + ((item * 4 + poly) * K + limb) * (size_t)n;
    };
    uint64_t x[16], y[16];
    {  // A1 and B1 of the first task
        const uint64_t *s1 = row_of(task, 1), *s3 = row_of(task, 3);
        const uint32_t t0 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) x[s] = s1[natural_index<L>(t0, s)];
#pragma unroll
        for (int s = 0; s < 16; s++) y[s] = s3[natural_index<L>(t0, s)];
    }
    for (;;) {
        const int limb = (int)(task % (uint32_t)K);
        const size_t item = task / (uint32_t)K;
        const PrimeConst &P = c.pc[limb];
        const uint64_t q = P.q, qi = P.qinv_neg, one_p = P.one_p;
        const Tw *tw = c.tw + (size_t)limb * n;
        const Tw *itw = c.itw + (size_t)limb * n;
        const uint64_t *src[4];
#pragma unroll
        for (int poly = 0; poly < 4; poly++) src[poly] = row_of(task, poly);
        uint64_t *d0 = Dt + ((item * 3 + 0) * K + limb) * (size_t)n;
        uint64_t *d1 = Dt + ((item * 3 + 1) * K + limb) * (size_t)n;
        uint64_t *d2 = Dt + ((item * 3 + 2) * K + limb) * (size_t)n;
        asm volatile("" ::: "memory");
        ntt_fwd_regs<L, 4, !LZ>(x, lds, tid, tw, q);
        auto pre_a0 = [&]() {
            if constexpr (PREFETCH) prefetch_row_lds<L>(lds, src[0], fresh(tid));
        };
        ntt_fwd_regs<L, 4, !LZ>(y, lds, tid, tw, q, pre_a0);
        // park A1 in d1 and a1 b1 in d2; B1 stays in y
        const uint32_t t1 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) {
            const uint32_t idx = bitrev_layout_index<L>(t1, s);
            const uint64_t a1 = fwd_operand<LZ>(x[s], q, one_p);
            y[s] = fwd_operand<LZ>(y[s], q, one_p);
            d1[idx] = a1;
            d2[idx] = mont_mul_lazy_u(a1, y[s], q, qi);
        }
        asm volatile("" ::: "memory");
        // A0
        const uint32_t t2 = fresh(tid);
        if (PREFETCH) {
            prefetch_wait();
#pragma unroll
            for (int s = 0; s < 16; s++) x[s] = prefetched(lds, t2, s);
        } else {
#pragma unroll
            for (int s = 0; s < 16; s++) x[s] = src[0][natural_index<L>(t2, s)];
        }
        auto pre_b0 = [&]() {
            if constexpr (PREFETCH) prefetch_row_lds<L>(lds, src[2], fresh(tid));
        };
        ntt_fwd_regs<L, 4, !LZ>(x, lds, tid, tw, q, pre_b0);
        // park a0 b1 in d0; A0 stays in x
        const uint32_t t3 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) {
            x[s] = fwd_operand<LZ>(x[s], q, one_p);
            d0[bitrev_layout_index<L>(t3, s)] = mont_mul_lazy_u(x[s], y[s], q, qi);
        }
        asm volatile("" ::: "memory");
        // B0
        const uint32_t t4 = fresh(tid);
        if (PREFETCH) {
            prefetch_wait();
#pragma unroll
            for (int s = 0; s < 16; s++) y[s] = prefetched(lds, t4, s);
        } else {
#pragma unroll
            for (int s = 0; s < 16; s++) y[s] = src[2][natural_index<L>(t4, s)];
        }
        ntt_fwd_regs<L, 4, !LZ>(y, lds, tid, tw, q);
        // d0 = a0 b0 in x, d1 = a1 b0 + a0 b1 in y (every thread rereads only the
        // positions it parked)
        const uint32_t t5 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) {
            const uint32_t idx = bitrev_layout_index<L>(t5, s);
            const uint64_t b0 = fwd_operand<LZ>(y[s], q, one_p);
            y[s] = mont_mul_lazy_u(d1[idx], b0, q, qi) + d0[idx];  // < 4q
            x[s] = mont_mul_lazy_u(x[s], b0, q, qi);
        }
        asm volatile("" ::: "memory");
        ntt_inv_regs<L, 4, LZ>(x, lds, tid, itw, q);
        const uint32_t t6 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) d0[natural_index<L>(t6, s)] = mul_shoup_s(x[s], P.ninvm, P.ninvm_p, q);
        // d2's parked product, read while d1 is transformed
        const uint32_t t7 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) x[s] = d2[bitrev_layout_index<L>(t7, s)];
        asm volatile("" ::: "memory");
        ntt_inv_regs<L, 4, LZ>(y, lds, tid, itw, q);
        const uint32_t t8 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) d1[natural_index<L>(t8, s)] = mul_shoup_s(y[s], P.ninvm, P.ninvm_p, q);
        // y is free (d1 stored): the next task's b1 goes there
        const uint32_t next = task + gridDim.x;
        const bool more = PERSIST && next < tasks;
        auto pre_next = [&]() {
            if constexpr (PERSIST) {
                if (more) {
                    const uint64_t *s3 = row_of(next, 3);
                    const uint32_t tn = fresh(tid);
#pragma unroll
                    for (int s = 0; s < 16; s++) y[s] = s3[natural_index<L>(tn, s)];
                }
            }
        };
        ntt_inv_regs<L, 4, LZ>(x, lds, tid, itw, q, pre_next);
        const uint32_t t9 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) d2[natural_index<L>(t9, s)] = mul_shoup_s(x[s], P.ninvm, P.ninvm_p, q);
        if (!more) break;
        {
            const uint64_t *s1 = row_of(next, 1);
            const uint32_t tn = fresh(tid);
#pragma unroll
            for (int s = 0; s < 16; s++) x[s] = s1[natural_index<L>(tn, s)];
        }
        task = next;
    }
}

// Squaring, transform phase fused: one task per (item, limb l), task = l + K
// item.  For limb l of item it transforms a0 and a1 (Q limbs straight from the
// ciphertext, P limbs from the lift in E), then forms d0 = a0^2, d1 = 2 a0 a1,
// d2 = a1^2 (Montgomery products) and inverse transforms each into
// Dt[item][comp][l].  Two rows live in registers: a0 and a1 are transformed
// side by side (one twiddle load for both); d1 (transform domain) is parked in
// its own output row, which this task alone touches, and read back while d2 is
// inverse transformed.  PERSIST: a resident grid of workgroups takes the tasks
// blockIdx.x, blockIdx.x + gridDim.x, ...; the next task's a1 row is loaded
// into the free registers of x during the last inverse transform of the
// current task (after its last vector-memory twiddle load), so that it
// arrives while that transform finishes and its output is stored, and its a0
// row right after that store.  Otherwise grid (K, items), one task per
// workgroup.
template <int L, bool LZ, bool PERSIST>
__global__ __launch_bounds__(Geo<L>::T) void k_square_tensor(DevCtx c, const uint64_t *__restrict__ a,
                                                            const uint64_t *__restrict__ E,
                                                            uint64_t *__restrict__ Dt, uint32_t tasks) {
    static_assert(!PERSIST || Geo<L>::NPASS >= 3, "the next task's rows load from the pass-2 exchange hook");
    __shared__ uint64_t lds[Geo<L>::lds_words];
    constexpr int n = Geo<L>::N;
    const uint32_t tid = threadIdx.x;
    const int k = c.k, K = c.K;
    uint32_t task = PERSIST ? blockIdx.x : blockIdx.x + blockIdx.y * (uint32_t)K;
    // rows a0 and a1 of a task (uniform: the task is the same in the whole workgroup)
    auto rows_of = [&](uint32_t t, const uint64_t *&s0, const uint64_t *&s1) {
        const int limb = (int)(t % (uint32_t)K);
        const size_t item = t / (uint32_t)K;
        if (limb < k) {
            s0 = a + ((item * 2 + 0) * k + limb) * (size_t)n;
            s1 = a + ((item * 2 + 1) * k + limb) * (size_t)n;
        } else {
            s0 = E + ((item * 2 + 0) * K + limb) * (size_t)n;
            s1 = E + ((item * 2 + 1) * K + limb) * (size_t)n;
        }
    };
    uint64_t x[16], y[16];
    {
        const uint64_t *src0, *src1;
        rows_of(task, src0, src1);
        const uint32_t t1 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) x[s] = src1[natural_index<L>(t1, s)];
#pragma unroll
        for (int s = 0; s < 16; s++) y[s] = src0[natural_index<L>(t1, s)];
    }
    for (;;) {
        const int limb = (int)(task % (uint32_t)K);
        const size_t item = task / (uint32_t)K;
        const PrimeConst &P = c.pc[limb];
        const uint64_t q = P.q, qi = P.qinv_neg, one_p = P.one_p;
        const Tw *tw = c.tw + (size_t)limb * n;
        const Tw *itw = c.itw + (size_t)limb * n;
        uint64_t *d0 = Dt + ((item * 3 + 0) * K + limb) * (size_t)n;
        uint64_t *d1 = Dt + ((item * 3 + 1) * K + limb) * (size_t)n;
        uint64_t *d2 = Dt + ((item * 3 + 2) * K + limb) * (size_t)n;
        asm volatile("" ::: "memory");
        ntt_fwd_regs2<L, 4, !LZ>(x, y, lds, tid, tw, q);  // A1, A0
        // d1 = 2 A0 A1 parked in d1; d0 = A0^2 in y, d2 = A1^2 in x (all below 4q)
        const uint32_t t2 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) {
            const uint64_t a1 = fwd_operand<LZ>(x[s], q, one_p);
            const uint64_t a0 = fwd_operand<LZ>(y[s], q, one_p);
            const uint64_t m = mont_mul_lazy_u(a0, a1, q, qi);
            d1[bitrev_layout_index<L>(t2, s)] = m + m;
            y[s] = mont_mul_lazy_u(a0, a0, q, qi);
            x[s] = mont_mul_lazy_u(a1, a1, q, qi);
        }
        asm volatile("" ::: "memory");
        ntt_inv_regs2<L, 4, LZ>(y, x, lds, tid, itw, q);
        const uint32_t t3 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) d0[natural_index<L>(t3, s)] = mul_shoup_s(y[s], P.ninvm, P.ninvm_p, q);
        // every thread rereads only the positions it parked
        const uint32_t t4 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) y[s] = d1[bitrev_layout_index<L>(t4, s)];
        const uint32_t t5 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) d2[natural_index<L>(t5, s)] = mul_shoup_s(x[s], P.ninvm, P.ninvm_p, q);
        asm volatile("" ::: "memory");
        // x is free (d2 stored): the next task's a1 goes there; its a0 is
        // loaded into y once y's row is stored
        const uint32_t next = task + gridDim.x;
        const bool more = PERSIST && next < tasks;
        auto pre_next = [&]() {
            if constexpr (PERSIST) {
                if (more) {
                    const uint64_t *src0, *src1;
                    rows_of(next, src0, src1);
                    const uint32_t tn = fresh(tid);
#pragma unroll
                    for (int s = 0; s < 16; s++) x[s] = src1[natural_index<L>(tn, s)];
                }
            }
        };
        ntt_inv_regs<L, 4, LZ>(y, lds, tid, itw, q, pre_next);
        const uint32_t t6 = fresh(tid);
#pragma unroll
        for (int s = 0; s < 16; s++) d1[natural_index<L>(t6, s)] = mul_shoup_s(y[s], P.ninvm, P.ninvm_p, q);
        if (!more) break;
        {
            const uint64_t *src0, *src1;
            rows_of(next, src0, src1);
            const uint32_t tn = fresh(tid);
#pragma unroll
            for (int s = 0; s < 16; s++) y[s] = src0[natural_index<L>(tn, s)];
        }
        task = next;
    }
}

// Product of two operands both already transformed: grid (K limbs, items).
// Item z multiplies input (item0 + z) mod na of Ahat by entry item0 + z of
// Bhat (both [.][2][K][n], transform domain, canonical): d0 = A0 B0,
// d1 = A0 B1 + A1 B0, d2 = A1 B1 (d2 parked in its own output row), three
// inverse transforms.  Used when every operand of a batch of products is
// reused (the power tree of the bridge caches the transforms of its powers).
template <int L, bool LZ>
__global__ __launch_bounds__(Geo<L>::T) void k_mul_tensor_pre2(DevCtx c, const uint64_t *__restrict__ Ahat,
                                                              int na, size_t item0,
                                                              const uint64_t *__restrict__ Bhat,
                                                              uint64_t *__restrict__ Dt) {
    __shared__ uint64_t lds[Geo<L>::lds_words];
    constexpr int n = Geo<L>::N;
    const uint32_t tid = threadIdx.x;
    const int limb = blockIdx.x;
    const size_t item = blockIdx.y;
    const int K = c.K;
    const PrimeConst &P = c.pc[limb];
    const uint64_t q = P.q, qi = P.qinv_neg;
    const Tw *itw = c.itw + (size_t)limb * n;
    const size_t ia = (item0 + item) % (size_t)na, ib = item0 + item;
    const uint64_t *a0h = Ahat + ((ia * 2 + 0) * K + limb) * (size_t)n;
    const uint64_t *a1h = Ahat + ((ia * 2 + 1) * K + limb) * (size_t)n;
    const uint64_t *b0h = Bhat + ((ib * 2 + 0) * K + limb) * (size_t)n;
    const uint64_t *b1h = Bhat + ((ib * 2 + 1) * K + limb) * (size_t)n;
    uint64_t *d0 = Dt + ((item * 3 + 0) * K + limb) * (size_t)n;
    uint64_t *d1 = Dt + ((item * 3 + 1) * K + limb) * (size_t)n;
    uint64_t *d2 = Dt + ((item * 3 + 2) * K + limb) * (size_t)n;
    uint64_t x[16], y[16];
    const uint32_t t2 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) {
        const uint32_t idx = bitrev_layout_index<L>(t2, s);
        const uint64_t a0 = a0h[idx], a1 = a1h[idx], b0 = b0h[idx], b1 = b1h[idx];
        d2[idx] = mont_mul_lazy_u(a1, b1, q, qi);
        x[s] = mont_mul_lazy_u(a0, b1, q, qi) + mont_mul_lazy_u(a1, b0, q, qi);  // below 4q
        y[s] = mont_mul_lazy_u(a0, b0, q, qi);
    }
    asm volatile("" ::: "memory");
    ntt_inv_regs2<L, 4, LZ>(y, x, lds, tid, itw, q);
    const uint32_t t3 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) d0[natural_index<L>(t3, s)] = mul_shoup_s(y[s], P.ninvm, P.ninvm_p, q);
    // every thread rereads only the positions it parked
    const uint32_t t4 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) y[s] = d2[bitrev_layout_index<L>(t4, s)];
    const uint32_t t5 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) d1[natural_index<L>(t5, s)] = mul_shoup_s(x[s], P.ninvm, P.ninvm_p, q);
    asm volatile("" ::: "memory");
    ntt_inv_regs<L, 4, LZ>(y, lds, tid, itw, q);
    const uint32_t t6 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) d2[natural_index<L>(t6, s)] = mul_shoup_s(y[s], P.ninvm, P.ninvm_p, q);
}

// Key switching fused: grid (k limbs j, items).  For every digit i the row
// [C2]_{q_i} is reduced mod q_j, transformed and multiply-accumulated with the
// key rows into two register accumulators (below 2q, or with LAZY summed
// unreduced and brought below 4q once at the end); both accumulators are then
// inverse transformed side by side and added into C0, C1.  The transformed digits
// never leave the chip.  rlk layout [digit i][comp l][limb j][n], transform
// domain, each entry premultiplied by n^-1 2^64 so that the Montgomery products
// give digit * key / n and the inverse transforms need no scaling.
// While digit i finishes its transform and inner product, each wave copies its
// share of digit i + 1 into its own LDS block (prefetch_row_lds).  LAZY: every
// q_j is below 2^64 / (4 (L + 1)) and 2^59, so the digit transforms skip the
// conditional subtractions (digits below 4 (L + 1) q_j, still a valid
// Montgomery operand against key entries below q_j) and the inverse transforms
// half of theirs (accumulators below 8q_j).  RAW (with LAZY): every Q prime
// is below 4 min_j q_j, so a digit word (below q_i) is already a valid lazy
// transform input modulo q_j and enters without the Shoup reduction by 1.
// The body for one (item, target limb j), run by Geo<L>::T threads (tid local
// to them) on their own LDS block of Geo<L>::lds_words words; store = false
// runs everything but the final read-modify-write of out (a workgroup member
// without a task of its own that must still take part in the barriers).
template <int L, bool LAZY, bool RAW>
__device__ __forceinline__ void relin_body(const DevCtx &c, const uint64_t *__restrict__ C2,
                                           const uint64_t *__restrict__ rlk, uint64_t *__restrict__ out,
                                           size_t item, int j, uint32_t tid, uint64_t *lds, bool store) {
    constexpr int n = Geo<L>::N;
    constexpr bool PREFETCH = Geo<L>::T >= 64;
    const int k = c.k;
    const PrimeConst &P = c.pc[j];
    const uint64_t q = P.q, qi = P.qinv_neg, q2 = q << 1, one_p = P.one_p;
    const Tw *tw = c.tw + (size_t)j * n;
    const uint64_t *c2 = C2 + item * (size_t)k * n;
    uint64_t acc0[16], acc1[16];
#pragma unroll
    for (int s = 0; s < 16; s++) {
        acc0[s] = 0;
        acc1[s] = 0;
    }
    for (int i = 0; i < k; i++) {
        uint64_t x[16];
        const uint32_t t0 = fresh(tid);
        if (PREFETCH && i > 0) {
            prefetch_wait();
#pragma unroll
            for (int s = 0; s < 16; s++) {  // digit mod q_j, < 4q
                const uint64_t v = prefetched(lds, t0, s);
                x[s] = RAW ? v : mul_shoup_lazy4_s(v, 1, one_p, q);
            }
        } else {
            const uint64_t *src = c2 + (size_t)i * n;
#pragma unroll
            for (int s = 0; s < 16; s++) {
                const uint64_t v = src[natural_index<L>(t0, s)];
                x[s] = RAW ? v : mul_shoup_lazy4_s(v, 1, one_p, q);
            }
        }
        auto hook = [&]() {
            if constexpr (PREFETCH)
                if (i + 1 < k) prefetch_row_lds<L>(lds, c2 + (size_t)(i + 1) * n, fresh(tid));
        };
        ntt_fwd_regs<L, 4, !LAZY>(x, lds, tid, tw, q, hook);
        // inner product with the key rows, the loads of slot pair s0 + 2 in
        // flight while pair s0 is multiplied
        const uint64_t *r0 = rlk + (((size_t)i * 2 + 0) * k + j) * n;
        const uint64_t *r1 = rlk + (((size_t)i * 2 + 1) * k + j) * n;
        const uint32_t t1 = fresh(tid);
        uint64_t ka[4], kb[4];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const uint32_t idx = bitrev_layout_index<L>(t1, u);
            ka[u] = r0[idx];
            kb[u] = r1[idx];
        }
#pragma unroll
        for (int s0 = 0; s0 < 16; s0 += 2) {
            if (s0 + 2 < 16) {
#pragma unroll
                for (int u = 0; u < 2; u++) {
                    const uint32_t idx = bitrev_layout_index<L>(t1, s0 + 2 + u);
                    ka[2 + u] = r0[idx];
                    kb[2 + u] = r1[idx];
                }
            }
            asm volatile("" ::: "memory");
#pragma unroll
            for (int u = 0; u < 2; u++) {
                // digit < 4 (L + 1) q and key entries < q: products below q 2^64,
                // each Montgomery result below 2q.  LAZY (q < 2^59): up to 16
                // of them are summed unreduced (below 32q); otherwise the sum is
                // kept below 2q.
                const uint64_t m0 = mont_mul_lazy(x[s0 + u], ka[u], q, qi);
                const uint64_t m1 = mont_mul_lazy(x[s0 + u], kb[u], q, qi);
                acc0[s0 + u] = LAZY ? acc0[s0 + u] + m0 : csub(acc0[s0 + u] + m0, q2);
                acc1[s0 + u] = LAZY ? acc1[s0 + u] + m1 : csub(acc1[s0 + u] + m1, q2);
            }
            ka[0] = ka[2];
            ka[1] = ka[3];
            kb[0] = kb[2];
            kb[1] = kb[3];
        }
    }
    uint64_t *o0 = out + (item * 2 * k + j) * (size_t)n;
    uint64_t *o1 = out + ((item * 2 + 1) * k + j) * (size_t)n;
    if constexpr (LAZY) {
#pragma unroll
        for (int s = 0; s < 16; s++) {  // below 32q (k <= 16) -> below 4q
            acc0[s] = csub(csub(csub(acc0[s], q << 4), q << 3), q << 2);
            acc1[s] = csub(csub(csub(acc1[s], q << 4), q << 3), q << 2);
        }
    }
    ntt_inv_regs2<L, 4, LAZY>(acc0, acc1, lds, tid, c.itw + (size_t)j * n, q);
    if (!store) return;
    const uint32_t t2 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) {
        const uint32_t idx = natural_index<L>(t2, s);
        o0[idx] = add_mod(canon8(acc0[s], q), o0[idx], q);
    }
    const uint32_t t3 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) {
        const uint32_t idx = natural_index<L>(t3, s);
        o1[idx] = add_mod(canon8(acc1[s], q), o1[idx], q);
    }
}

template <int L, bool LAZY, bool RAW>
__global__ __launch_bounds__(Geo<L>::T) void k_relin_fused(DevCtx c, const uint64_t *__restrict__ C2,
                                                          const uint64_t *__restrict__ rlk,
                                                          uint64_t *__restrict__ out) {
    __shared__ uint64_t lds[Geo<L>::lds_words];
    relin_body<L, LAZY, RAW>(c, C2, rlk, out, blockIdx.y, (int)blockIdx.x, threadIdx.x, lds, true);
}

// ---- key switching of several parts (ring sizes) in one persistent launch --
// Every workgroup (1024 threads, one row of 16384 words of LDS plus padding)
// takes tasks from a queue until it is empty.  A task is one (item, limb)
// row of a part at n = 16384, or two (n = 8192) or four (n = 4096)
// consecutive (item, limb) rows run side by side by 512- or 256-thread
// sub-groups with their own LDS blocks.  Parts come in the queue in the
// order given (largest ring first fills the chip with long tasks and leaves
// the short ones for the end).  The queue is one counter, zero at launch.
// Every part must have the key-switching variant (LAZY, RAW) of the launch.
// The row's item and limb come from the task index by the part's
// multiply-high reciprocal of k (exact for flat < 2^32 / k): an integer
// division would leave them in vector registers and with them every constant
// and twiddle address of the row.
template <int L, bool LAZY, bool RAW>
__device__ __forceinline__ void relin_persist_task(const RelinPart &P, uint32_t local, uint32_t tid, uint64_t *lds) {
    constexpr int T = Geo<L>::T, S = 1024 / T;
    static_assert(T % 64 == 0, "a wave lies inside one sub-group");
    // the sub-group (and with it the row: item, limb, constants, LDS block)
    // is the same in a whole wave: scalar values
    const uint32_t sub = __builtin_amdgcn_readfirstlane(tid / T), lt = tid - sub * T;
    const uint32_t k = P.c.k;
    const uint32_t total = P.items * k;
    uint32_t flat = local * S + sub;
    const bool active = flat < total;
    if (!active) flat = 0;  // a valid row to run alongside, nothing stored
    const uint32_t item = __umulhi(flat, P.kmagic), j = flat - item * k;
    relin_body<L, LAZY, RAW>(P.c, P.C2, P.rlk, P.out, item, (int)j, lt, lds + (size_t)sub * Geo<L>::lds_words,
                             active);
}

// The parts travel as a kernel argument (constant memory the compiler may
// reload at will, which keeps their fields out of the registers).
template <bool LAZY, bool RAW>
__global__ __launch_bounds__(1024) void k_relin_persist(const RelinQueue Q, unsigned int *__restrict__ queue) {
    // each workgroup leaves the loop once the counter has passed the last
    // task: every wave reads the same task index, so all of them leave
    __shared__ uint64_t lds[Geo<14>::lds_words];
    __shared__ uint32_t task_sh;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) task_sh = atomicAdd(&queue[0], 1u);
        __syncthreads();
        uint32_t local = __builtin_amdgcn_readfirstlane(task_sh);
        __syncthreads();
        int p = 0;
        while (p < Q.nparts && local >= Q.part[p].wg_tasks) {
            local -= Q.part[p].wg_tasks;
            p++;
        }
        if (p >= Q.nparts) break;  // the same decision in every wave
        const RelinPart &P = Q.part[p];
        switch (P.c.L) {
            case 12: relin_persist_task<12, LAZY, RAW>(P, local, tid, lds); break;
            case 13: relin_persist_task<13, LAZY, RAW>(P, local, tid, lds); break;
            default: relin_persist_task<14, LAZY, RAW>(P, local, tid, lds); break;
        }
    }
}

template <int L>
struct NttL {
    template <bool FWD, bool LZ>
    static hipError_t rows_dir(const DevCtx &c, uint64_t *data, size_t nrows, int kmod, int off, int mode,
                               hipStream_t s) {
        // one resident pass of workgroups over the chip (row loop inside)
        static int per_chip = 0;
        if (per_chip == 0) {
            int nb = 0, dev = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ntt_rows<L, FWD, LZ>, Geo<L>::T, 0) !=
                    hipSuccess ||
                hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                nb < 1 || cus < 1)
                return hipErrorInvalidValue;
            per_chip = nb * cus;
        }
        const size_t grid = nrows < (size_t)per_chip ? nrows : (size_t)per_chip;
        hipLaunchKernelGGL((k_ntt_rows<L, FWD, LZ>), dim3((unsigned)grid), dim3(Geo<L>::T), 0, s, c, data,
                           nrows, kmod, off, mode);
        return hipGetLastError();
    }
    static hipError_t rows(const DevCtx &c, uint64_t *data, size_t nrows, int kmod, int off, int mode,
                           hipStream_t s) {
        const bool fwd = mode == NTT_FWD || mode == NTT_FWD_NINVM;
        const uint64_t span = (kmod >= 64 ? ~0ull : (1ull << kmod) - 1) << off;
        if ((c.lazy_limbs & span) == span)
            return fwd ? rows_dir<true, true>(c, data, nrows, kmod, off, mode, s)
                       : rows_dir<false, true>(c, data, nrows, kmod, off, mode, s);
        return fwd ? rows_dir<true, false>(c, data, nrows, kmod, off, mode, s)
                   : rows_dir<false, false>(c, data, nrows, kmod, off, mode, s);
    }
    static hipError_t fwd_ext(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *E,
                              int npoly, size_t items, hipStream_t s) {
        const dim3 grid(c.K, npoly, (unsigned)items);
        if (c.lazy_all)
            hipLaunchKernelGGL((k_fwd_ext<L, true>), grid, dim3(Geo<L>::T), 0, s, c, a, b, E, npoly);
        else
            hipLaunchKernelGGL((k_fwd_ext<L, false>), grid, dim3(Geo<L>::T), 0, s, c, a, b, E, npoly);
        return hipGetLastError();
    }
    template <bool SQ>
    static void tensor_sq(const DevCtx &c, const uint64_t *E, uint64_t *Dt, size_t items, hipStream_t s) {
        const dim3 grid(c.K, 3, (unsigned)items);
        if (c.lazy_all)
            hipLaunchKernelGGL((k_tensor_intt<L, SQ, true>), grid, dim3(Geo<L>::T), 0, s, c, E, Dt);
        else
            hipLaunchKernelGGL((k_tensor_intt<L, SQ, false>), grid, dim3(Geo<L>::T), 0, s, c, E, Dt);
    }
    static hipError_t tensor(const DevCtx &c, const uint64_t *E, uint64_t *Dt, bool sq, size_t items,
                             hipStream_t s) {
        if (sq) tensor_sq<true>(c, E, Dt, items, s);
        else tensor_sq<false>(c, E, Dt, items, s);
        return hipGetLastError();
    }
    template <bool LZ>
    static hipError_t mul_tensor_lz(const DevCtx &c, const uint64_t *a, const uint64_t *b, const uint64_t *E,
                                    uint64_t *Dt, size_t items, hipStream_t s) {
        const uint32_t tasks = (uint32_t)(c.K * items);
        if constexpr (Geo<L>::NPASS >= 3) {
            static int resident = 0;  // workgroups of the resident grid the chip holds
            if (resident == 0) {
                int nb = 0, dev = 0, cus = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mul_tensor<L, LZ, true>, Geo<L>::T, 0) !=
                        hipSuccess ||
                    hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                    nb < 1 || cus < 1)
                    return hipErrorInvalidValue;
                resident = nb * cus;
            }
            if (tasks > (uint32_t)resident) {
                hipLaunchKernelGGL((k_mul_tensor<L, LZ, true>), dim3((unsigned)resident), dim3(Geo<L>::T), 0, s, c,
                                   a, b, E, Dt, tasks);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_mul_tensor<L, LZ, false>), dim3(c.K, (unsigned)items), dim3(Geo<L>::T), 0, s, c, a, b,
                           E, Dt, tasks);
        return hipGetLastError();
    }
    static hipError_t mul_tensor(const DevCtx &c, const uint64_t *a, const uint64_t *b, const uint64_t *E,
                                 uint64_t *Dt, size_t items, hipStream_t s) {
        return c.lazy_all ? mul_tensor_lz<true>(c, a, b, E, Dt, items, s)
                          : mul_tensor_lz<false>(c, a, b, E, Dt, items, s);
    }
    static hipError_t mul_tensor_pre2(const DevCtx &c, const uint64_t *Ahat, int na, size_t item0,
                                      const uint64_t *Bhat, uint64_t *Dt, size_t items, hipStream_t s) {
        const dim3 grid(c.K, (unsigned)items);
        if (c.lazy_all)
            hipLaunchKernelGGL((k_mul_tensor_pre2<L, true>), grid, dim3(Geo<L>::T), 0, s, c, Ahat, na, item0, Bhat,
                               Dt);
        else
            hipLaunchKernelGGL((k_mul_tensor_pre2<L, false>), grid, dim3(Geo<L>::T), 0, s, c, Ahat, na, item0,
                               Bhat, Dt);
        return hipGetLastError();
    }
    template <bool LZ>
    static hipError_t square_tensor_lz(const DevCtx &c, const uint64_t *a, const uint64_t *E, uint64_t *Dt,
                                       size_t items, hipStream_t s) {
        const uint32_t tasks = (uint32_t)(c.K * items);
        if constexpr (Geo<L>::NPASS >= 3) {
            // resident workgroups of the persistent kernel (same for both variants)
            static int resident = 0;
            if (resident == 0) {
                int nb = 0, dev = 0, cus = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_square_tensor<L, LZ, true>, Geo<L>::T, 0) !=
                        hipSuccess ||
                    hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                    nb < 1 || cus < 1)
                    return hipErrorInvalidValue;
                resident = nb * cus;
            }
            if (tasks > (uint32_t)resident) {
                hipLaunchKernelGGL((k_square_tensor<L, LZ, true>), dim3((unsigned)resident), dim3(Geo<L>::T), 0, s,
                                   c, a, E, Dt, tasks);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_square_tensor<L, LZ, false>), dim3(c.K, (unsigned)items), dim3(Geo<L>::T), 0, s, c, a,
                           E, Dt, tasks);
        return hipGetLastError();
    }
    static hipError_t square_tensor(const DevCtx &c, const uint64_t *a, const uint64_t *E, uint64_t *Dt,
                                    size_t items, hipStream_t s) {
        return c.lazy_all ? square_tensor_lz<true>(c, a, E, Dt, items, s)
                          : square_tensor_lz<false>(c, a, E, Dt, items, s);
    }
    static hipError_t relin_fused(const DevCtx &c, const uint64_t *C2, const uint64_t *rlk, uint64_t *out,
                                  size_t items, hipStream_t s) {
        const dim3 grid(c.k, (unsigned)items);
        if (c.lazy_q && c.digit_raw)
            hipLaunchKernelGGL((k_relin_fused<L, true, true>), grid, dim3(Geo<L>::T), 0, s, c, C2, rlk, out);
        else if (c.lazy_q)
            hipLaunchKernelGGL((k_relin_fused<L, true, false>), grid, dim3(Geo<L>::T), 0, s, c, C2, rlk, out);
        else
            hipLaunchKernelGGL((k_relin_fused<L, false, false>), grid, dim3(Geo<L>::T), 0, s, c, C2, rlk, out);
        return hipGetLastError();
    }
};

#define FHE_DISPATCH_L(Lval, CALL)            \
    switch (Lval) {                           \
        case 4: return NttL<4>::CALL;         \
        case 5: return NttL<5>::CALL;         \
        case 6: return NttL<6>::CALL;         \
        case 7: return NttL<7>::CALL;         \
        case 8: return NttL<8>::CALL;         \
        case 9: return NttL<9>::CALL;         \
        case 10: return NttL<10>::CALL;       \
        case 11: return NttL<11>::CALL;       \
        case 12: return NttL<12>::CALL;       \
        case 13: return NttL<13>::CALL;       \
        case 14: return NttL<14>::CALL;       \
        default: return hipErrorInvalidValue; \
    }

}  // namespace

hipError_t launch_ntt_rows(const DevCtx &c, uint64_t *data, size_t nrows, int kmod, int limb_off,
                           int mode, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    FHE_DISPATCH_L(c.L, rows(c, data, nrows, kmod, limb_off, mode, s));
}

hipError_t launch_fwd_ext(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *E,
                          int npoly, size_t items, hipStream_t s) {
    if (items == 0) return hipSuccess;
    FHE_DISPATCH_L(c.L, fwd_ext(c, a, b, E, npoly, items, s));
}

hipError_t launch_tensor_intt(const DevCtx &c, const uint64_t *E, uint64_t *Dt, bool square,
                              size_t items, hipStream_t s) {
    if (items == 0) return hipSuccess;
    FHE_DISPATCH_L(c.L, tensor(c, E, Dt, square, items, s));
}

hipError_t launch_mul_tensor(const DevCtx &c, const uint64_t *a, const uint64_t *b, const uint64_t *E,
                             uint64_t *Dt, size_t items, hipStream_t s) {
    if (items == 0) return hipSuccess;
    FHE_DISPATCH_L(c.L, mul_tensor(c, a, b, E, Dt, items, s));
}

hipError_t launch_mul_tensor_pre2(const DevCtx &c, const uint64_t *Ahat, int na, size_t item0, const uint64_t *Bhat,
                                  uint64_t *Dt, size_t items, hipStream_t s) {
    if (items == 0) return hipSuccess;
    FHE_DISPATCH_L(c.L, mul_tensor_pre2(c, Ahat, na, item0, Bhat, Dt, items, s));
}

hipError_t launch_square_tensor(const DevCtx &c, const uint64_t *a, const uint64_t *E, uint64_t *Dt,
                                size_t items, hipStream_t s) {
    if (items == 0) return hipSuccess;
    FHE_DISPATCH_L(c.L, square_tensor(c, a, E, Dt, items, s));
}

hipError_t launch_relin_fused(const DevCtx &c, const uint64_t *C2, const uint64_t *rlk, uint64_t *out,
                              size_t items, hipStream_t s) {
    if (items == 0) return hipSuccess;
    FHE_DISPATCH_L(c.L, relin_fused(c, C2, rlk, out, items, s));
}

hipError_t launch_relin_persist(const RelinQueue &Q, int lazy, int raw, unsigned int *queue, size_t tasks,
                                hipStream_t s) {
    if (Q.nparts <= 0 || tasks == 0) return hipSuccess;
    auto kern = lazy ? (raw ? k_relin_persist<true, true> : k_relin_persist<true, false>)
                     : k_relin_persist<false, false>;
    if (!lazy && raw) return hipErrorInvalidValue;
    static int resident = 0;  // workgroups the chip holds at once (same for every variant)
    if (resident == 0) {
        int nb = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 1024, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || nb < 1 ||
            cus < 1)
            return hipErrorInvalidValue;
        resident = nb * cus;
    }
    const unsigned grid = (unsigned)(tasks < (size_t)resident ? tasks : (size_t)resident);
    if (hipMemsetAsync(queue, 0, sizeof(unsigned int), s) != hipSuccess) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), 0, s, Q, queue);
    return hipGetLastError();
}
