// The first radix-16 pass of the forward transform on the int8 matrix cores,
// beside the same pass on the vector ALU: a measured comparison of the two
// (the transforms of the product pipeline use the vector ALU).
//
// Pass 0 of the forward transform (levels 0..3 of the Cooley-Tukey network)
// treats every group of 16 residues x_e = a[g + e n/16] (e = 0..15,
// g = 0..n/16 - 1) alike: slot j of the group receives sum_e M[j][e] x_e mod q
// for one fixed 16 x 16 matrix M per prime.  Over all groups of a row that is
// a matrix product, so it can run on the matrix cores exactly:
//   x_e   = sum_u 2^(7u) x_{e,u}                 (8 limbs of 7 bits, x < 2^56)
//   y_j   = sum_e sum_u x_{e,u} (M[j][e] 2^(7u) mod q)
//         = sum_v 2^(7v) P_{j,v},  P_{j,v} = sum_{(e,u)} x_{e,u} W_v[j][(e,u)]
// with W_v the 7-bit limb v of (M[j][e] 2^(7u) mod q): a contraction of
// length 128 whose int8 products and int32 sums are exact (every P_{j,v} is
// below 128 * 127 * 127 < 2^21; for q < 2^55 limb 7 is below 2^6, so P_{j,7}
// < 2^20).  The shift 2^(7u) of the input limbs is folded into the matrix, so
// each output recombines only 8 partial sums: sum_{v<7} P_v 2^(7v) < 2^64,
// and y < 33 * 2^64.
//
// Operand layout (v_mfma_i32_16x16x64_i8, A rows x K, B K x columns, D rows x
// columns; A and B use the same K order): A = W_v (rows j), B = the limbs of 16
// groups (columns = groups), the contraction index kappa = (element e, limb u)
// taken as e = 4 (lane / 16) + 2h + byte / 8, u = byte % 8 in half h of the
// contraction (two instructions per output tile).  Lane l then holds the four
// residues x_e of group (l mod 16) with e = 4 (l/16) + i, i = 0..3, and
// receives D[j][group] for the same j = 4 (l/16) + i, for all 8 limbs v: the
// recombination stays in the lane, and the results feed the next pass as
// they are.
#include "kernels.hpp"
#include "modarith.hpp"
#include "ntt_core.hpp"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t canon8_p0(uint64_t x, uint64_t q) {  // [0, 8q) -> [0, q)
    return csub(csub(csub(x, q << 2), q << 1), q);
}

// 28 bits -> four bytes of 7 bits each (byte b = bits 7b .. 7b + 6).
__device__ __forceinline__ uint32_t spread7(uint32_t t) {
    t &= 0x0FFFFFFFu;
    const uint32_t s = (t & 0x3FFFu) | ((t & 0x0FFFC000u) << 2);
    return (s & 0x007F007Fu) | ((s & 0x3F803F80u) << 1);
}

// VALU reference: thread g holds group g (slots e at g + e n/16), runs the
// four butterfly levels of the forward transform's first pass `reps` times
// (values stay below 8q between passes) and stores the canonical results in
// place.
template <int L>
__global__ __launch_bounds__(Geo<L>::T) void k_pass0_valu(DevCtx c, uint64_t *__restrict__ data, int kmod,
                                                         int limb_off, int reps) {
    constexpr int n = 1 << L;
    const size_t row = blockIdx.x;
    const int limb = (int)(row % kmod) + limb_off;
    const uint64_t q = c.pc[limb].q;
    uint64_t *ptr = data + row * n;
    const uint32_t tid = threadIdx.x;
    uint64_t x[16];
#pragma unroll
    for (int s = 0; s < 16; s++) x[s] = ptr[natural_index<L>(tid, s)];
    for (int rep = 0; rep < reps; rep++) fwd_pass<L, 4, 0, true>(x, (int)tid, c.tw + (size_t)limb * n, q);
    const uint32_t t1 = fresh(tid);
#pragma unroll
    for (int s = 0; s < 16; s++) ptr[natural_index<L>(t1, s)] = canon8_p0(x[s], q);
}

// Matrix-core version.  Workgroup = one row, four waves; wave w handles the
// tiles (16 consecutive groups each) [w TPW, (w + 1) TPW).  Lane l holds slots
// 4 (l/16) + i (i = 0..3) of group 16 tile + (l mod 16): the slots it loads are
// the slots it receives, so `reps` passes run back to back on the registers.
// Wt: per limb [h][v][lane] 16-byte A operands, built for that layout with the
// factor 2^64 folded in, so that one Montgomery reduction of the recombined
// sum y = H 2^64 + lo (H <= 32) returns y 2^-64 = (M x)_j mod q.
template <int L>
__global__ __launch_bounds__(256) void k_pass0_mfma(DevCtx c, const v4i *__restrict__ Wt,
                                                   uint64_t *__restrict__ data, int kmod, int limb_off, int reps) {
    constexpr int n = 1 << L, S = n / 16, TPW = S / 64;
    static_assert(TPW >= 1, "rows of at least 1024 residues");
    const size_t row = blockIdx.x;
    const int limb = (int)(row % kmod) + limb_off;
    const PrimeConst &P = c.pc[limb];
    const uint64_t q = P.q, qi = P.qinv_neg;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t col = lane & 15u, kg = lane >> 4;
    const v4i *wl = Wt + (size_t)limb * 16 * 64;
    v4i A[2][8];
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
        for (int v = 0; v < 8; v++) A[h][v] = wl[(h * 8 + v) * 64 + lane];
    uint64_t *ptr = data + row * n;
    for (int tile = 0; tile < TPW; tile++) {
        const uint32_t g = (wave * TPW + tile) * 16u + col;
        uint64_t y[4];
#pragma unroll
        for (int i = 0; i < 4; i++) y[i] = ptr[g + (4u * kg + i) * S];
        for (int rep = 0; rep < reps; rep++) {
            v4i B[2];
#pragma unroll
            for (int h = 0; h < 2; h++)
                B[h] = v4i{(int)spread7((uint32_t)y[2 * h]), (int)spread7((uint32_t)(y[2 * h] >> 28)),
                           (int)spread7((uint32_t)y[2 * h + 1]), (int)spread7((uint32_t)(y[2 * h + 1] >> 28))};
            v4i acc[8];
#pragma unroll
            for (int v = 0; v < 8; v++) {
                acc[v] = v4i{0, 0, 0, 0};
                acc[v] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[0][v], B[0], acc[v], 0, 0, 0);
                acc[v] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[1][v], B[1], acc[v], 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; i++) {
                // y = sum_v 2^(7v) P_v = H 2^64 + lo
                uint64_t s = 0;
#pragma unroll
                for (int v = 0; v < 7; v++) s += (uint64_t)(uint32_t)acc[v][i] << (7 * v);
                const uint32_t p7 = (uint32_t)acc[7][i];
                const uint64_t lo = s + ((uint64_t)(p7 & 0x7FFFu) << 49);
                const uint64_t H = (p7 >> 15) + (lo < s ? 1u : 0u);
                y[i] = csub(redc_lazy(H, lo, q, qi), q);
            }
        }
        // every lane's loads of this tile were consumed before any store
#pragma unroll
        for (int i = 0; i < 4; i++) ptr[g + (4u * kg + i) * S] = y[i];
    }
}

template <int L>
struct Pass0L {
    static hipError_t run(const DevCtx &c, int method, const void *Wt, uint64_t *data, size_t nrows, int kmod,
                          int limb_off, int reps, hipStream_t s) {
        if (method == 0)
            hipLaunchKernelGGL((k_pass0_valu<L>), dim3((unsigned)nrows), dim3(Geo<L>::T), 0, s, c, data, kmod,
                               limb_off, reps);
        else
            hipLaunchKernelGGL((k_pass0_mfma<L>), dim3((unsigned)nrows), dim3(256), 0, s, c, (const v4i *)Wt, data,
                               kmod, limb_off, reps);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_pass0(const DevCtx &c, int method, const void *Wt, uint64_t *data, size_t nrows, int kmod,
                        int limb_off, int reps, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    switch (c.L) {
        case 10: return Pass0L<10>::run(c, method, Wt, data, nrows, kmod, limb_off, reps, s);
        case 11: return Pass0L<11>::run(c, method, Wt, data, nrows, kmod, limb_off, reps, s);
        case 12: return Pass0L<12>::run(c, method, Wt, data, nrows, kmod, limb_off, reps, s);
        case 13: return Pass0L<13>::run(c, method, Wt, data, nrows, kmod, limb_off, reps, s);
        case 14: return Pass0L<14>::run(c, method, Wt, data, nrows, kmod, limb_off, reps, s);
        default: return hipErrorInvalidValue;
    }
}
