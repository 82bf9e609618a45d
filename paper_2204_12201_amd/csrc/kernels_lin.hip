// Integer-weighted sums of ciphertexts (the modular stage of the paper's
// genotype-imputation case study, Section 4.4):
//   out[m] (+)= sum_{j < nj} w[m][j] in[j]   word by word, modulo the word's prime.
//
// Exact without 128-bit arithmetic: a word x < q < 2^61 splits as
// x = x_hi 2^32 + x_lo with x_hi < 2^29.  With every weight row's sum of
// |w| below 2^30, the signed sums
//   S_hi = sum w x_hi               (|S_hi| < 2^59)
//   S_lo = sum w (x_lo - 2^31) + 2^31 sum w  = sum w x_lo   (|S_lo| < 2^62)
// fit 64-bit integers (one v_mad_i64_i32 each per term, the weight a
// wave-uniform scalar); shifted by multiples of q (off59, off62) they become
// non-negative and below 2^64, and S = S_hi 2^32 + S_lo mod q is two Shoup
// products (by 2^32 mod q and by 1), each in [0, 4q), summed and reduced.
//
// The kernel is bound by writing the outputs (one word per output per input
// word position); the inputs of a position are read once per block of WS_M
// outputs and stay in the L2 / last-level cache between blocks.
#include "kernels.hpp"
#include "modarith.hpp"

namespace {

constexpr int WS_J = 32;  // inputs held in registers per launch
constexpr int WS_G = 8;   // weight rows are padded with zeros to a multiple of WS_G
constexpr int WS_M = 64;  // outputs per workgroup row

__device__ __forceinline__ uint64_t canon8w(uint64_t x, uint64_t q) {  // [0, 8q) -> [0, q)
    return csub(csub(csub(x, q << 2), q << 1), q);
}

// The constants of a word's prime that the final reduction uses, held in
// registers: read through the table after a store to out, the compiler would
// reload them, and the wait for the reload would also wait for every store
// before it.
struct LinPrime {
    uint64_t q, off59, off62, r32, r32_p, one_p;
};

__device__ __forceinline__ LinPrime lin_prime(const PrimeConst &P) {
    return LinPrime{P.q, P.off59, P.off62, P.r32, P.r32_p, P.one_p};
}

// S = S_hi 2^32 + S_lo mod q from the two signed sums (S_lo still without
// its 2^31 sum(w) correction), written or added to *o.
__device__ __forceinline__ void finish(int64_t sl, int64_t sh, int32_t ws, const LinPrime &P, uint64_t *o,
                                       int accumulate) {
    const uint64_t q = P.q;
    sl += (int64_t)ws * ((int64_t)1 << 31);
    const uint64_t a = (uint64_t)(sh + (int64_t)P.off59);
    const uint64_t b = (uint64_t)(sl + (int64_t)P.off62);
    uint64_t r = canon8w(mul_shoup_lazy4(a, P.r32, P.r32_p, q) + mul_shoup_lazy4(b, 1, P.one_p, q), q);
    if (accumulate) r = add_mod(r, *o, q);
    *o = r;
}

// grid (ceil(W / 256), ceil(nout / WS_M), items); W = 2 k n words per
// ciphertext.  Item z reads its nj <= WS_J inputs at in + z in_is + j in_js
// (one_first: input 0 is instead the noiseless encryption of 1, (Delta, 0),
// and input j >= 1 is at index j - 1), and writes output m at
// out + z out_is + m out_ms.  w: rows of stride wstride (device, zero beyond
// the last input of the row); accumulate: add into out instead of writing it.
__global__ __launch_bounds__(256) void k_weighted_sum(DevCtx c, const uint64_t *__restrict__ in, size_t in_js,
                                                      size_t in_is, int nj, int one_first,
                                                      const int32_t *__restrict__ w, int wstride,
                                                      size_t nout, uint64_t *__restrict__ out, size_t out_ms,
                                                      size_t out_is, int accumulate) {
    const size_t W = (size_t)2 * c.k * c.n;
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= W) return;
    const int limb = (int)((p >> c.L) % (size_t)c.k);
    const LinPrime P = lin_prime(c.pc[limb]);
    in += blockIdx.z * in_is;
    out += blockIdx.z * out_is;
    // the constant coefficient of the first polynomial carries Delta in the encryption of 1
    const uint64_t one = p < (size_t)c.k * c.n && (p & (c.n - 1)) == 0 ? c.cc->delta_q[limb] : 0;
    int32_t xl[WS_J], xh[WS_J];
#pragma unroll
    for (int j = 0; j < WS_J; j++) {
        uint64_t x = 0;
        if (j < nj) x = (one_first && j == 0) ? one : in[(size_t)(j - one_first) * in_js + p];
        xl[j] = (int32_t)((uint32_t)x ^ 0x80000000u);  // x_lo - 2^31
        xh[j] = (int32_t)(x >> 32);
        // opaque: keeps the products signed 32 x 32 bit (v_mad_i64_i32)
        // instead of being rewritten around the unsigned low word
        asm("" : "+v"(xl[j]), "+v"(xh[j]));
    }
    const size_t m0 = (size_t)blockIdx.y * WS_M;
    const size_t m1 = m0 + WS_M < nout ? m0 + WS_M : nout;
    // two outputs per iteration: four independent multiply-add chains
    for (size_t m = m0; m < m1; m += 2) {
        const bool two = m + 1 < m1;
        const int32_t *wr0 = w + m * (size_t)wstride;
        const int32_t *wr1 = two ? wr0 + wstride : wr0;
        int64_t sl0 = 0, sh0 = 0, sl1 = 0, sh1 = 0;
        int32_t ws0 = 0, ws1 = 0;
#pragma unroll
        for (int g = 0; g < WS_J / WS_G; g++) {
            if (g * WS_G < nj) {
#pragma unroll
                for (int u = 0; u < WS_G; u++) {
                    const int j = g * WS_G + u;
                    const int32_t w0 = wr0[j], w1 = wr1[j];
                    sl0 += (int64_t)w0 * xl[j];
                    sh0 += (int64_t)w0 * xh[j];
                    sl1 += (int64_t)w1 * xl[j];
                    sh1 += (int64_t)w1 * xh[j];
                    ws0 += w0;
                    ws1 += w1;
                }
            }
        }
        uint64_t *o = out + m * out_ms + p;
        finish(sl0, sh0, ws0, P, o, accumulate);
        if (two) finish(sl1, sh1, ws1, P, o + out_ms, accumulate);
    }
}

// ------------------------------------------------ on the int8 matrix cores --
//
// For weights of at most 127 in absolute value the sums are a matrix product,
// weights (outputs x inputs) times words (inputs x word positions), run on the
// int8 matrix cores exactly.  Every input word x (< q < 2^61) is written in
// balanced base-256 digits d_u in [-128, 127] (the bytes of (x + B) xor B, B
// = 0x80 in every byte), and per tile of 16 outputs x 16 word positions and
// pass of at most 64 inputs, one v_mfma_i32_16x16x64_i8 per digit u gives
//   P_u[m][p] = sum_j w[m][j] d_u(x_j[p]),   |P_u| <= 64 * 127 * 128 < 2^20.
// Started at FHE_MX_BIAS (so every P'_u is positive), the eight sums
// recombine without carries as T' = sum_u 256^u P'_u = B + A 2^32, where
// x = P'_0 + 2^8 P'_1 + 2^16 P'_2 + 2^24 P'_3 and w = P'_4 + ... + 2^24 P'_7
// (both below 2^47), A = floor(x / 2^32) + w and B = x mod 2^32.  With E =
// -FHE_MX_BIAS sum_u 256^u mod q (PrimeConst::mx_neg_bias) added, T' + E is
// the sum modulo q: (A + E_hi) r32 + (B + E_lo), two Shoup products.
//
// Operand layout (as for the base conversions): lane l of a wave supplies row
// l mod 16 of A (output 16 mt + l mod 16) and column l mod 16 of B (word
// position p0 + l mod 16), both with the 16 inputs 16 (l / 16) + b, b = 0..15,
// in bytes b; it receives outputs 16 mt + 4 (l / 16) + i, i = 0..3, of its
// column.

typedef int ws_v4i __attribute__((ext_vector_type(4)));

// Waves per workgroup of the matrix-core weighted sum (each a tile of 16 word positions).
constexpr int WSX_WAVES = 4;

__device__ __forceinline__ uint64_t ws_digits(uint64_t x) {
    constexpr uint64_t B = 0x8080808080808080ull;
    return (x + B) ^ B;
}

// Byte u of each of four words, packed (word i in byte i).
__device__ __forceinline__ uint32_t ws_gather(const uint64_t *d, int u) {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) r |= (uint32_t)((d[i] >> (8 * u)) & 0xFFu) << (8 * i);
    return r;
}

// Wave w of workgroup x takes word positions p0 = 16 (WSX_WAVES x + w) .. p0 + 15
// (input j at in + j in_js, output m at out + m out_ms) for the output tiles
// blockIdx.y, blockIdx.y + gridDim.y, ... < nmt; wt: the pass's A operands
// [nmt][64] (16 bytes each); accumulate: add into out.
__global__ __launch_bounds__(64 * WSX_WAVES) void k_weighted_sum_mx(DevCtx c, const uint64_t *__restrict__ in, size_t in_js,
                                                         int nj, const ws_v4i *__restrict__ wt, int nmt,
                                                         size_t nout, uint64_t *__restrict__ out, size_t out_ms,
                                                         int accumulate) {
    const size_t W = (size_t)2 * c.k * c.n;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, col = lane & 15u, g = lane >> 4;
    const size_t p0 = ((size_t)blockIdx.x * WSX_WAVES + wave) * 16;
    if (p0 >= W) return;  // whole waves
    const size_t p = p0 + col;
    const int limb = (int)((p0 >> c.L) % (size_t)c.k);
    // the prime's constants in registers (a store to out could alias the
    // table for the compiler, which would reload them, and wait, per output)
    const PrimeConst &P = c.pc[limb];
    const uint64_t q = P.q, E = P.mx_neg_bias, r32 = P.r32, r32p = P.r32_p, onep = P.one_p;
    // digits of the lane's 16 inputs, then one B operand per digit u
    uint64_t d[16];
#pragma unroll
    for (int b = 0; b < 16; b++) {
        const int j = (int)g * 16 + b;
        d[b] = j < nj ? ws_digits(in[(size_t)j * in_js + p]) : 0;
    }
    ws_v4i Bu[8];
#pragma unroll
    for (int u = 0; u < 8; u++)
        Bu[u] = ws_v4i{(int)ws_gather(d, u), (int)ws_gather(d + 4, u), (int)ws_gather(d + 8, u),
                       (int)ws_gather(d + 12, u)};
    const ws_v4i bias = {FHE_MX_BIAS, FHE_MX_BIAS, FHE_MX_BIAS, FHE_MX_BIAS};
    for (int mt = (int)blockIdx.y; mt < nmt; mt += (int)gridDim.y) {
        const ws_v4i A = wt[(size_t)mt * 64 + lane];
        ws_v4i acc[8];
#pragma unroll
        for (int u = 0; u < 8; u++) acc[u] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, Bu[u], bias, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const size_t m = (size_t)mt * 16 + 4 * g + i;
            if (m >= nout) continue;
            const uint32_t a01 = (uint32_t)acc[0][i] + ((uint32_t)acc[1][i] << 8);
            const uint32_t a23 = (uint32_t)acc[2][i] + ((uint32_t)acc[3][i] << 8);
            const uint32_t a45 = (uint32_t)acc[4][i] + ((uint32_t)acc[5][i] << 8);
            const uint32_t a67 = (uint32_t)acc[6][i] + ((uint32_t)acc[7][i] << 8);
            const uint64_t x = (uint64_t)a01 + ((uint64_t)a23 << 16);
            const uint64_t w = (uint64_t)a45 + ((uint64_t)a67 << 16);
            const uint64_t hi = (x >> 32) + w + (E >> 32), lo = (x & 0xFFFFFFFFull) + (uint32_t)E;
            uint64_t r = canon8w(mul_shoup_lazy4(hi, r32, r32p, q) + mul_shoup_lazy4(lo, 1, onep, q), q);
            uint64_t *o = out + m * out_ms + p;
            if (accumulate) r = add_mod(r, *o, q);
            *o = r;
        }
    }
}

}  // namespace

size_t weighted_sum_row_stride(size_t nin) { return (nin + WS_G - 1) / WS_G * WS_G; }

size_t weighted_sum_mx_bytes(size_t nout, size_t nin) {
    return ((nout + 15) / 16) * ((nin + 63) / 64) * 64 * 16;
}

void weighted_sum_mx_table(const int32_t *w, size_t nout, size_t nin, int8_t *tab) {
    const size_t nmt = (nout + 15) / 16, npass = (nin + 63) / 64;
    for (size_t pp = 0; pp < npass; pp++)
        for (size_t mt = 0; mt < nmt; mt++)
            for (int lane = 0; lane < 64; lane++)
                for (int b = 0; b < 16; b++) {
                    const size_t m = mt * 16 + lane % 16, j = pp * 64 + (lane / 16) * 16 + b;
                    tab[((pp * nmt + mt) * 64 + lane) * 16 + b] =
                        (int8_t)(m < nout && j < nin ? w[m * nin + j] : 0);
                }
}

hipError_t launch_weighted_sum_mx(const DevCtx &c, const uint64_t *in, size_t nin, const void *tab, size_t nout,
                                  uint64_t *out, hipStream_t s) {
    const size_t W = (size_t)2 * c.k * c.n;
    const size_t nmt = (nout + 15) / 16, npass = (nin + 63) / 64;
    const size_t nbx = (W + 16 * WSX_WAVES - 1) / (16 * WSX_WAVES);
    size_t gy = (16384 / WSX_WAVES + nbx - 1) / nbx;  // about 16384 waves in all
    if (gy > nmt) gy = nmt;
    if (gy > 65535) gy = 65535;
    if (gy < 1) gy = 1;
    const ws_v4i *wt = (const ws_v4i *)tab;
    for (size_t pp = 0; pp < npass; pp++) {
        const int nj = (int)(nin - pp * 64 < 64 ? nin - pp * 64 : 64);
        hipLaunchKernelGGL(k_weighted_sum_mx, dim3((unsigned)nbx, (unsigned)gy), dim3(64 * WSX_WAVES), 0, s, c,
                           in + pp * 64 * W, W, nj, wt + pp * nmt * 64, (int)nmt, nout, out, W, pp > 0 ? 1 : 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_weighted_sum(const DevCtx &c, const uint64_t *in, size_t nin, const int32_t *w, size_t nout,
                               uint64_t *out, hipStream_t s) {
    const size_t W = (size_t)2 * c.k * c.n;
    return launch_weighted_sum_items(c, in, W, 0, nin, 0, w, nout, out, W, 0, 1, s);
}

hipError_t launch_weighted_sum_items(const DevCtx &c, const uint64_t *in, size_t in_js, size_t in_is, size_t nin,
                                     int one_first, const int32_t *w, size_t nout, uint64_t *out, size_t out_ms,
                                     size_t out_is, size_t items, hipStream_t s) {
    const size_t W = (size_t)2 * c.k * c.n;
    const size_t wstride = weighted_sum_row_stride(nin);
    const dim3 grid((unsigned)((W + 255) / 256), (unsigned)((nout + WS_M - 1) / WS_M), (unsigned)items);
    for (size_t j0 = 0; j0 < nin; j0 += WS_J) {
        const int nj = (int)(nin - j0 < (size_t)WS_J ? nin - j0 : (size_t)WS_J);
        const int first = j0 == 0 ? one_first : 0;
        const uint64_t *src = in + (j0 - (j0 ? (size_t)one_first : 0)) * in_js;
        hipLaunchKernelGGL(k_weighted_sum, grid, dim3(256), 0, s, c, src, in_js, in_is, nj, first, w + j0,
                           (int)wstride, nout, out, out_ms, out_is, j0 > 0 ? 1 : 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
