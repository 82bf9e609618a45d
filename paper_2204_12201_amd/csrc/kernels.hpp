// Kernel launch interface shared by the host code and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tables.hpp"

struct Tw;

// Everything a kernel needs to know about the context, passed by value.
struct DevCtx {
    int n, L, k, kp, K;
    uint64_t t;
    const PrimeConst *pc;   // [K]
    const Tw *tw;           // [K][n] forward twiddles psi^bitrev(i)
    const Tw *itw;          // [K][n] inverse twiddles psi^-bitrev(i)
    const ConvConst *cc;
    const MrcConst *mrc_q;  // basis Q -> targets P (and t in the last slot)
    const MrcConst *mrc_p;  // basis P -> targets Q
    unsigned long long *fallback;  // count of coefficients that took the exact path
    int lazy_q;             // every Q prime below 2^64 / (4 (L + 1)) and 2^59: lazy key switching
    int lazy_all;           // every prime of Q and P below 2^64 / (4 (L + 1)): lazy transforms
    uint64_t lazy_limbs;    // bit l: prime l (Q then P) below 2^64 / (4 (L + 1))
    int digit_raw;          // every Q prime below 4 min(Q): digits enter the lazy transforms as they are
    const ConvMx *mx;       // matrix-core base conversion tables, or null (vector ALU conversions)
};

// Kernel kinds (timing and profiling names).
enum KernelKind {
    KK_LIFT = 0,
    KK_SQUARE_TENSOR,
    KK_SCALE,
    KK_RELIN_FUSED,
    KK_NTT_ROWS,
    KK_ELEMENTWISE,
    KK_BRIDGE,
    KK_MISC,
    KK_MUL_TENSOR,
    KK_FWD_EXT,
    KK_TENSOR_INTT,
    KK_PASS0_VALU,
    KK_PASS0_MFMA,
    KK_COUNT
};

// Row transform modes of launch_ntt_rows.
enum NttMode {
    NTT_FWD = 0,         // natural -> bit-reversed positions, canonical
    NTT_INV = 1,         // inverse, times n^-1, canonical
    NTT_INV_MONT = 2,    // inverse, times n^-1 2^64 (after Montgomery products)
    NTT_FWD_NINVM = 3    // forward, then times n^-1 2^64 (relinearization key form)
};

// ---- transforms (kernels_ntt.hip) ----
hipError_t launch_ntt_rows(const DevCtx &c, uint64_t *data, size_t nrows, int kmod, int limb_off,
                           int mode, hipStream_t s);
// Forward transforms of the extended inputs: rows (item, poly, limb) with the
// Q limbs read from a (polys 0,1) / b (polys 2,3) and the P limbs read from E.
hipError_t launch_fwd_ext(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *E,
                          int npoly, size_t items, hipStream_t s);
hipError_t launch_tensor_intt(const DevCtx &c, const uint64_t *E, uint64_t *Dt, bool square,
                              size_t items, hipStream_t s);
// Squaring: forward transforms of a0, a1 (P limbs from E) and the three
// inverse-transformed tensor components, one workgroup per (limb, item).
hipError_t launch_mul_tensor(const DevCtx &c, const uint64_t *a, const uint64_t *b, const uint64_t *E,
                             uint64_t *Dt, size_t items, hipStream_t s);
// Products of two transformed operands: item z multiplies input (item0 + z)
// mod na of Ahat by entry item0 + z of Bhat (both [.][2][K][n], transform
// domain, canonical); tensor into Dt.
hipError_t launch_mul_tensor_pre2(const DevCtx &c, const uint64_t *Ahat, int na, size_t item0, const uint64_t *Bhat,
                                  uint64_t *Dt, size_t items, hipStream_t s);
hipError_t launch_square_tensor(const DevCtx &c, const uint64_t *a, const uint64_t *E, uint64_t *Dt,
                                size_t items, hipStream_t s);
// Key switching: out[item][l] += sum_i [C2]_{q_i} rlk_i[l] for l = 0, 1.
hipError_t launch_relin_fused(const DevCtx &c, const uint64_t *C2, const uint64_t *rlk, uint64_t *out,
                              size_t items, hipStream_t s);
// One part of the persistent key switching over several ring sizes (n = 4096,
// 8192 or 16384): `items` products of context c; wg_tasks = ceil(items k /
// (16384 / n)) queue entries; kmagic = ceil(2^32 / k).
struct RelinPart {
    DevCtx c;
    const uint64_t *C2, *rlk;
    uint64_t *out;
    uint32_t items, wg_tasks, kmagic;
};
constexpr int kRelinQueueParts = 4;
struct RelinQueue {
    RelinPart part[kRelinQueueParts];
    int nparts;
};
// The key switching of every part of Q in one launch of persistent
// workgroups (1024 threads; as many as the chip holds, at most `tasks`, the
// sum of the parts' wg_tasks) taking tasks from the counter `queue` (cleared
// on the stream first).  Every part has lazy_q == lazy and digit_raw == raw.
hipError_t launch_relin_persist(const RelinQueue &Q, int lazy, int raw, unsigned int *queue, size_t tasks,
                                hipStream_t s);


// ---- base conversions and elementwise (kernels_conv.hip) ----
hipError_t launch_lift(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *E, int npoly,
                       size_t items, hipStream_t s);
hipError_t launch_scale(const DevCtx &c, const uint64_t *Dt, uint64_t *out, uint64_t *C2,
                        size_t items, hipStream_t s, int comp0 = 0, int ncomp = 3);
// Shared first squaring of the bridge chains (kernels_conv.hip, k_bridge_gamma
// and k_scale_chain): per-chain constant-coefficient corrections, then the
// chains' components 0 and 1 from the inputs' tensor plus key-switching output.
hipError_t launch_bridge_gamma(const DevCtx &c, const uint64_t *x, const uint64_t *E, uint64_t *gam,
                               size_t chains, int tcount, int c0, hipStream_t s);
hipError_t launch_scale_chain(const DevCtx &c, const uint64_t *Dt, const uint64_t *x, const uint64_t *E,
                              const uint64_t *gam, const uint64_t *R, uint64_t *y, size_t chains, int tcount,
                              hipStream_t s);
hipError_t launch_decrypt_scale(const DevCtx &c, const uint64_t *X, uint64_t *pt, size_t count,
                                hipStream_t s);
// op: 0 add, 1 sub, 2 neg (b unused)
hipError_t launch_addsub(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *out,
                         size_t nrows, int op, hipStream_t s);
// out = a with c0's constant coefficient +/- Delta*cval (sign: +1 / -1)
hipError_t launch_plain_const(const DevCtx &c, const uint64_t *a, uint64_t *out, size_t count,
                              uint64_t cval, int sign, hipStream_t s);
// small signed integers (int8 when is8, else int32) -> residues, rows [count][k][n]
hipError_t launch_small_to_rns(const DevCtx &c, const void *v, int is8, uint64_t *out, size_t count,
                               hipStream_t s);
// out = a * b * 2^-64 (canonical), rows with limb = row % k; bcast: b has k rows only
hipError_t launch_pointwise_mont(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *out,
                                 size_t nrows, int bcast, hipStream_t s);
// out_j = -(prod_j + e_j) + [j == digit] s2_j  (digit < 0: no s^2 term)
hipError_t launch_key_b(const DevCtx &c, const uint64_t *prod, const uint64_t *e_rns,
                        const uint64_t *s2, int digit, uint64_t *out, hipStream_t s);
// ct[j] = (prod[0][j] + e[j][0] + Delta m_j, prod[1][j] + e[j][1]); prod [2][count][k][n]
hipError_t launch_encrypt_finish(const DevCtx &c, const uint64_t *prod, const int32_t *e,
                                 const uint64_t *pt, uint64_t *ct, size_t count, hipStream_t s);
hipError_t launch_bridge_combine(const DevCtx &c, const uint64_t *y, uint64_t *bits, uint64_t *eq,
                                 size_t count, int tcount, int nbits, int c0, hipStream_t s);
// out = sum_b 2^b bits[b] by Horner; signed_top: the leading bit weighs -2^(nbits-1)
hipError_t launch_horner(const DevCtx &c, const uint64_t *bits, int nbits, uint64_t *out,
                         size_t count, int signed_top, hipStream_t s);
// flag[0] |= 1 if some word of rows [nrows][n] (limb = row % kmod + off) is >= its prime
hipError_t launch_validate(const DevCtx &c, const uint64_t *a, size_t nrows, int kmod, int off,
                           unsigned int *flag, hipStream_t s);

// ---- first transform pass on the matrix cores (kernels_mfma.hip) ----
// Levels 0..3 of the forward transform of rows [nrows][n] (limb = row % kmod +
// limb_off), applied `reps` times, in place, canonical.  method 0: vector ALU;
// 1: int8 matrix cores with the per-limb operand table Wt (16 KiB per limb);
// n >= 1024.
hipError_t launch_pass0(const DevCtx &c, int method, const void *Wt, uint64_t *data, size_t nrows, int kmod,
                        int limb_off, int reps, hipStream_t s);

// ---- integer-weighted sums (kernels_lin.hip) ----
// Matrix-core variant for weights in [-127, 127]: the operand table (bytes
// weighted_sum_mx_bytes) built on the host by weighted_sum_mx_table from the
// weights [nout][nin], then out[m] = sum_j w[m][j] in[j] (in, out: [.][2][k][n]).
size_t weighted_sum_mx_bytes(size_t nout, size_t nin);
void weighted_sum_mx_table(const int32_t *w, size_t nout, size_t nin, int8_t *tab);
hipError_t launch_weighted_sum_mx(const DevCtx &c, const uint64_t *in, size_t nin, const void *tab, size_t nout,
                                  uint64_t *out, hipStream_t s);
// Row stride (in weights) of the device weight matrix: rows padded with zeros.
size_t weighted_sum_row_stride(size_t nin);
// out[m] = sum_j w[m][j] in[j] for the padded device matrix w [nout][stride].
hipError_t launch_weighted_sum(const DevCtx &c, const uint64_t *in, size_t nin, const int32_t *w, size_t nout,
                               uint64_t *out, hipStream_t s);
// The same over `items` independent sets with one weight matrix: set z reads
// input j at in + z in_is + j in_js and writes output m at out + z out_is +
// m out_ms; one_first: input 0 is the noiseless encryption of 1 (not read)
// and input j >= 1 sits at index j - 1.
hipError_t launch_weighted_sum_items(const DevCtx &c, const uint64_t *in, size_t in_js, size_t in_is, size_t nin,
                                     int one_first, const int32_t *w, size_t nout, uint64_t *out, size_t out_ms,
                                     size_t out_is, size_t items, hipStream_t s);
