/*
 * fhe.h -- C ABI of the gfx950 BFV multiply+relinearize and p-ary bridge library.
 *
 * Scheme: BFV (Fan-Vercauteren 2012, the BFV citation of the paper's
 * introduction) in residue-number-system form.  The paper runs BFV through
 * SEAL and fixes nothing about its internals; the operations below compute the
 * textbook FV12 results exactly, so every output word is uniquely defined:
 *
 *   multiply      C_j = round(t D_j / q) mod q, D the exact integer tensor of the
 *                 centred lifts (D0 = A0 B0, D1 = A0 B1 + A1 B0, D2 = A1 B1);
 *   relinearize   c'_l = C_l + sum_i [C2]_{q_i} rlk_i[l]  (mod q), one digit per
 *                 RNS prime, rlk_i = (-(a_i s + e_i) + eps_i s^2, a_i);
 *   bridge        the paper's conversion SecureMod -> SecureUint (Section 3.2.3,
 *                 its equation with Fermat equality tests 1 - (x - c)^(t-1), its
 *                 pow listing for the power): eq_c for every c in [0, t), then
 *                 bit j = sum over c in [1, t) with bit j of c set of eq_c.
 *
 * Data layout (all words uint64, little endian, canonical residues in [0, q_i)):
 *   polynomial   [k][n]        limb-major: limb i is n contiguous coefficients
 *   ciphertext   [2][k][n]     (c0, c1);   a batch is [count][2][k][n]
 *   public key   [2][k][n]     coefficient form
 *   relin key    internal, fhe_rlk_words() words, produced only by fhe_keygen or
 *                fhe_rlk_import (transform domain, resident on the device)
 *   plaintext    [n] coefficients in [0, t) (host)
 *
 * Ownership: the caller allocates every buffer (device buffers with its own
 * allocator, e.g. torch); the library never keeps a pointer after a call
 * returns.  Device-side tables belong to the context.  Workspace ("ws") is
 * caller-provided device memory of at least fhe_workspace_bytes() bytes.
 *
 * Streams: every call enqueues its kernels on `stream` (NULL = default stream)
 * and returns without synchronising, except the calls that return host data
 * (fhe_decrypt) which synchronise the stream.  Argument and shape errors are
 * returned synchronously before anything is enqueued; launch failures return
 * FHE_EDEVICE; a fault of a kernel already enqueued surfaces as FHE_EDEVICE
 * from fhe_sync (or from the next call that synchronises).  A context is not
 * thread safe: one context per host thread.
 *
 * Aliasing: where a call documents it, `out` may be exactly `a` or `b`
 * (in place).  Any other overlap between an output and an input, or between
 * the workspace and an operand of the multiply calls, is rejected with
 * FHE_EINVAL before anything is enqueued (the checks compare address ranges
 * on the host).
 *
 * Inputs must be canonical residues.  With the environment variable
 * FHE_VALIDATE=1 the elementwise, multiply and bridge calls check this first
 * and return FHE_ENONCANON.
 */
#ifndef FHE_H
#define FHE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FHE_OK = 0,
    FHE_EINVAL = -1,       /* null pointer, bad count, bad op code, overlap */
    FHE_EPARAM = -2,       /* parameter set rejected by fhe_ctx_create */
    FHE_ENOMEM = -3,       /* device allocation of context tables failed */
    FHE_EDEVICE = -4,      /* HIP error (launch failure, bad device) */
    FHE_ESHAPE = -5,       /* size arguments inconsistent with the context */
    FHE_ENONCANON = -6,    /* FHE_VALIDATE: an input word is not < its prime */
    FHE_EUNSUPPORTED = -7, /* operation not defined for this parameter set */
    FHE_EWORKSPACE = -8    /* workspace smaller than fhe_workspace_bytes() */
} fhe_status;

enum { FHE_ENC_SLOTS = 0, FHE_ENC_COEFF = 1 };

/* op codes for fhe_workspace_bytes */
enum {
    FHE_OP_MUL_RELIN = 1,
    FHE_OP_SQUARE_RELIN = 2,
    FHE_OP_BRIDGE = 3,
    FHE_OP_KEYGEN = 4,
    FHE_OP_ENCRYPT = 5,
    FHE_OP_DECRYPT = 6,
    FHE_OP_RLK_IMPORT = 7,
    FHE_OP_WEIGHTED_SUM = 8, /* count = nout * nin weights */
    FHE_OP_GATE = 9,         /* count = ciphertexts per operand */
    FHE_OP_COMPARE = 10,     /* count = pairs of bit vectors */
    FHE_OP_ARGMAX = 11,      /* count = score sets */
    FHE_OP_MOD_TO_INT = 12,  /* count = inputs */
    FHE_OP_BRIDGE_POWERS = 13 /* count = inputs */
};

/* gates of fhe_gate */
enum {
    FHE_GATE_AND = 0,
    FHE_GATE_NAND = 1,
    FHE_GATE_OR = 2,
    FHE_GATE_NOR = 3,
    FHE_GATE_XOR = 4,
    FHE_GATE_XNOR = 5,
    FHE_GATE_NOT = 6,
    FHE_GATE_MUX = 7
};

typedef struct fhe_ctx fhe_ctx;

typedef struct {
    uint32_t n;        /* ring degree, power of two in [16, 16384] */
    uint32_t k;        /* number of RNS primes of q, 1..16 */
    uint64_t t;        /* plaintext modulus, 2 <= t < 2^62, gcd(t, q) = 1 */
    const uint64_t *q; /* host array of k distinct primes, q_i = 1 mod 2n, q_i < 2^61 */
    uint32_t encoding; /* FHE_ENC_SLOTS (needs t prime, t = 1 mod 2n) or FHE_ENC_COEFF */
} fhe_params;

/* Validate parameters and build the context's device tables on `hip_device`.
 * Rejects (FHE_EPARAM) n not a power of two in [16, 16384], k outside 1..16,
 * composite / repeated / too large q_i, q_i != 1 mod 2n, gcd(t, q) != 1, and
 * slot encoding without a prime t = 1 mod 2n.  Parameter checks run before any
 * device call.  *out is set only on FHE_OK. */
fhe_status fhe_ctx_create(const fhe_params *params, int hip_device, fhe_ctx **out);
void fhe_ctx_destroy(fhe_ctx *ctx);

size_t fhe_ct_words(const fhe_ctx *ctx);  /* 2 k n */
size_t fhe_pk_words(const fhe_ctx *ctx);  /* 2 k n */
size_t fhe_rlk_words(const fhe_ctx *ctx); /* 2 k^2 n (internal transform domain) */
/* Number of auxiliary primes the exact multiply extends q with (internal). */
uint32_t fhe_aux_primes(const fhe_ctx *ctx);

/* Device workspace, in bytes, for `op` on `count` items (ciphertext pairs for
 * multiply, inputs for the bridge, ciphertexts for encrypt/decrypt). */
size_t fhe_workspace_bytes(const fhe_ctx *ctx, int op, size_t count);

/* Cap on the number of products one multiply launch sequence processes; larger
 * counts run in chunks (workspace is sized for min(count, cap)).  0 restores
 * the default (about 8 GiB of workspace). */
fhe_status fhe_set_batch_limit(fhe_ctx *ctx, size_t max_items);

/* Launch-shape switch of the product pipeline: chunks of at least min_rows
 * (item, limb) workgroups take the fused transform kernel, smaller ones the
 * unfused kernels (square != 0: the squaring path, whose default is 0 =
 * always fused; products default to 128).  Same words either way. */
fhe_status fhe_set_fused_threshold(fhe_ctx *ctx, int square, size_t min_rows);

/* Where the base conversions of `multiply` (top of this file) run: the
 * centred lift of the inputs from q to the auxiliary basis P, and the
 * rounding of t D / q computed in P and brought back to q: method 0 on the
 * vector ALU (64-bit
 * multiply-accumulates), method 1 on the int8 matrix cores, as an exact
 * matrix product of balanced base-256 digits with int32 sums and one
 * Montgomery reduction per output.  Both give the same words (coefficients
 * whose floating estimate lies near a rounding boundary take the exact
 * mixed-radix path either way).  Method 1 needs at most 8 primes in q and in
 * P and every prime at least 2^20 (else FHE_EUNSUPPORTED); it is the default
 * where it applies.  With method 1, fhe_weighted_sum also runs on the matrix
 * cores when every weight lies in [-127, 127] (same words).  Drops the
 * context's squaring-chain graphs. */
fhe_status fhe_set_conv_method(fhe_ctx *ctx, int method);
/* The current method of fhe_set_conv_method (0 for a NULL context). */
int fhe_conv_method(const fhe_ctx *ctx);

/* ---------------------------------------------------------------- keys --- *
 * Key generation from explicit randomness (host arrays):
 *   s      int8[n]          secret key, entries in {-1, 0, 1}
 *   pk_a   uint64[k][n]     uniform residues (public-key mask)
 *   pk_e   int32[n]         public-key error
 *   rlk_a  uint64[k][k][n]  mask of relinearization digit i
 *   rlk_e  int32[k][n]      error of relinearization digit i
 * Writes pk (device, [2][k][n], coefficient form: pk0 = -(a s + e), pk1 = a) and
 * rlk (device, internal form).  ws: FHE_OP_KEYGEN bytes. */
fhe_status fhe_keygen(fhe_ctx *ctx, const int8_t *s, const uint64_t *pk_a, const int32_t *pk_e,
                      const uint64_t *rlk_a, const int32_t *rlk_e, uint64_t *pk_dev,
                      uint64_t *rlk_dev, void *ws, size_t ws_bytes, hipStream_t stream);

/* Convert a relinearization key given in coefficient form, device
 * uint64[k digits][2][k][n] (rlk_i = (b_i, a_i)), into the internal form used by
 * fhe_mul_relin.  ws: FHE_OP_RLK_IMPORT bytes. */
fhe_status fhe_rlk_import(fhe_ctx *ctx, const uint64_t *rlk_coeff_dev, uint64_t *rlk_dev,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------ encoding --- *
 * Host-side plaintext encoding of n values in [0, t).  Slots: m with
 * m(psi_t^(2j+1)) = vals[j] mod t, psi_t = g^((t-1)/2n) for g the smallest
 * primitive root of t (3 for t = 65537).  Coefficient: m = vals. */
fhe_status fhe_encode(const fhe_ctx *ctx, const uint64_t *vals, uint64_t *pt);
fhe_status fhe_decode(const fhe_ctx *ctx, const uint64_t *pt, uint64_t *vals);

/* ------------------------------------------------------ enc / dec -------- *
 * ct[j] = ([pk0 u_j + e_j[0] + Delta m_j]_q, [pk1 u_j + e_j[1]]_q), Delta = floor(q/t).
 *   pt   host uint64[count][n] plaintext polynomials, coefficients < t
 *   u    host int8[count][n] ternary; e host int32[count][2][n]
 *   ct   device uint64[count][2][k][n]. ws: FHE_OP_ENCRYPT bytes. */
fhe_status fhe_encrypt(fhe_ctx *ctx, const uint64_t *pk_dev, const uint64_t *pt, const int8_t *u,
                       const int32_t *e, uint64_t *ct_dev, size_t count, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/* pt[j] = [round(t [c0 + c1 s]_q / q)]_t per coefficient (exact).  s host
 * int8[n]; pt host uint64[count][n].  Synchronises `stream`.
 * ws: FHE_OP_DECRYPT bytes. */
fhe_status fhe_decrypt(fhe_ctx *ctx, const int8_t *s, const uint64_t *ct_dev, uint64_t *pt,
                       size_t count, void *ws, size_t ws_bytes, hipStream_t stream);

/* --------------------------------------------------------- elementwise --- *
 * Batches of `count` ciphertexts, device pointers, modulo each q_i.
 * add_plain_const / sub_plain_const add / subtract Delta*c to the constant
 * coefficient of c0 (the encoding of the constant polynomial c, 0 <= c < t). */
fhe_status fhe_add(fhe_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t count,
                   hipStream_t stream);
fhe_status fhe_sub(fhe_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t count,
                   hipStream_t stream);
fhe_status fhe_neg(fhe_ctx *ctx, const uint64_t *a, uint64_t *out, size_t count, hipStream_t stream);
fhe_status fhe_add_plain_const(fhe_ctx *ctx, const uint64_t *a, uint64_t c, uint64_t *out,
                               size_t count, hipStream_t stream);
fhe_status fhe_sub_plain_const(fhe_ctx *ctx, const uint64_t *a, uint64_t c, uint64_t *out,
                               size_t count, hipStream_t stream);

/* ----------------------------------------------------------- hot path ---- *
 * out[j] = relinearize(multiply(a[j], b[j])) for j < count, the FV12 product
 * and one-digit-per-prime key switching (see the top of this file).
 * a, b, out: device [count][2][k][n]; rlk from fhe_keygen / fhe_rlk_import.
 * a == b (same pointer) selects the squaring kernels (same result).
 * count == 0 is a no-op.  ws: FHE_OP_MUL_RELIN (or FHE_OP_SQUARE_RELIN when
 * a == b) bytes for count. */
fhe_status fhe_mul_relin(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *a,
                         const uint64_t *b, uint64_t *out, size_t count, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the words
 * of fhe_mul_relin(ctx, rlk_dev, a, b, out, count, ...) without a caller
 * workspace.  The workspace is a static device array of FHE_STATIC_WS_BYTES
 * bytes inside the library, one per device, held from the first context on
 * that device until the process ends; the call allocates nothing (no
 * hipMalloc, no events: per-launch timing is skipped for it).  A call needs
 * fhe_workspace_bytes(ctx, FHE_OP_MUL_RELIN or FHE_OP_SQUARE_RELIN when
 * a == b, count) bytes, i.e. min(count, batch limit) products' worth; more
 * than FHE_STATIC_WS_BYTES returns FHE_EWORKSPACE before anything is enqueued
 * (split the call or lower fhe_set_batch_limit).  Every call on a device, from
 * any context or stream, uses the same array: calls that overlap in time on
 * one device race and give undefined words; serialise them (one stream, or
 * events).  Nothing in the array needs to start at zero: each call writes the
 * part it reads.  Aliasing and the other arguments as for fhe_mul_relin. */
#define FHE_STATIC_WS_BYTES (64u << 20)
fhe_status fhe_mul_relin_static(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *a,
                                const uint64_t *b, uint64_t *out, size_t count, hipStream_t stream);

/* Autotuner of the product pipeline's launch shape for this context: times
 * fhe_mul_relin(a, b, out) for count items (a == b: the squaring path) with
 * chunk caps count, count/2, count/4 (never above the current cap) and with
 * the fused transform kernel or the unfused ones, three timed runs each after
 * a warm-up on `stream` (synchronous), and keeps the fastest: the chunk cap
 * (as fhe_set_batch_limit) and the fused/unfused threshold of that product
 * kind, set so that chunks of the chosen size take the chosen path.  Results
 * of every call are the same words whatever the choice; only speed changes.
 * *chunk and *fused (may be NULL) receive the choice.  out is overwritten.
 * ws: FHE_OP_MUL_RELIN (FHE_OP_SQUARE_RELIN when a == b) bytes for count. */
fhe_status fhe_autotune_mul_relin(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *a,
                                  const uint64_t *b, uint64_t *out, size_t count, void *ws,
                                  size_t ws_bytes, hipStream_t stream, size_t *chunk, int *fused);

/* Several product batches, possibly of different contexts (ring sizes,
 * primes), in one call: part i computes what fhe_mul_relin(parts[i].ctx, ...)
 * computes.  Each part runs on its context's own stream (created on first use,
 * default priority), which first waits for the work already queued on `stream`;
 * `stream` then waits for all parts, so parts of different contexts overlap on
 * the device.  The call returns once everything is enqueued.  Since parts run
 * concurrently, an output or workspace range of one part must not overlap the
 * inputs, output or workspace of any other part (FHE_EINVAL, checked before
 * anything is enqueued); parts of one context run one after the other.  If an
 * error stops the call after some parts were enqueued, `stream` still waits
 * for those parts before the error is returned.  All contexts must be on the
 * current device.  Arguments as for fhe_mul_relin (each ws sized for its
 * part). */
typedef struct {
    fhe_ctx *ctx;
    const uint64_t *rlk_dev, *a, *b;
    uint64_t *out;
    size_t count;
    void *ws;
    size_t ws_bytes;
} fhe_mul_part;
fhe_status fhe_mul_relin_multi(const fhe_mul_part *parts, size_t nparts, hipStream_t stream);

/* Key switching of fhe_mul_relin_multi in one persistent launch (same words).
 * When the call's first context allows it (enable != 0; off by default), at
 * most 4 parts with products, of at least two of the ring sizes 4096, 8192
 * and 16384, each fitting one chunk of its context's batch limit and all with
 * the same key-switching variant (every configured parameter set has it): the
 * parts run up to the third tensor component on their streams, then `stream`
 * waits for all of them and one launch of resident workgroups takes
 * (ciphertext, limb, ring size) tasks from a device counter (one row of
 * 16384, two of 8192 or four of 4096 per workgroup task, the largest ring
 * first) until every part is key-switched.  Other calls, or enable == 0,
 * key-switch each part on its own stream. */
fhe_status fhe_set_multi_persistent(fhe_ctx *ctx, int enable);

/* Autotuner of fhe_mul_relin_multi's key switching for these parts: where the
 * persistent launch applies, times the call (synchronously, on `stream`) with
 * each part key-switched on its own stream and with the persistent launch,
 * three runs each after a warm-up, and keeps the faster in parts[0].ctx (as
 * fhe_set_multi_persistent); elsewhere it keeps the per-stream mode.  The
 * parts' outputs are overwritten (same words either way).  *persistent (may be
 * NULL) receives the choice. */
fhe_status fhe_autotune_mul_relin_multi(const fhe_mul_part *parts, size_t nparts, hipStream_t stream,
                                        int *persistent);

/* Repeated squaring in place: x[j] <- x[j]^(2^depth), i.e. depth calls of
 * fhe_mul_relin(x, x, x) (same words), for j < count.  graph != 0 records the
 * launch sequence once into a HIP graph kept by the context, keyed by
 * (rlk_dev, x, ws, ws_bytes, count, depth) and the launch shape it recorded
 * (batch limit, fused threshold of squarings), and replays it on later calls
 * with the same key.  fhe_set_batch_limit, fhe_set_fused_threshold and
 * fhe_autotune_mul_relin drop every recorded graph; at most 16 are kept
 * (the oldest is dropped first).  A graph holds the buffers' addresses: they
 * must stay allocated while the graph is kept.  Per-launch timing or
 * validation makes the call run eagerly.  ws: FHE_OP_SQUARE_RELIN bytes for
 * count. */
fhe_status fhe_square_chain(fhe_ctx *ctx, const uint64_t *rlk_dev, uint64_t *x, uint32_t depth,
                            size_t count, void *ws, size_t ws_bytes, int graph, hipStream_t stream);

/* The paper's SecureMod -> SecureUint conversion for prime t (Section 3.2.3):
 * for each input x[j] (device [count][2][k][n]) and each c in [0, t):
 *   y = x - c (sub_plain_const), y = y^(t-1) by repeated squaring
 *   (mul_relin, t-1 a power of two: log2(t-1) squarings), eq_c = 1 - y;
 * bits[j][b] = sum over c in [1, t) with bit b of c set of eq_c, b < nbits.
 *   bits  device [count][nbits][2][k][n]
 *   eq    device [count][t][2][k][n], or NULL to skip writing the eq_c
 * Requires coefficient encoding, t prime, t - 1 a power of two, and
 * 2^nbits >= t (else FHE_EUNSUPPORTED / FHE_EINVAL).  Inputs should encrypt
 * constant polynomials (the equality test is coefficient-wise only for
 * those); the words are defined for any input.  With eq == NULL the test
 * c = 0, which enters no bit, is not evaluated (same bits).
 * ws: FHE_OP_BRIDGE bytes. */
fhe_status fhe_bridge_to_bits(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *x,
                              uint32_t nbits, uint64_t *bits, uint64_t *eq, size_t count,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* ----------------------------------------------- modular linear stage --- *
 * Integer-weighted sums of ciphertexts, word by word modulo each q_i:
 *   out[m] = sum_{j < nin} w[m * nin + j] * in[j],   m < nout,
 * the modular stage of the paper's genotype-imputation case study (Section
 * 4.4, p-Impute with bridging: per-class scores as weighted sums of encrypted
 * genotypes, before the bridge).  A weighted sum of encryptions encrypts the
 * same weighted sum of the plaintexts modulo t (noise scaled by sum |w|).
 *   in   device uint64 [nin][2][k][n]      out device uint64 [nout][2][k][n]
 *   w    host int32 [nout][nin]; every row must have sum_j |w| < 2^30
 *        (FHE_EINVAL otherwise); copied into ws before the call returns
 * out must not overlap in (FHE_EINVAL).  nout == 0 is a no-op; nin == 0
 * writes zero ciphertexts.  ws: FHE_OP_WEIGHTED_SUM bytes for nout * nin. */
fhe_status fhe_weighted_sum(fhe_ctx *ctx, const uint64_t *in, size_t nin, const int32_t *w,
                            size_t nout, uint64_t *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------- bit-level side ----- *
 * Homomorphic gates on ciphertexts of bits (Section 3.1, the logic-gate
 * expressions over {0, 1}; any t), batched over count ciphertexts per operand,
 * evaluated exactly in this order (mul = fhe_mul_relin, 1 = add_plain_const 1):
 *   AND  p = a b                     NAND  1 - a b = add_plain(neg(p), 1)
 *   OR   (a + b) - a b               NOR   add_plain(neg(OR), 1)
 *   XOR  ((a + b) - a b) - a b       XNOR  add_plain(neg(XOR), 1)
 *   NOT  add_plain(neg(a), 1)        MUX   a (b - c) + c   (a ? b : c)
 * a, b, c, out: device [count][2][k][n]; b is unused by NOT, c is read by MUX
 * only (NULL allowed where unused).  out may equal an input.
 * ws: FHE_OP_GATE bytes for count. */
fhe_status fhe_gate(fhe_ctx *ctx, const uint64_t *rlk_dev, int gate, const uint64_t *a,
                    const uint64_t *b, const uint64_t *c, uint64_t *out, size_t count, void *ws,
                    size_t ws_bytes, hipStream_t stream);

/* Encrypted comparison of unsigned bit vectors (Section 3.1: comparisons are
 * built from the gates as standard combinational circuits), least significant bit
 * first as fhe_bridge_to_bits writes them:
 *   out[j] = [a_j < b_j] for a_j = sum_i 2^i a[j][i], b_j likewise.
 * Circuit, per bit i: p_i = a_i b_i; d_i = b_i - p_i (= NOT a_i AND b_i);
 * e_i = 1 - ((a_i + b_i) - p_i - p_i) (XNOR); lt = d_0, then for i >= 1
 * lt = e_i (lt - d_i) + d_i (MUX(e_i, lt, d_i)).  Multiplicative depth nbits.
 *   a, b device [count][nbits][2][k][n];  out device [count][2][k][n]
 * nbits >= 1.  ws: FHE_OP_COMPARE bytes for count. */
fhe_status fhe_less_than(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *a, const uint64_t *b,
                         uint32_t nbits, uint64_t *out, size_t count, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* One-hot argmax of ncls encrypted unsigned scores per set, ties to the lower
 * class: for every pair a < b (a ascending, then b) l = [s_a < s_b]
 * (fhe_less_than); out_a takes the factor 1 - l, out_b the factor l; a class's
 * first factor is copied, later ones multiplied in (fhe_mul_relin).
 *   scores device [ncls][count][nbits][2][k][n];  out device [ncls][count][2][k][n]
 * 2 <= ncls <= 16.  ws: FHE_OP_ARGMAX bytes for count. */
fhe_status fhe_argmax(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *scores, uint32_t ncls,
                      uint32_t nbits, uint64_t *out, size_t count, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* The paper's signed casts.
 * SecureInt -> SecureMod (Section 3.2.2): out[j] encrypts the two's complement
 * value sum_{b < nbits-1} 2^b bits[j][b] - 2^(nbits-1) bits[j][nbits-1] modulo
 * t, i.e. the paper's t - 2^s + sum 2^b x_b for a negative input; evaluated
 * linearly (Horner with the leading bit negated: no multiplication, where the
 * paper's selection spends two).  bits device [count][nbits][2][k][n]; out
 * device [count][2][k][n]; needs 2^nbits >= t for the value to fit. */
fhe_status fhe_int_to_mod(fhe_ctx *ctx, const uint64_t *bits, uint32_t nbits, uint64_t *out, size_t count,
                          hipStream_t stream);

/* SecureMod -> SecureInt (Section 3.2.4, its equation): X = the unsigned bits
 * of x (fhe_bridge_to_bits), then the sign adjustment, evaluated as
 *   A = X + (2^s - t) in s-bit arithmetic, a ripple-carry adder of the gates
 *       over the constant's bits (bit 0: A_i = X_i XOR carry, carry = X_i AND
 *       carry; bit 1: A_i = XNOR, carry = OR; no product while the carry is
 *       known to be zero),
 *   Y_i = MUX(X_{s-1}, A_i, X_i) = X_{s-1} (A_i - X_i) + X_i,
 * so x >= 2^(s-1) (the values the paper reads as negative) becomes x - t in
 * two's complement.  x device [count][2][k][n]; bits device
 * [count][nbits][2][k][n] (least significant first).  Preconditions of
 * fhe_bridge_to_bits.  ws: FHE_OP_MOD_TO_INT bytes for count. */
fhe_status fhe_mod_to_int(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *x, uint32_t nbits,
                          uint64_t *bits, size_t count, void *ws, size_t ws_bytes, hipStream_t stream);

/* The same bits as fhe_bridge_to_bits, evaluated from the powers of x instead
 * of one squaring chain per test: the t tests (x - c)^(t-1) share
 * x^1..x^(t-1), computed once per input by a least-depth product tree
 * (x^(h+r) = x^h x^r, h the largest power of two below h + r; t - 2
 * products, depth ceil(log2(t-1))), and each bit is one integer-weighted sum
 * of [1, x, ..., x^(t-1)] with the weights of the binomial expansion of
 * sum over c in [1, t) with bit b of c set of 1 - (x - c)^(t-1) (centred mod
 * t; 1 = the noiseless encryption (Delta, 0)).  Decrypts to the same bits
 * with 15 instead of 68 products at t = 17; the words differ from
 * fhe_bridge_to_bits (another circuit).  Requires coefficient encoding, t
 * prime, 3 <= t <= 257, 2^nbits >= t.  x device [count][2][k][n]; bits device
 * [count][nbits][2][k][n].  ws: FHE_OP_BRIDGE_POWERS bytes for count. */
fhe_status fhe_bridge_to_bits_powers(fhe_ctx *ctx, const uint64_t *rlk_dev, const uint64_t *x, uint32_t nbits,
                                     uint64_t *bits, size_t count, void *ws, size_t ws_bytes,
                                     hipStream_t stream);

/* The paper's SecureUint -> SecureMod cast (Section 3.2.1, Horner):
 * out[j] = sum_b 2^b bits[j][b], evaluated as r = bit_{nbits-1}; r = r + r + bit_b.
 * bits device [count][nbits][2][k][n]; out device [count][2][k][n]. */
fhe_status fhe_bits_to_mod(fhe_ctx *ctx, const uint64_t *bits, uint32_t nbits, uint64_t *out,
                           size_t count, hipStream_t stream);

/* ---------------------------------------------------- kernel-level test -- *
 * Negacyclic transform of `count` polynomials [count][k][n] in place, limb i
 * modulo q_i with psi_i = x^((q_i-1)/2n) for the smallest x >= 2 giving
 * psi_i^n = -1.  Forward: position bitrev(j) receives sum_i a_i psi^(i(2j+1)).
 * Inverse (inverse != 0) undoes it.  Outputs canonical. */
fhe_status fhe_ntt(fhe_ctx *ctx, int inverse, uint64_t *polys, size_t count, hipStream_t stream);

/* The first radix-16 pass of fhe_ntt's forward transform (butterfly levels
 * 0..3), alone, in place on `count` polynomials [count][k][n] of canonical
 * residues: every group of 16 residues a[g + e n/16] (e = 0..15) becomes
 * y_j = sum_e M_i[j][e] a[g + e n/16] mod q_i at position g + j n/16, with
 * M_i the 16 x 16 matrix of those four levels of the negacyclic transform
 * (y_j = sum_e a[g + e n/16] zeta^(e (2 bitrev4(j) + 1)), zeta = psi_i^(n/16));
 * applied `reps` times (1..1024) on the chip before the store (M_i^reps: the
 * compute rate of the pass without its memory traffic); outputs canonical.  method 0 computes it with the vector ALU butterflies of
 * the transforms, method 1 as an exact matrix product on the int8 matrix cores
 * (7-bit limbs, int32 sums; same words).  A kernel-level comparison of the two
 * ways to run a transform pass (the transforms of the product pipeline move to
 * the matrix cores only if they are faster there); n >= 1024, and for method
 * 1 every q_i < 2^55 (else FHE_EUNSUPPORTED).  The first method-1 call builds
 * the context's operand tables (16 KiB per prime of q). */
fhe_status fhe_ntt_pass0(fhe_ctx *ctx, int method, uint32_t reps, uint64_t *polys, size_t count,
                         hipStream_t stream);

/* ------------------------------------------------------------- timing ---- *
 * When enabled, every kernel launch is bracketed by HIP events on its stream
 * and its duration is accumulated per kernel kind (costs one event pair per
 * launch; off by default).  fhe_kernel_stats synchronises the events and
 * returns the total milliseconds and launch count of kernel kind `kind`
 * (see fhe_kernel_name; kinds are 0 .. fhe_kernel_kinds()-1). */
fhe_status fhe_set_timing(fhe_ctx *ctx, int enable);
int fhe_kernel_kinds(void);
const char *fhe_kernel_name(int kind);
fhe_status fhe_kernel_stats(fhe_ctx *ctx, int kind, double *total_ms, uint64_t *launches);
fhe_status fhe_reset_kernel_stats(fhe_ctx *ctx);

/* Number of coefficients that took the exact (multi-word) path in the base
 * conversions since the context was created (diagnostic; synchronises). */
fhe_status fhe_fallback_count(fhe_ctx *ctx, uint64_t *count);

/* Waits for all work enqueued on `stream` and returns FHE_EDEVICE if any of
 * it failed on the device (the asynchronous errors of the calls above). */
fhe_status fhe_sync(fhe_ctx *ctx, hipStream_t stream);

const char *fhe_status_str(fhe_status status);

#ifdef __cplusplus
}
#endif
#endif /* FHE_H */
