// Device-side constant tables of a context.
//
// Basis Q = {q_0..q_{k-1}} (the ciphertext modulus) is extended by an
// auxiliary basis P = {p_0..p_{k'-1}} (primes below 2^61 chosen by the
// library) with P > t n q, so that round(t D / q) of the exact tensor D is
// uniquely represented modulo P.  Rows of an extended polynomial are ordered
// Q limbs first, then P limbs ("prime index" 0..K-1, K = k + k').
#pragma once
#include <stdint.h>

constexpr int FHE_MAXK = 16;   // Q primes
constexpr int FHE_MAXKP = 20;  // P primes
constexpr int FHE_MAXB = 20;   // largest basis handled by the exact path

struct PrimeConst {
    uint64_t q;
    uint64_t qinv_neg;   // -q^-1 mod 2^64
    uint64_t one_p;      // floor(2^64 / q): Shoup companion of 1
    uint64_t ninv, ninv_p;     // n^-1 mod q (Shoup pair)
    uint64_t ninvm, ninvm_p;   // n^-1 2^64 mod q (Shoup pair): inverse after Montgomery products
    uint64_t r32, r32_p;       // 2^32 mod q (Shoup pair)
    uint64_t off59, off62;     // smallest multiples of q at least 2^59 and 2^62
    uint64_t mx_neg_bias;      // -FHE_MX_BIAS sum_{u < 8} 256^u mod q (matrix-core weighted sums)
};

// Exact mixed-radix (Garner) conversion of a value given in basis M.
struct MrcConst {
    uint32_t K;                              // basis size
    uint32_t ntarget;                        // number of target primes
    uint64_t m[FHE_MAXB];                    // basis primes
    uint64_t inv[FHE_MAXB][FHE_MAXB];        // [m_a^-1]_{m_b}, a < b
    uint64_t inv_p[FHE_MAXB][FHE_MAXB];      //   Shoup companions (mod m_b)
    uint64_t one_p[FHE_MAXB];                // floor(2^64 / m_b)
    uint64_t half_digit[FHE_MAXB];           // mixed-radix digits of (M - 1) / 2
    uint64_t target[FHE_MAXB + 1];           // target primes (last slot: t for decryption)
    uint64_t tgt_one_p[FHE_MAXB + 1];
    uint64_t m_mod_t[FHE_MAXB][FHE_MAXB + 1];    // [m_a]_{target_j}
    uint64_t m_mod_t_p[FHE_MAXB][FHE_MAXB + 1];  //   Shoup companions
    uint64_t M_mod_t[FHE_MAXB + 1];              // [M]_{target_j}
};

// Constants of the fast base conversions.  Each output residue is one
// Montgomery reduction of a 128-bit sum of products sum_t a_t b_t, where the b_t
// are stored premultiplied by 2^64 mod the target prime; additive constants
// (overflow corrections, offsets) enter the same sum as extra terms.  Tables
// are target-major so one output's constants are contiguous.
struct ConvConst {
    uint32_t k, kp;
    uint64_t t;
    // 1 when every multiply-accumulate of the conversion stays below 2^64 (2 m - 1)
    // for its target prime m, so one Montgomery reduction (below 3m) suffices
    // without first reducing the high word: lift Q -> P, scale in P, P -> Q.
    uint32_t fast_lift, fast_scale_p, fast_p2q, pad_fast;
    // basis primes and their reduction helpers
    uint64_t q[FHE_MAXK], q_qinv[FHE_MAXK], q_one[FHE_MAXK];     // Q: prime, -q^-1 mod 2^64, floor(2^64/q)
    uint64_t p[FHE_MAXKP], p_qinv[FHE_MAXKP], p_one[FHE_MAXKP];  // P: likewise
    // ---- Q -> P, centred (lift of the inputs) ----
    uint64_t qhinv[FHE_MAXK], qhinv_p[FHE_MAXK];  // [qhat_i^-1]_{q_i} (Shoup pair)
    double inv_q[FHE_MAXK];                        // 1 / q_i
    // lift_m[j][i] = [qhat_i]_{p_j} 2^64 (i < k); lift_m[j][k] = [-q]_{p_j} 2^64 (times beta)
    uint64_t lift_m[FHE_MAXKP][FHE_MAXK + 1];
    // ---- scale: C = floor((t D + h) / q) modulo P, h = (q-1)/2 ----
    uint64_t tqhinv[FHE_MAXK], tqhinv_p[FHE_MAXK];  // [t qhat_i^-1]_{q_i}
    uint64_t hqhinv[FHE_MAXK];                       // [h qhat_i^-1]_{q_i}
    // scale_m[j][i] = [-q_i^-1]_{p_j} 2^64 (i < k), then [t q^-1]_{p_j} 2^64 (times D_{p_j}),
    // [1]_{p_j} 2^64 (times v), [h q^-1]_{p_j} 2^64 (times 1)
    uint64_t scale_m[FHE_MAXKP][FHE_MAXK + 3];
    // ---- P -> Q, centred ----
    uint64_t phinv[FHE_MAXKP], phinv_p[FHE_MAXKP];  // [phat_j^-1]_{p_j}
    double inv_p[FHE_MAXKP];
    // p2q_m[i][j] = [phat_j]_{q_i} 2^64 (j < k'); p2q_m[i][k'] = [-P]_{q_i} 2^64 (times beta)
    uint64_t p2q_m[FHE_MAXK][FHE_MAXKP + 1];
    // ---- exact path of the scale ----
    uint64_t h_q[FHE_MAXK];                              // [h]_{q_i}
    uint64_t h_p[FHE_MAXKP];                             // [h]_{p_j}
    uint64_t t_q[FHE_MAXK], t_qs[FHE_MAXK];              // [t]_{q_i}
    uint64_t t_p[FHE_MAXKP], t_ps[FHE_MAXKP];            // [t]_{p_j}
    uint64_t qinv_p[FHE_MAXKP], qinv_ps[FHE_MAXKP];      // [q^-1]_{p_j}
    // ---- decryption: m = (h - [Y]_q) q^-1 mod t ----
    uint64_t h_t, qinv_t, qinv_ts, t_one_p;
    // ---- plaintext constant: Delta = floor(q / t) ----
    uint64_t delta_q[FHE_MAXK], delta_qs[FHE_MAXK];      // [Delta]_{q_i}
};

// Threshold of the floating estimate: the estimate of sum y_i / m_i is within
// 2^-44.8 of the exact value for bases of up to 16 primes below 2^62 (see the
// error bound next to the estimate); coefficients whose fractional part is
// within this margin of the rounding boundary take the exact path.
constexpr double FHE_EST_MARGIN = 9.094947017729282e-13;  // 2^-40

// Operand tables of the base conversions on the int8 matrix cores, for bases
// of at most 8 primes on each side.  A conversion r_t = sum_s x_s W[t][s] mod
// m_t (sources s, targets t, weights in Montgomery form) runs as four products
// v_mfma_i32_16x16x64_i8 per 16 coefficients: every x_s < 2^62 is written in
// balanced base-256 digits, x_s = sum_u d_{s,u} 256^u with d in [-128, 127],
// the weight of digit u is W[t][s] 256^u mod m_t, itself split into balanced
// digits w_v (v = 0..7), and the products give P_{t,v} = sum_{s,u} d_{s,u}
// w_v(W[t][s] 256^u mod m_t), exactly (|P| <= 2^20 per product of 64 terms,
// 2^21 for two chained products).  With the int32 accumulators started at
// FHE_MX_BIAS, r_t = (sum_v 256^v P'_{t,v} + extra terms + E_t) 2^-64 mod m_t,
// where E_t = -FHE_MX_BIAS sum_v 256^v mod m_t (plus any additive constant of
// the conversion) removes the bias.
// Operand a_*[mm][lane] (four int32 = 16 bytes): row lane % 16 of product mm
// is target 4 (mm / 2) + (lane % 16) / 4, digit v = 4 (mm % 2) + lane % 4;
// byte b is source lane / 16 + 4 (b / 8), digit u = b % 8.  Lane l then
// supplies the digits of sources l/16 and l/16 + 4 and receives P' of targets
// l/16 and l/16 + 4 for column l % 16.
constexpr int FHE_MX_MAXB = 8;
constexpr int32_t FHE_MX_BIAS = 1 << 21;
struct ConvMx {
    int32_t a_lift[4][64][4];   // Q -> P centred lift: W[j][i] = [qhat_i]_{p_j} 2^64
    int32_t a_scale[4][64][4];  // scale in P: W[j][i] = [-q_i^-1 phat_j^-1]_{p_j} 2^64
    int32_t a_sdp[4][64][4];    // scale in P, sources D_{p_s}: W[j][s] = [s == j] [t q^-1 phat_j^-1]_{p_j} 2^64
    int32_t a_p2q[4][64][4];    // P -> Q: W[i][j] = [phat_j]_{q_i} 2^64
    uint64_t e_lift[FHE_MX_MAXB];   // bias removal mod p_j
    uint64_t e_scale[FHE_MX_MAXB];  // bias removal plus [h q^-1 phat_j^-1]_{p_j} 2^64
    uint64_t e_p2q[FHE_MX_MAXB];    // bias removal mod q_i
    uint64_t s_v[FHE_MX_MAXB];      // [phat_j^-1]_{p_j} 2^64 (times v)
    uint64_t l_beta[FHE_MX_MAXB];   // [-q]_{p_j} 2^64 (times beta of the lift)
    uint64_t p_beta[FHE_MX_MAXB];   // [-P]_{q_i} 2^64 (times beta of P -> Q)
};
