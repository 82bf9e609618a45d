// Exact base conversions (lift, scale-and-round, P -> Q), decryption scaling,
// elementwise ciphertext operations and the bridge glue.
//
// Base conversions follow the "fast conversion with exact overflow count"
// pattern: for a value X known by residues x_i in basis {m_i},
//   y_i = [x_i (M/m_i)^-1]_{m_i},   sum_i y_i M/m_i = X + v M,  v = floor(sum y_i/m_i),
// so X modulo another prime p is sum_i y_i [M/m_i]_p - v [M]_p.  The overflow v
// (or, for the centred lift, round(sum y_i / m_i)) is read off a double
// precision estimate of sum y_i / m_i; when that estimate is within
// FHE_EST_MARGIN of the decision boundary the coefficient is recomputed
// exactly by mixed-radix (Garner) conversion instead, so every output word is
// the exact one.
#include "kernels.hpp"
#include "modarith.hpp"

namespace {

// A table word read through the constant address space: the tables do not
// change while a kernel runs, and wave-uniform reads then become scalar loads
// (the multiply-add asm takes its constant operand from SGPRs).
__device__ __forceinline__ uint64_t ldc(const uint64_t *p) {
    return *(const __attribute__((address_space(4))) uint64_t *)p;
}

// ---------------------------------------------------------------- exact path --

// The exact path runs for a tiny fraction of the coefficients: its loops stay
// rolled so that it does not raise the register count (and so the occupancy)
// of the fast path that shares the kernel.

// Garner digits d of X (residues r in basis M): X = sum_b d_b prod_{a<b} m_a.
template <int MB>
__device__ __forceinline__ void mrc_digits(const MrcConst &M, const uint64_t (&r)[MB],
                                           uint64_t (&d)[MB]) {
    const int K = (int)M.K;
#pragma unroll 1
    for (int b = 0; b < MB; b++) {
        d[b] = 0;
        if (b < K) {
            const uint64_t mb = M.m[b];
            uint64_t v = r[b];
#pragma unroll 1
            for (int a = 0; a < MB; a++) {
                if (a < b) {
                    const uint64_t da = mul_shoup(d[a], 1, M.one_p[b], mb);
                    v = sub_mod(v, da, mb);
                    v = mul_shoup(v, M.inv[a][b], M.inv_p[a][b], mb);
                }
            }
            d[b] = v;
        }
    }
}

// X > (M - 1) / 2 ?  (lexicographic on the digits, most significant first)
template <int MB>
__device__ __forceinline__ bool mrc_gt_half(const MrcConst &M, const uint64_t (&d)[MB]) {
    int res = 0;
#pragma unroll 1
    for (int b = MB - 1; b >= 0; b--) {
        if (b < (int)M.K && res == 0) {
            const uint64_t h = M.half_digit[b];
            res = d[b] > h ? 1 : (d[b] < h ? -1 : 0);
        }
    }
    return res == 1;
}

// X mod target j by Horner on the digits: acc = acc * m_b + d_b, b = K-1 .. 0.
template <int MB>
__device__ __forceinline__ uint64_t mrc_eval(const MrcConst &M, const uint64_t (&d)[MB], int j) {
    const uint64_t p = M.target[j], op = M.tgt_one_p[j];
    uint64_t acc = 0;
#pragma unroll 1
    for (int b = MB - 1; b >= 0; b--) {
        if (b < (int)M.K) {
            acc = mul_shoup(acc, M.m_mod_t[b][j], M.m_mod_t_p[b][j], p);
            acc = add_mod(acc, mul_shoup(d[b], 1, op, p), p);
        }
    }
    return acc;
}

// ---------------------------------------------------------------- lift ------

// Exact centred lift of one coefficient (residues x in Q) by mixed-radix
// conversion; put(j, r) receives r = x~ mod p_j.  Counts the coefficient in
// the fallback counter.
template <int MK, int MKP, bool EX, class Put>
__device__ __forceinline__ void lift_exact(const DevCtx &c, const uint64_t (&x)[MK], Put put) {
    const int kp = EX ? MKP : c.kp;
    const ConvConst &cc = *c.cc;
    atomicAdd(c.fallback, 1ull);
    const MrcConst &M = *c.mrc_q;
    uint64_t dg[MK];
    mrc_digits<MK>(M, x, dg);
    const bool gt = mrc_gt_half<MK>(M, dg);
#pragma unroll 1
    for (int j = 0; j < MKP; j++) {
        if (j < kp) {
            uint64_t r = mrc_eval<MK>(M, dg, j);
            if (gt) r = sub_mod(r, M.M_mod_t[j], cc.p[j]);
            put(j, r);
        }
    }
}

// Centred lift of one coefficient given by its residues x in Q:
//   x~ = sum_i y_i qhat_i - beta q,  y_i = [x_i qhat_i^-1]_{q_i},  beta = round(sum_i y_i / q_i),
// in (-q/2, q/2); put(j, r) receives r = x~ mod p_j for every P prime.
template <int MK, int MKP, bool EX, class Put>
__device__ __forceinline__ void lift_coef(const DevCtx &c, const uint64_t (&x)[MK], Put put) {
    const int k = EX ? MK : c.k, kp = EX ? MKP : c.kp;
    const ConvConst &cc = *c.cc;
    uint64_t y[MK];
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < MK; i++) {
        y[i] = 0;
        if (i < k) {
            y[i] = mul_shoup(x[i], cc.qhinv[i], cc.qhinv_p[i], cc.q[i]);
            e = fma((double)y[i], cc.inv_q[i], e);
        }
    }
    // |e - sum y_i/q_i| <= (2.01 K + 1.01 K^2) 2^-53 < 2^-44 for K <= 20.
    const double fl = floor(e), d = e - fl;
    if (fabs(d - 0.5) >= FHE_EST_MARGIN) {
        const uint64_t beta = (uint64_t)fl + (d > 0.5 ? 1 : 0);
#pragma unroll
        for (int j = 0; j < MKP; j++) {
            if (j < kp) {
                const uint64_t *m = cc.lift_m[j];
                Acc3 acc;
                acc3_init(acc);
#pragma unroll
                for (int i = 0; i < MK; i++)
                    if (i < k) acc3_mac(acc, y[i], ldc(m + i));
                acc3_mac(acc, beta, ldc(m + k));
                put(j, cc.fast_lift ? acc_reduce_mont_small(acc3_value(acc), cc.p[j], cc.p_qinv[j])
                                     : acc_reduce_mont(acc3_value(acc), cc.p[j], cc.p_qinv[j], cc.p_one[j]));
            }
        }
    } else {
        lift_exact<MK, MKP, EX>(c, x, put);
    }
}

// Extended rows of the inputs: for every coefficient of poly `blockIdx.y` of
// item `blockIdx.z`, the centred lift x~ in (-q/2, q/2) written modulo each
// P prime into E[item][poly][k + j].
// EX: the basis sizes are exactly MK and MKP (loops without per-term branches).
template <int MK, int MKP, bool EX>
__global__ __launch_bounds__(256) void k_lift(DevCtx c, const uint64_t *__restrict__ a,
                                              const uint64_t *__restrict__ b,
                                              uint64_t *__restrict__ E, int npoly) {
    const int n = c.n, k = EX ? MK : c.k, K = EX ? MK + MKP : c.K;
    const int coef = blockIdx.x * 256 + threadIdx.x;
    if (coef >= n) return;
    const int poly = blockIdx.y;
    const size_t item = blockIdx.z;
    const uint64_t *src = poly < 2 ? a + (item * 2 + poly) * (size_t)k * n
                                   : b + (item * 2 + poly - 2) * (size_t)k * n;
    uint64_t *dst = E + ((item * npoly + poly) * K + k) * (size_t)n;
    uint64_t x[MK];
#pragma unroll
    for (int i = 0; i < MK; i++) x[i] = i < k ? src[(size_t)i * n + coef] : 0;
    lift_coef<MK, MKP, EX>(c, x, [&](int j, uint64_t r) { dst[(size_t)j * n + coef] = r; });
}

// ------------------------------------------------------- scale and round ----

// C = round(t D / q) = floor((t D + h) / q), h = (q - 1)/2, for D given by its
// residues in Q and P (rows Dt[item][comp][0..K)), written in basis Q.
// Step 1 (in P):   C_{p_j} = [t q^-1 D_{p_j} + h q^-1 + v - sum_i y_i q_i^-1]_{p_j},
//                  y_i = [(t D_{q_i} + h) qhat_i^-1]_{q_i}, v = floor(sum_i y_i / q_i).
// Step 2 (P -> Q): centred conversion of C, which satisfies |C| < P/2.

// Exact scale-and-round of one coefficient: Y = t D + h; [Y]_q by Garner over
// Q; C_p = (Y_p - [Y]_q) q^-1; then the centred value of C by Garner over P.
// Counts the coefficient in the fallback counter.
template <int MK, int MKP, bool EX, class Put>
__device__ __forceinline__ void scale_exact(const DevCtx &c, const uint64_t (&dq)[MK], const uint64_t (&dp)[MKP],
                                            Put put) {
    const int k = EX ? MK : c.k, kp = EX ? MKP : c.kp;
    const ConvConst &cc = *c.cc;
    atomicAdd(c.fallback, 1ull);
    const MrcConst &MQ = *c.mrc_q;
    const MrcConst &MP = *c.mrc_p;
    uint64_t yq[MK], dgq[MK];
#pragma unroll
    for (int i = 0; i < MK; i++) {
        yq[i] = 0;
        if (i < k) yq[i] = add_mod(mul_shoup(dq[i], cc.t_q[i], cc.t_qs[i], cc.q[i]), cc.h_q[i], cc.q[i]);
    }
    mrc_digits<MK>(MQ, yq, dgq);
    uint64_t cp[MKP], dgp[MKP];
#pragma unroll 1
    for (int j = 0; j < MKP; j++) {
        cp[j] = 0;
        if (j < kp) {
            const uint64_t pj = cc.p[j];
            const uint64_t ypj = add_mod(mul_shoup(dp[j], cc.t_p[j], cc.t_ps[j], pj), cc.h_p[j], pj);
            const uint64_t xpj = mrc_eval<MK>(MQ, dgq, j);
            cp[j] = mul_shoup(sub_mod(ypj, xpj, pj), cc.qinv_p[j], cc.qinv_ps[j], pj);
        }
    }
    mrc_digits<MKP>(MP, cp, dgp);
    const bool gt = mrc_gt_half<MKP>(MP, dgp);
#pragma unroll 1
    for (int i = 0; i < MK; i++) {
        if (i < k) {
            uint64_t r = mrc_eval<MKP>(MP, dgp, i);
            if (gt) r = sub_mod(r, MP.M_mod_t[i], cc.q[i]);
            put(i, r);
        }
    }
}

// One coefficient of round(t D / q): D given by its residues dq in Q and dp
// in P (canonical); put(i, r) receives r = C mod q_i.
template <int MK, int MKP, bool EX, class Put>
__device__ __forceinline__ void scale_coef(const DevCtx &c, const uint64_t (&dq)[MK], const uint64_t (&dp)[MKP],
                                           Put put) {
    const int k = EX ? MK : c.k, kp = EX ? MKP : c.kp;
    const ConvConst &cc = *c.cc;
    uint64_t y[MK];
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < MK; i++) {
        y[i] = 0;
        if (i < k) {
            y[i] = add_mod(mul_shoup(dq[i], cc.tqhinv[i], cc.tqhinv_p[i], cc.q[i]), cc.hqhinv[i], cc.q[i]);
            e = fma((double)y[i], cc.inv_q[i], e);
        }
    }
    const double fl = floor(e), d = e - fl;
    bool exact = (d < FHE_EST_MARGIN) || (d > 1.0 - FHE_EST_MARGIN);
    const uint64_t v = (uint64_t)fl;

    uint64_t z[MKP];
    double e2 = 0.0;
#pragma unroll
    for (int j = 0; j < MKP; j++) {
        z[j] = 0;
        if (j < kp) {
            const uint64_t *m = cc.scale_m[j];
            Acc3 acc;
            acc3_init(acc);
#pragma unroll
            for (int i = 0; i < MK; i++)
                if (i < k) acc3_mac(acc, y[i], ldc(m + i));
            acc3_mac(acc, dp[j], ldc(m + k));
            acc3_mac(acc, v, ldc(m + k + 1));
            acc3_add(acc, ldc(m + k + 2));
            const uint64_t r = cc.fast_scale_p  // C_{p_j}
                                   ? acc_reduce_mont_small(acc3_value(acc), cc.p[j], cc.p_qinv[j])
                                   : acc_reduce_mont(acc3_value(acc), cc.p[j], cc.p_qinv[j], cc.p_one[j]);
            z[j] = mul_shoup(r, cc.phinv[j], cc.phinv_p[j], cc.p[j]);
            e2 = fma((double)z[j], cc.inv_p[j], e2);
        }
    }
    const double fl2 = floor(e2), d2 = e2 - fl2;
    exact = exact || (fabs(d2 - 0.5) < FHE_EST_MARGIN);
    if (!exact) {
        const uint64_t beta = (uint64_t)fl2 + (d2 > 0.5 ? 1 : 0);
#pragma unroll
        for (int i = 0; i < MK; i++) {
            if (i < k) {
                const uint64_t *m = cc.p2q_m[i];
                Acc3 acc;
                acc3_init(acc);
#pragma unroll
                for (int j = 0; j < MKP; j++)
                    if (j < kp) acc3_mac(acc, z[j], ldc(m + j));
                acc3_mac(acc, beta, ldc(m + kp));
                put(i, cc.fast_p2q ? acc_reduce_mont_small(acc3_value(acc), cc.q[i], cc.q_qinv[i])
                                  : acc_reduce_mont(acc3_value(acc), cc.q[i], cc.q_qinv[i], cc.q_one[i]));
            }
        }
        return;
    }
    scale_exact<MK, MKP, EX>(c, dq, dp, put);
}

// Component comp0 + blockIdx.y of item blockIdx.z: components 0 and 1 go to
// out (a ciphertext), component 2 to C2.
template <int MK, int MKP, bool EX>
__global__ __launch_bounds__(256) void k_scale(DevCtx c, const uint64_t *__restrict__ Dt,
                                               uint64_t *__restrict__ out,
                                               uint64_t *__restrict__ C2, int comp0) {
    const int n = c.n, k = EX ? MK : c.k, kp = EX ? MKP : c.kp, K = EX ? MK + MKP : c.K;
    const int coef = blockIdx.x * 256 + threadIdx.x;
    if (coef >= n) return;
    const int comp = comp0 + (int)blockIdx.y;
    const size_t item = blockIdx.z;
    const uint64_t *src = Dt + (item * 3 + comp) * (size_t)K * n;
    uint64_t *dst = comp < 2 ? out + (item * 2 + comp) * (size_t)k * n : C2 + item * (size_t)k * n;
    uint64_t dq[MK], dp[MKP];
#pragma unroll
    for (int i = 0; i < MK; i++) dq[i] = i < k ? src[(size_t)i * n + coef] : 0;
#pragma unroll
    for (int j = 0; j < MKP; j++) dp[j] = j < kp ? src[(size_t)(k + j) * n + coef] : 0;
    scale_coef<MK, MKP, EX>(c, dq, dp, [&](int i, uint64_t r) { dst[(size_t)i * n + coef] = r; });
}

// First squaring of the bridge chains, shared work.  Chain c of input j is
// y_c = x_j - (Delta c, 0); its centred lift differs from that of x_j only by
// an integer gamma_c in the constant coefficient of the first polynomial, so
// its exact tensor is
//   D0(y_c) = D0(x_j) + 2 gamma_c x~0 + gamma_c^2,  D1(y_c) = D1(x_j) + 2 gamma_c x~1,
//   D2(y_c) = D2(x_j)
// (x~ the centred lift of x_j over Q and P).  k_scale_chain rebuilds D0, D1 of
// the chain from x_j's tensor and rounds them; D2, and with it the key
// switching, is computed once per input.
//
// gamma table per chain and prime l of Q then P: [2 gamma 2^64 mod p_l,
// gamma^2 mod p_l] (the first a Montgomery multiplier).

// (hi 2^64 + lo) mod p for p < 2^62, by 64 doubling steps (setup only).
__device__ uint64_t mod128_slow(uint64_t hi, uint64_t lo, uint64_t p) {
    uint64_t r = hi % p;
    for (int b = 63; b >= 0; b--) {
        r = (r << 1) | ((lo >> b) & 1u);
        if (r >= p) r -= p;
    }
    return r;
}

__device__ uint64_t mulmod_slow(uint64_t a, uint64_t b, uint64_t p) {
    uint64_t lo, hi;
    mul128(a, b, lo, hi);
    return mod128_slow(hi, lo, p);
}

// One thread per chain (input j = chain / tcount, c = c0 + chain % tcount).
// x: the inputs [count][2][k][n]; E: their lift [count][2][K][n] (P rows).
template <int MK, int MKP, bool EX>
__global__ __launch_bounds__(64) void k_bridge_gamma(DevCtx c, const uint64_t *__restrict__ x,
                                                     const uint64_t *__restrict__ E,
                                                     uint64_t *__restrict__ gam, size_t chains, int tcount,
                                                     int c0) {
    const size_t chain = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (chain >= chains) return;
    const int n = c.n, k = EX ? MK : c.k, kp = EX ? MKP : c.kp, K = EX ? MK + MKP : c.K;
    const size_t j = chain / tcount;
    const uint64_t cv = c0 + chain % tcount;
    const ConvConst &cc = *c.cc;
    uint64_t *g = gam + chain * 2 * (size_t)K;
    uint64_t x0[MK];
#pragma unroll
    for (int i = 0; i < MK; i++) {
        x0[i] = 0;
        if (i < k) {
            const uint64_t q = cc.q[i];
            const uint64_t dc = mul_shoup(cv % q, cc.delta_q[i], cc.delta_qs[i], q);
            x0[i] = sub_mod(x[(j * 2) * (size_t)k * n + (size_t)i * n], dc, q);
            const uint64_t gm = dc ? q - dc : 0;  // gamma mod q_i = -Delta c
            const uint64_t r1 = (uint64_t)0 - cc.q_one[i] * q;  // 2^64 mod q (< q)
            g[2 * i] = mulmod_slow(add_mod(gm, gm, q), r1, q);
            g[2 * i + 1] = mulmod_slow(gm, gm, q);
        }
    }
    lift_coef<MK, MKP, EX>(c, x0, [&](int jp, uint64_t r) {
        const uint64_t p = cc.p[jp];
        const uint64_t gm = sub_mod(r, E[(j * 2) * (size_t)K * n + (size_t)(k + jp) * n], p);
        const uint64_t r1 = (uint64_t)0 - cc.p_one[jp] * p;
        g[2 * (k + jp)] = mulmod_slow(add_mod(gm, gm, p), r1, p);
        g[2 * (k + jp) + 1] = mulmod_slow(gm, gm, p);
    });
    (void)kp;
}

// Components 0 and 1 (blockIdx.y) of the first squaring of chain blockIdx.z:
// D rebuilt from the input's tensor Dt [count][3][K][n], its lift x~ (Q rows
// from x, P rows from E) and the gamma table; the rounded value plus the input's
// key-switching output R [count][2][k][n] is the chain's ciphertext in y.
template <int MK, int MKP, bool EX>
__global__ __launch_bounds__(256) void k_scale_chain(DevCtx c, const uint64_t *__restrict__ Dt,
                                                     const uint64_t *__restrict__ x,
                                                     const uint64_t *__restrict__ E,
                                                     const uint64_t *__restrict__ gam,
                                                     const uint64_t *__restrict__ R,
                                                     uint64_t *__restrict__ y, int tcount) {
    const int n = c.n, k = EX ? MK : c.k, kp = EX ? MKP : c.kp, K = EX ? MK + MKP : c.K;
    const int coef = blockIdx.x * 256 + threadIdx.x;
    if (coef >= n) return;
    const int comp = blockIdx.y;
    const size_t chain = blockIdx.z, j = chain / tcount;
    const ConvConst &cc = *c.cc;
    const uint64_t *src = Dt + (j * 3 + comp) * (size_t)K * n;
    const uint64_t *xq = x + (j * 2 + comp) * (size_t)k * n;
    const uint64_t *xp = E + (j * 2 + comp) * (size_t)K * n;
    const uint64_t *g = gam + chain * 2 * (size_t)K;
    const bool sq = comp == 0 && coef == 0;
    uint64_t dq[MK], dp[MKP];
#pragma unroll
    for (int i = 0; i < MK; i++) {
        dq[i] = 0;
        if (i < k) {
            const uint64_t q = cc.q[i];
            uint64_t v = src[(size_t)i * n + coef] + mont_mul_lazy(xq[(size_t)i * n + coef], ldc(g + 2 * i), q,
                                                                   cc.q_qinv[i]);
            if (sq) v += ldc(g + 2 * i + 1);
            dq[i] = csub(csub(v, q << 1), q);  // < 4q before
        }
    }
#pragma unroll
    for (int jp = 0; jp < MKP; jp++) {
        dp[jp] = 0;
        if (jp < kp) {
            const uint64_t p = cc.p[jp];
            const int l = k + jp;
            uint64_t v = src[(size_t)l * n + coef] + mont_mul_lazy(xp[(size_t)l * n + coef], ldc(g + 2 * l), p,
                                                                   cc.p_qinv[jp]);
            if (sq) v += ldc(g + 2 * l + 1);
            dp[jp] = csub(csub(v, p << 1), p);
        }
    }
    const uint64_t *r = R + (j * 2 + comp) * (size_t)k * n;
    uint64_t *dst = y + (chain * 2 + comp) * (size_t)k * n;
    scale_coef<MK, MKP, EX>(c, dq, dp, [&](int i, uint64_t v) {
        dst[(size_t)i * n + coef] = add_mod(v, r[(size_t)i * n + coef], cc.q[i]);
    });
}

// -------------------------------------------------------- decryption ------

// pt = floor((t X + h) / q) mod t = (h - [t X + h]_q) q^-1 mod t, X = [c0 + c1 s]_q.
template <int MK>
__global__ __launch_bounds__(256) void k_decrypt_scale(DevCtx c, const uint64_t *__restrict__ X,
                                                       uint64_t *__restrict__ pt) {
    const int n = c.n, k = c.k, kp = c.kp;
    const int coef = blockIdx.x * 256 + threadIdx.x;
    if (coef >= n) return;
    const size_t item = blockIdx.y;
    const ConvConst &cc = *c.cc;
    const MrcConst &MQ = *c.mrc_q;
    uint64_t y[MK], d[MK];
#pragma unroll
    for (int i = 0; i < MK; i++) {
        y[i] = 0;
        if (i < k) {
            const uint64_t qi = c.pc[i].q;
            const uint64_t xv = X[(item * k + i) * (size_t)n + coef];
            y[i] = add_mod(mul_shoup(xv, cc.t_q[i], cc.t_qs[i], qi), cc.h_q[i], qi);
        }
    }
    mrc_digits<MK>(MQ, y, d);
    const uint64_t t = c.t;
    const uint64_t yt = mrc_eval<MK>(MQ, d, kp);  // target slot kp is t
    pt[item * n + coef] = mul_shoup(sub_mod(cc.h_t, yt, t), cc.qinv_t, cc.qinv_ts, t);
}

// ------------------------------------------------------- elementwise ------

__global__ void k_addsub(DevCtx c, const uint64_t *__restrict__ a, const uint64_t *__restrict__ b,
                         uint64_t *__restrict__ out, size_t words, int op) {
    const size_t n = c.n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x) {
        const int limb = (int)((i / n) % c.k);
        const uint64_t q = c.pc[limb].q;
        const uint64_t x = a[i];
        uint64_t r;
        if (op == 0) r = add_mod(x, b[i], q);
        else if (op == 1) r = sub_mod(x, b[i], q);
        else r = x == 0 ? 0 : q - x;
        out[i] = r;
    }
}

// out = a, except c0's constant coefficient +/- Delta * cval.
__global__ void k_plain_const(DevCtx c, const uint64_t *__restrict__ a, uint64_t *__restrict__ out,
                              size_t words, uint64_t cval, int sign) {
    const size_t n = c.n, k = c.k;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x) {
        uint64_t x = a[i];
        const size_t coef = i % n, row = i / n;
        const size_t limb = row % k, poly = (row / k) % 2;
        if (coef == 0 && poly == 0) {
            const uint64_t q = c.pc[limb].q;
            const uint64_t dc = mul_shoup(cval % q, c.cc->delta_q[limb], c.cc->delta_qs[limb], q);
            x = sign > 0 ? add_mod(x, dc, q) : sub_mod(x, dc, q);
        }
        out[i] = x;
    }
}

__global__ void k_small_to_rns(DevCtx c, const void *__restrict__ v, int is8,
                               uint64_t *__restrict__ out, size_t count) {
    const size_t n = c.n, k = c.k;
    const size_t total = count * k * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t coef = i % n, limb = (i / n) % k, item = i / (n * k);
        const int64_t s = is8 ? (int64_t)((const int8_t *)v)[item * n + coef]
                              : (int64_t)((const int32_t *)v)[item * n + coef];
        const uint64_t q = c.pc[limb].q;
        out[i] = s >= 0 ? (uint64_t)s % q : (q - ((uint64_t)(-s) % q)) % q;
    }
}

__global__ void k_pointwise_mont(DevCtx c, const uint64_t *__restrict__ a,
                                 const uint64_t *__restrict__ b, uint64_t *__restrict__ out,
                                 size_t words, int bcast) {
    const size_t n = c.n, k = c.k;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t limb = (i / n) % k;
        const PrimeConst &P = c.pc[limb];
        const uint64_t bv = bcast ? b[limb * n + i % n] : b[i];
        out[i] = csub(mont_mul_lazy(a[i], bv, P.q, P.qinv_neg), P.q);
    }
}

__global__ void k_key_b(DevCtx c, const uint64_t *__restrict__ prod, const uint64_t *__restrict__ e,
                        const uint64_t *__restrict__ s2, int digit, uint64_t *__restrict__ out) {
    const size_t n = c.n, k = c.k;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < k * n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t limb = i / n;
        const uint64_t q = c.pc[limb].q;
        uint64_t r = add_mod(prod[i], e[i], q);
        r = r == 0 ? 0 : q - r;
        if ((int)limb == digit) r = add_mod(r, s2[i], q);
        out[i] = r;
    }
}

// ct[j] = (prod[0][j] + e[j][0] + Delta m_j, prod[1][j] + e[j][1]); prod is [2][count][k][n].
__global__ void k_encrypt_finish(DevCtx c, const uint64_t *__restrict__ prod,
                                 const int32_t *__restrict__ e, const uint64_t *__restrict__ pt,
                                 uint64_t *__restrict__ ct, size_t count) {
    const size_t n = c.n, k = c.k;
    const size_t total = count * 2 * k * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t coef = i % n, limb = (i / n) % k, poly = (i / (n * k)) % 2,
                     item = i / (2 * n * k);
        const uint64_t q = c.pc[limb].q;
        const int64_t ev = e[(item * 2 + poly) * n + coef];
        const uint64_t er = ev >= 0 ? (uint64_t)ev % q : (q - ((uint64_t)(-ev) % q)) % q;
        uint64_t r = add_mod(prod[((poly * count + item) * k + limb) * n + coef], er, q);
        if (poly == 0) {
            const uint64_t m = pt[item * n + coef] % q;
            r = add_mod(r, mul_shoup(m, c.cc->delta_q[limb], c.cc->delta_qs[limb], q), q);
        }
        ct[i] = r;
    }
}

// eq_c = Delta [coefficient 0 of c0] - y_c;  bits_b = sum_{c in [1,T), bit b of c} eq_c.
// y holds chains c = c0 .. c0 + tcount - 1 of every input (c0 = 0 or 1).
constexpr int FHE_MAXNB = 20;
__global__ __launch_bounds__(256) void k_bridge_combine(DevCtx c, const uint64_t *__restrict__ y,
                                                        uint64_t *__restrict__ bits,
                                                        uint64_t *__restrict__ eq, int tcount,
                                                        int nbits, int c0) {
    const int n = c.n, k = c.k;
    const int coef = blockIdx.x * 256 + threadIdx.x;
    if (coef >= n) return;
    const int row = blockIdx.y;  // poly * k + limb
    const int limb = row % k, poly = row / k;
    const size_t j = blockIdx.z;
    const size_t ctw = 2 * (size_t)k * n;
    const uint64_t q = c.pc[limb].q;
    const uint64_t one = (poly == 0 && coef == 0) ? c.cc->delta_q[limb] : 0;
    uint64_t acc[FHE_MAXNB];
#pragma unroll
    for (int b = 0; b < FHE_MAXNB; b++) acc[b] = 0;
    const size_t off = (size_t)row * n + coef;
    for (int cc = 0; cc < tcount; cc++) {
        const int cv = c0 + cc;
        const uint64_t yv = y[(j * tcount + cc) * ctw + off];
        const uint64_t ev = sub_mod(one, yv, q);
        if (eq) eq[(j * tcount + cc) * ctw + off] = ev;
#pragma unroll
        for (int b = 0; b < FHE_MAXNB; b++)
            if (b < nbits && ((cv >> b) & 1)) acc[b] = add_mod(acc[b], ev, q);
    }
#pragma unroll
    for (int b = 0; b < FHE_MAXNB; b++)
        if (b < nbits) bits[(j * nbits + b) * ctw + off] = acc[b];
}

// out = sum_b 2^b bits_b by Horner: r = bits_{nb-1}; r = r + r + bits_b.
// signed_top: the leading bit enters negated (two's complement weight).
__global__ void k_horner(DevCtx c, const uint64_t *__restrict__ bits, int nbits,
                         uint64_t *__restrict__ out, size_t count, int signed_top) {
    const size_t n = c.n, k = c.k, ctw = 2 * k * n;
    const size_t total = count * ctw;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t w = i % ctw, j = i / ctw;
        const uint64_t q = c.pc[(w / n) % k].q;
        uint64_t r = bits[(j * nbits + nbits - 1) * ctw + w];
        if (signed_top) r = sub_mod(0, r, q);
        for (int b = nbits - 2; b >= 0; b--) {
            r = add_mod(r, r, q);
            r = add_mod(r, bits[(j * nbits + b) * ctw + w], q);
        }
        out[i] = r;
    }
}

__global__ void k_validate(DevCtx c, const uint64_t *__restrict__ a, size_t words, int kmod, int off,
                           unsigned int *flag) {
    const size_t n = c.n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x) {
        const int limb = (int)((i / n) % kmod) + off;
        if (a[i] >= c.pc[limb].q) atomicOr(flag, 1u);
    }
}

// ------------------------------------------ conversions on the matrix cores --
//
// The base conversions of the lift and of the scale-and-round are dense
// contractions (coefficients x sources against a sources x targets matrix of
// constants), so for bases of at most 8 primes on each side they run on the
// int8 matrix cores, exactly, with the operand tables of ConvMx.  Per tile of
// 16 coefficients and per conversion: four v_mfma_i32_16x16x64_i8 give every
// target's eight partial sums (eight in the scale's first conversion, whose
// D_p term is a second, block-diagonal block chained onto the first); each
// lane recombines the sums of its two targets, adds the conversion's extra
// terms and reduces once (Montgomery).
// The floating estimates are summed over the four lanes of a column.  A
// coefficient whose estimate falls within FHE_EST_MARGIN of a decision
// boundary is queued in LDS and converted exactly (mixed radix) by one thread
// after the tiles; every output word is therefore the exact one, as on the
// vector ALU path.  The operand tables and the constants of every slot (prime
// s of the source and target bases) are staged in LDS and read per tile,
// which keeps the register count of a wave low.

typedef int mx_v4i __attribute__((ext_vector_type(4)));

// Coefficients per workgroup (four waves, tiles of 16).
constexpr int kMxSpan = 1024;

// Balanced base-256 digits of x as eight signed bytes: the bytes of x + B
// (B = 0x80 in every byte) are d_u + 128, and xor 0x80 turns each into d_u in
// two's complement.  Valid while x + B < 2^64 (x <= 0x7F7F7F7F7F7F7F7F, about
// 2^63 - 2^55); every value decomposed here is below 2^62.
__device__ __forceinline__ uint64_t mx_digits(uint64_t x) {
    constexpr uint64_t B = 0x8080808080808080ull;
    return (x + B) ^ B;
}

// B operand of a lane: the digits of its two sources (bytes 0..7, 8..15).
__device__ __forceinline__ mx_v4i mx_operand(uint64_t x0, uint64_t x1) {
    const uint64_t a = mx_digits(x0), b = mx_digits(x1);
    return mx_v4i{(int)(uint32_t)a, (int)(uint32_t)(a >> 32), (int)(uint32_t)b, (int)(uint32_t)(b >> 32)};
}

// LDS of a workgroup: the operand tables of its conversions, the constants of
// each slot on the Q side and on the P side, and the exact-path queue
// (offsets of coefficients within the workgroup's span).
struct MxShared {
    mx_v4i a[3][4][64];
    uint64_t cq[FHE_MX_MAXB][10];
    uint64_t cp[FHE_MX_MAXB][8];
    int item[kMxSpan];
    int count;
};

// acc[mm] = FHE_MX_BIAS + A[mm] B, mm = 0..3 (A = table `t` of the LDS): lane
// gets P' of target l/16 (acc[0]: digits 0..3, acc[1]: 4..7) and of target
// l/16 + 4 (acc[2], acc[3]).
__device__ __forceinline__ void mx_products(const MxShared &sh, int t, uint32_t lane, const mx_v4i B,
                                            mx_v4i (&acc)[4]) {
    const mx_v4i bias = {FHE_MX_BIAS, FHE_MX_BIAS, FHE_MX_BIAS, FHE_MX_BIAS};
#pragma unroll
    for (int mm = 0; mm < 4; mm++) acc[mm] = __builtin_amdgcn_mfma_i32_16x16x64_i8(sh.a[t][mm][lane], B, bias, 0, 0, 0);
}

// acc[mm] += A[mm] B (table `t`): a second block of 64 (source, digit) pairs.
__device__ __forceinline__ void mx_products_add(const MxShared &sh, int t, uint32_t lane, const mx_v4i B,
                                                mx_v4i (&acc)[4]) {
#pragma unroll
    for (int mm = 0; mm < 4; mm++)
        acc[mm] = __builtin_amdgcn_mfma_i32_16x16x64_i8(sh.a[t][mm][lane], B, acc[mm], 0, 0, 0);
}

// hi:lo = sum_v 256^v P'_v with P'_v = a[v] (v < 4), b[v - 4] (v >= 4), each in
// [0, 2^22]: pairs within 32 bits (< 2^31), then x = a01 + a23 2^16 and
// w = a45 + a67 2^16 (< 2^47), and the sum x + w 2^32 (< 2^79).
__device__ __forceinline__ void mx_recombine(const mx_v4i a, const mx_v4i b, uint64_t &lo, uint64_t &hi) {
    const uint32_t a01 = (uint32_t)a[0] + ((uint32_t)a[1] << 8);
    const uint32_t a23 = (uint32_t)a[2] + ((uint32_t)a[3] << 8);
    const uint32_t a45 = (uint32_t)b[0] + ((uint32_t)b[1] << 8);
    const uint32_t a67 = (uint32_t)b[2] + ((uint32_t)b[3] << 8);
    const uint64_t x = (uint64_t)a01 + ((uint64_t)a23 << 16);
    const uint64_t w = (uint64_t)a45 + ((uint64_t)a67 << 16);
    lo = x + (w << 32);
    hi = (w >> 32) + (lo < x ? 1u : 0u);
}

// (hi:lo) 2^-64 mod m in [0, m) for the sums of the matrix-core tiles: below
// 2^79 plus two 64-bit constants, so hi < 2^16 < m - 1 (every prime here is at
// least 2^20) and the Montgomery reduction hi + floor(m' m / 2^64) + [lo != 0]
// (m' = lo (-m^-1) mod 2^64) is already below 2m: one conditional subtraction.
__device__ __forceinline__ uint64_t mx_reduce(uint64_t lo, uint64_t hi, uint64_t m, uint64_t minv_neg) {
    return csub(redc_lazy(hi, lo, m, minv_neg), m);
}

__device__ __forceinline__ void mx_add(uint64_t &lo, uint64_t &hi, uint64_t alo, uint64_t ahi) {
    lo += alo;
    hi += ahi + (lo < alo ? 1u : 0u);
}

// Sum over the four lanes of a column (l, l ^ 16, l ^ 32, l ^ 48); every one
// of them gets the same value (each addition pairs the same two operands).
// a16, a32: byte addresses (l ^ 16) 4 and (l ^ 32) 4 of the lane exchange.
__device__ __forceinline__ double mx_swap(double x, int a) {
    const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(x));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double mx_colsum(double x, int a16, int a32) {
    x += mx_swap(x, a16);
    x += mx_swap(x, a32);
    return x;
}

// Tiles w, w + 4, ... (< ntiles) of wave w with their inputs loaded one tile
// ahead: load(R, tile) fills R, body(R, tile) uses it.
template <class Regs, class Load, class Body>
__device__ __forceinline__ void mx_tiles1(int wave, int ntiles, Load load, Body body) {
    Regs r;
    if (wave < ntiles) load(r, wave);
    for (int tile = wave; tile < ntiles; tile += 4) {
        asm volatile("" ::: "memory");  // read the LDS constants per tile
        const Regs cur = r;
        if (tile + 4 < ntiles) load(r, tile + 4);
        body(cur, tile);
    }
}

// The same with the inputs loaded two tiles ahead into two register sets.
template <class Regs, class Load, class Body>
__device__ __forceinline__ void mx_tiles(int wave, int ntiles, Load load, Body body) {
    Regs r0, r1;
    if (wave < ntiles) load(r0, wave);
    if (wave + 4 < ntiles) load(r1, wave + 4);
    for (int tile = wave; tile < ntiles; tile += 8) {
        asm volatile("" ::: "memory");  // read the LDS constants per tile
        {
            const Regs cur = r0;
            if (tile + 8 < ntiles) load(r0, tile + 8);
            body(cur, tile);
        }
        if (tile + 4 < ntiles) {
            asm volatile("" ::: "memory");
            const Regs cur = r1;
            if (tile + 12 < ntiles) load(r1, tile + 12);
            body(cur, tile + 4);
        }
    }
}

__device__ __forceinline__ double mx_f64(uint64_t bits) { return __longlong_as_double((long long)bits); }

// Table t of the LDS := operand table `src` (256 entries of 16 bytes; one per thread).
__device__ __forceinline__ void mx_stage_table(MxShared &sh, int t, const int32_t (*src)[64][4]) {
    const int e = (int)threadIdx.x;
    sh.a[t][e >> 6][e & 63] = reinterpret_cast<const mx_v4i *>(&src[0][0][0])[e];
}

// Scale slot constants.  Q side of slot s: q, -q^-1 mod 2^64, [t qhat^-1]
// (Shoup pair), [h qhat^-1], [-P] 2^64, bias removal, 1/q; P side: p,
// -p^-1 mod 2^64, (word 2 unused), the v multiplier, bias removal plus
// constant, 1/p.  Absent primes: zeros.
__device__ __forceinline__ void mx_stage_scale_slots(MxShared &sh, const DevCtx &c) {
    const ConvConst &cc = *c.cc;
    const ConvMx &mx = *c.mx;
    const int t = (int)threadIdx.x;
    if (t < FHE_MX_MAXB) {
        uint64_t *w = sh.cq[t];
        const bool ok = t < c.k;
        w[0] = ok ? cc.q[t] : 0;
        w[1] = ok ? cc.q_qinv[t] : 0;
        w[2] = ok ? cc.tqhinv[t] : 0;
        w[3] = ok ? cc.tqhinv_p[t] : 0;
        w[4] = ok ? cc.hqhinv[t] : 0;
        w[5] = ok ? mx.p_beta[t] : 0;
        w[6] = ok ? mx.e_p2q[t] : 0;
        w[7] = ok ? (uint64_t)__double_as_longlong(cc.inv_q[t]) : 0;
    } else if (t < 2 * FHE_MX_MAXB) {
        const int s = t - FHE_MX_MAXB;
        uint64_t *w = sh.cp[s];
        const bool ok = s < c.kp;
        w[0] = ok ? cc.p[s] : 0;
        w[1] = ok ? cc.p_qinv[s] : 0;
        w[3] = ok ? mx.s_v[s] : 0;
        w[4] = ok ? mx.e_scale[s] : 0;
        w[5] = ok ? (uint64_t)__double_as_longlong(cc.inv_p[s]) : 0;
    }
}

// Scale-and-round of one tile column on the matrix cores (tables 0: scale in
// P from the y_i, 1: P -> Q, 2: scale in P from D_p, block-diagonal).  dq,
// dp: the lane's two Q and two P residues of D, any representatives below
// 2^62 (absent primes read a present row; their constants and weights are
// zero); jv[h]: slot g + 4h is a P prime.  Returns false when the coefficient must take the exact path, else
// the lane's two outputs C mod q_s in out.
__device__ __forceinline__ bool mx_scale_tile(const MxShared &sh, uint32_t lane, int a16, int a32,
                                              const uint64_t (&dq)[2], const uint64_t (&dp)[2], const bool (&jv)[2],
                                              uint64_t (&out)[2]) {
    const uint32_t g = lane >> 4;
    uint64_t y[2];
    double e = 0.0;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint64_t *Q = sh.cq[g + 4 * h];
        y[h] = add_mod(mul_shoup(dq[h], Q[2], Q[3], Q[0]), Q[4], Q[0]);
        e = fma((double)y[h], mx_f64(Q[7]), e);
    }
    e = mx_colsum(e, a16, a32);
    const double fl = floor(e), d = e - fl;
    bool exact = (d < FHE_EST_MARGIN) || (d > 1.0 - FHE_EST_MARGIN);
    const uint64_t v = (uint32_t)fl;  // < k
    mx_v4i acc[4];
    mx_products(sh, 0, lane, mx_operand(y[0], y[1]), acc);
    mx_products_add(sh, 2, lane, mx_operand(dp[0], dp[1]), acc);
    uint64_t z[2];
    double e2 = 0.0;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint64_t *Pc = sh.cp[g + 4 * h];
        uint64_t lo, hi;
        mx_recombine(acc[2 * h], acc[2 * h + 1], lo, hi);
        mx_add(lo, hi, v * Pc[3], 0);
        mx_add(lo, hi, Pc[4], 0);
        // z_j = C_{p_j} phat_j^-1 mod p_j (the factor is folded into the table)
        z[h] = jv[h] ? mx_reduce(lo, hi, Pc[0], Pc[1]) : 0;
        e2 = fma((double)z[h], mx_f64(Pc[5]), e2);
    }
    e2 = mx_colsum(e2, a16, a32);
    const double fl2 = floor(e2), d2 = e2 - fl2;
    exact = exact || (fabs(d2 - 0.5) < FHE_EST_MARGIN);
    const uint64_t beta = (uint32_t)fl2 + (d2 > 0.5 ? 1u : 0u);  // <= k'
    mx_products(sh, 1, lane, mx_operand(z[0], z[1]), acc);
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint64_t *Q = sh.cq[g + 4 * h];
        uint64_t lo, hi;
        mx_recombine(acc[2 * h], acc[2 * h + 1], lo, hi);
        mx_add(lo, hi, beta * Q[5], 0);
        mx_add(lo, hi, Q[6], 0);
        out[h] = mx_reduce(lo, hi, Q[0], Q[1]);
    }
    return !exact;
}

// Row offsets (in words) of the lane's two slots: slot s = l/16 + 4h, clamped
// to the basis (an absent prime reads a present row; its constants are zero,
// so the words read there do not enter any output).
__device__ __forceinline__ uint32_t mx_row(int s, int nb, int first, int n) {
    return (uint32_t)((first + (s < nb ? s : nb - 1)) * n);
}

// Component comp0 + blockIdx.y of item blockIdx.z, coefficients
// [blockIdx.x span, (blockIdx.x + 1) span): the outputs of k_scale.
__global__ __launch_bounds__(256) void k_scale_mx(DevCtx c, const uint64_t *__restrict__ Dt,
                                                  uint64_t *__restrict__ out, uint64_t *__restrict__ C2, int comp0,
                                                  int span) {
    __shared__ MxShared sh;
    const int n = c.n, k = c.k, kp = c.kp, K = c.K;
    const int comp = comp0 + (int)blockIdx.y;
    const size_t item = blockIdx.z;
    const uint64_t *src = Dt + (item * 3 + comp) * (size_t)K * n;
    uint64_t *dst = comp < 2 ? out + (item * 2 + comp) * (size_t)k * n : C2 + item * (size_t)k * n;
    const int base = (int)blockIdx.x * span;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, col = lane & 15u, g = lane >> 4;
    mx_stage_table(sh, 0, c.mx->a_scale);
    mx_stage_table(sh, 1, c.mx->a_p2q);
    mx_stage_table(sh, 2, c.mx->a_sdp);
    mx_stage_scale_slots(sh, c);
    if (threadIdx.x == 0) sh.count = 0;
    __syncthreads();
    const int a16 = (int)((lane ^ 16u) << 2), a32 = (int)((lane ^ 32u) << 2);
    bool iv[2], jv[2];
    uint32_t rq[2], rp[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int s = (int)g + 4 * h;
        iv[h] = s < k;
        jv[h] = s < kp;
        rq[h] = mx_row(s, k, 0, n);
        rp[h] = mx_row(s, kp, k, n);
    }
    struct Regs {
        uint64_t q[2], p[2];
    };
    auto load = [&](Regs &R, int tile) {
        const uint64_t *t = src + base + tile * 16 + col;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            R.q[h] = t[rq[h]];
            R.p[h] = t[rp[h]];
        }
    };
    auto body = [&](const Regs &R, int tile) {
        const int coef = base + tile * 16 + (int)col;
        uint64_t r[2];
        if (mx_scale_tile(sh, lane, a16, a32, R.q, R.p, jv, r)) {
#pragma unroll
            for (int h = 0; h < 2; h++)
                if (iv[h]) dst[(size_t)(g + 4 * h) * n + coef] = r[h];
        } else if (g == 0) {
            sh.item[atomicAdd(&sh.count, 1)] = coef - base;
        }
    };
    mx_tiles<Regs>((int)wave, span / 16, load, body);
    __syncthreads();
    const int cnt = sh.count;
    for (int e = (int)threadIdx.x; e < cnt; e += 256) {
        const int coef = base + sh.item[e];
        uint64_t dqa[FHE_MX_MAXB], dpa[FHE_MX_MAXB];
#pragma unroll
        for (int i = 0; i < FHE_MX_MAXB; i++) {
            dqa[i] = i < k ? src[(size_t)i * n + coef] : 0;
            dpa[i] = i < kp ? src[(size_t)(k + i) * n + coef] : 0;
        }
        scale_exact<FHE_MX_MAXB, FHE_MX_MAXB, false>(c, dqa, dpa,
                                                      [&](int i, uint64_t r) { dst[(size_t)i * n + coef] = r; });
    }
}

// D of a bridge chain at one prime m (k_scale_chain): the input's tensor t
// plus 2 gamma x~ (g1 = [2 gamma]_m 2^64, a Montgomery multiplier) and, in the
// constant coefficient of component 0 (sq), gamma^2 (g2), in [0, 2m) (one
// conditional subtraction from [0, 4m)): the matrix-core scale takes any
// representative below 2^62 (a Shoup product for the Q side, digits for the
// P side).
__device__ __forceinline__ uint64_t mx_chain_dl(uint64_t t, uint64_t xl, uint64_t g1, uint64_t g2, uint64_t m,
                                                uint64_t mqi, bool sq) {
    uint64_t v = t + mont_mul_lazy(xl, g1, m, mqi);
    if (sq) v += g2;
    return csub(v, m << 1);
}

// The same, canonical (the exact path).
__device__ __forceinline__ uint64_t mx_chain_d(uint64_t t, uint64_t xl, uint64_t g1, uint64_t g2, uint64_t m,
                                               uint64_t mqi, bool sq) {
    return csub(mx_chain_dl(t, xl, g1, g2, m, mqi, sq), m);
}

// k_scale_chain on the matrix cores: component blockIdx.y of chain blockIdx.z
// (register budget of four waves per SIMD).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_scale_chain_mx(DevCtx c, const uint64_t *__restrict__ Dt,
                                                        const uint64_t *__restrict__ x,
                                                        const uint64_t *__restrict__ E,
                                                        const uint64_t *__restrict__ gam,
                                                        const uint64_t *__restrict__ R, uint64_t *__restrict__ y,
                                                        int tcount, int span) {
    __shared__ MxShared sh;
    const int n = c.n, k = c.k, kp = c.kp, K = c.K;
    const int comp = (int)blockIdx.y;
    const size_t chain = blockIdx.z, jin = chain / tcount;
    const ConvConst &cc = *c.cc;
    const uint64_t *src = Dt + (jin * 3 + comp) * (size_t)K * n;
    const uint64_t *xin = x + (jin * 2 + comp) * (size_t)k * n;
    const uint64_t *xp = E + (jin * 2 + comp) * (size_t)K * n;
    const uint64_t *gm = gam + chain * 2 * (size_t)K;
    const uint64_t *rr = R + (jin * 2 + comp) * (size_t)k * n;
    uint64_t *dst = y + (chain * 2 + comp) * (size_t)k * n;
    const int base = (int)blockIdx.x * span;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, col = lane & 15u, g = lane >> 4;
    mx_stage_table(sh, 0, c.mx->a_scale);
    mx_stage_table(sh, 1, c.mx->a_p2q);
    mx_stage_table(sh, 2, c.mx->a_sdp);
    mx_stage_scale_slots(sh, c);
    {
        // the chain's gamma multipliers: Q side words 8, 9, P side words 6, 7
        const int t = (int)threadIdx.x - 2 * FHE_MX_MAXB;
        if (t >= 0 && t < FHE_MX_MAXB) {
            sh.cq[t][8] = t < k ? gm[2 * t] : 0;
            sh.cq[t][9] = t < k ? gm[2 * t + 1] : 0;
        } else if (t >= FHE_MX_MAXB && t < 2 * FHE_MX_MAXB) {
            const int s = t - FHE_MX_MAXB;
            sh.cp[s][6] = s < kp ? gm[2 * (k + s)] : 0;
            sh.cp[s][7] = s < kp ? gm[2 * (k + s) + 1] : 0;
        }
    }
    if (threadIdx.x == 0) sh.count = 0;
    __syncthreads();
    const int a16 = (int)((lane ^ 16u) << 2), a32 = (int)((lane ^ 32u) << 2);
    bool iv[2], jv[2];
    uint32_t rq[2], rp[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int s = (int)g + 4 * h;
        iv[h] = s < k;
        jv[h] = s < kp;
        rq[h] = mx_row(s, k, 0, n);
        rp[h] = mx_row(s, kp, k, n);
    }
    struct Regs {
        uint64_t t[2], x[2], r[2], tp[2], xp[2];
    };
    auto load = [&](Regs &Rg, int tile) {
        const size_t o = (size_t)(base + tile * 16 + (int)col);
#pragma unroll
        for (int h = 0; h < 2; h++) {
            Rg.t[h] = src[o + rq[h]];
            Rg.x[h] = xin[o + rq[h]];
            Rg.r[h] = rr[o + rq[h]];
            Rg.tp[h] = src[o + rp[h]];
            Rg.xp[h] = xp[o + rp[h]];
        }
    };
    auto body = [&](const Regs &Rg, int tile) {
        const int coef = base + tile * 16 + (int)col;
        const bool sq = comp == 0 && coef == 0;
        uint64_t dq[2], dp[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const uint64_t *Q = sh.cq[g + 4 * h], *Pc = sh.cp[g + 4 * h];
            dq[h] = mx_chain_dl(Rg.t[h], Rg.x[h], Q[8], Q[9], Q[0], Q[1], sq);
            dp[h] = mx_chain_dl(Rg.tp[h], Rg.xp[h], Pc[6], Pc[7], Pc[0], Pc[1], sq);
        }
        uint64_t r[2];
        if (mx_scale_tile(sh, lane, a16, a32, dq, dp, jv, r)) {
#pragma unroll
            for (int h = 0; h < 2; h++)
                if (iv[h]) dst[(size_t)(g + 4 * h) * n + coef] = add_mod(r[h], Rg.r[h], sh.cq[g + 4 * h][0]);
        } else if (g == 0) {
            sh.item[atomicAdd(&sh.count, 1)] = coef - base;
        }
    };
    mx_tiles1<Regs>((int)wave, span / 16, load, body);  // five input streams: one tile ahead
    __syncthreads();
    const int cnt = sh.count;
    for (int e = (int)threadIdx.x; e < cnt; e += 256) {
        const int coef = base + sh.item[e];
        const bool sq = comp == 0 && coef == 0;
        uint64_t dqa[FHE_MX_MAXB], dpa[FHE_MX_MAXB];
#pragma unroll
        for (int i = 0; i < FHE_MX_MAXB; i++) {
            dqa[i] = i < k ? mx_chain_d(src[(size_t)i * n + coef], xin[(size_t)i * n + coef], gm[2 * i],
                                        gm[2 * i + 1], cc.q[i], cc.q_qinv[i], sq)
                           : 0;
            dpa[i] = i < kp ? mx_chain_d(src[(size_t)(k + i) * n + coef], xp[(size_t)(k + i) * n + coef],
                                         gm[2 * (k + i)], gm[2 * (k + i) + 1], cc.p[i], cc.p_qinv[i], sq)
                            : 0;
        }
        scale_exact<FHE_MX_MAXB, FHE_MX_MAXB, false>(c, dqa, dpa, [&](int i, uint64_t r) {
            dst[(size_t)i * n + coef] = add_mod(r, rr[(size_t)i * n + coef], cc.q[i]);
        });
    }
}

// k_lift on the matrix cores: poly blockIdx.y of item blockIdx.z.  Slot
// constants: Q side q, [qhat^-1] (Shoup pair), 1/q; P side p, -p^-1 mod 2^64,
// [-q] 2^64, bias removal.
__global__ __launch_bounds__(256) void k_lift_mx(DevCtx c, const uint64_t *__restrict__ a,
                                                 const uint64_t *__restrict__ b, uint64_t *__restrict__ E,
                                                 int npoly, int span) {
    __shared__ MxShared sh;
    const int n = c.n, k = c.k, kp = c.kp, K = c.K;
    const int poly = (int)blockIdx.y;
    const size_t item = blockIdx.z;
    const ConvConst &cc = *c.cc;
    const ConvMx &mx = *c.mx;
    const uint64_t *src = poly < 2 ? a + (item * 2 + poly) * (size_t)k * n
                                   : b + (item * 2 + poly - 2) * (size_t)k * n;
    uint64_t *dst = E + ((item * npoly + poly) * K + k) * (size_t)n;
    const int base = (int)blockIdx.x * span;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, col = lane & 15u, g = lane >> 4;
    mx_stage_table(sh, 0, mx.a_lift);
    {
        const int t = (int)threadIdx.x;
        if (t < FHE_MX_MAXB) {
            const bool ok = t < k;
            sh.cq[t][0] = ok ? cc.q[t] : 0;
            sh.cq[t][1] = ok ? cc.qhinv[t] : 0;
            sh.cq[t][2] = ok ? cc.qhinv_p[t] : 0;
            sh.cq[t][3] = ok ? (uint64_t)__double_as_longlong(cc.inv_q[t]) : 0;
        } else if (t < 2 * FHE_MX_MAXB) {
            const int s = t - FHE_MX_MAXB;
            const bool ok = s < kp;
            sh.cp[s][0] = ok ? cc.p[s] : 0;
            sh.cp[s][1] = ok ? cc.p_qinv[s] : 0;
            sh.cp[s][2] = ok ? mx.l_beta[s] : 0;
            sh.cp[s][3] = ok ? mx.e_lift[s] : 0;
        }
    }
    if (threadIdx.x == 0) sh.count = 0;
    __syncthreads();
    const int a16 = (int)((lane ^ 16u) << 2), a32 = (int)((lane ^ 32u) << 2);
    bool jv[2];
    uint32_t rq[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int s = (int)g + 4 * h;
        jv[h] = s < kp;
        rq[h] = mx_row(s, k, 0, n);
    }
    struct Regs {
        uint64_t x[2];
    };
    auto load = [&](Regs &R, int tile) {
        const uint64_t *t = src + base + tile * 16 + col;
#pragma unroll
        for (int h = 0; h < 2; h++) R.x[h] = t[rq[h]];
    };
    auto body = [&](const Regs &R, int tile) {
        const int coef = base + tile * 16 + (int)col;
        uint64_t yv[2];
        double e = 0.0;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const uint64_t *Q = sh.cq[g + 4 * h];
            yv[h] = mul_shoup(R.x[h], Q[1], Q[2], Q[0]);
            e = fma((double)yv[h], mx_f64(Q[3]), e);
        }
        e = mx_colsum(e, a16, a32);
        const double fl = floor(e), d = e - fl;
        const bool exact = fabs(d - 0.5) < FHE_EST_MARGIN;
        const uint64_t beta = (uint32_t)fl + (d > 0.5 ? 1u : 0u);  // <= k
        mx_v4i acc[4];
        mx_products(sh, 0, lane, mx_operand(yv[0], yv[1]), acc);
        if (!exact) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                if (jv[h]) {
                    const uint64_t *Pc = sh.cp[g + 4 * h];
                    uint64_t lo, hi;
                    mx_recombine(acc[2 * h], acc[2 * h + 1], lo, hi);
                    mx_add(lo, hi, beta * Pc[2], 0);
                    mx_add(lo, hi, Pc[3], 0);
                    dst[(size_t)(g + 4 * h) * n + coef] = mx_reduce(lo, hi, Pc[0], Pc[1]);
                }
            }
        } else if (g == 0) {
            sh.item[atomicAdd(&sh.count, 1)] = coef - base;
        }
    };
    mx_tiles<Regs>((int)wave, span / 16, load, body);
    __syncthreads();
    const int cnt = sh.count;
    for (int e = (int)threadIdx.x; e < cnt; e += 256) {
        const int coef = base + sh.item[e];
        uint64_t xa[FHE_MX_MAXB];
#pragma unroll
        for (int i = 0; i < FHE_MX_MAXB; i++) xa[i] = i < k ? src[(size_t)i * n + coef] : 0;
        lift_exact<FHE_MX_MAXB, FHE_MX_MAXB, false>(c, xa,
                                                     [&](int j, uint64_t r) { dst[(size_t)j * n + coef] = r; });
    }
}

inline int mx_span(int n) { return n < kMxSpan ? n : kMxSpan; }

inline unsigned grid_for(size_t words, unsigned block = 256) {
    size_t g = (words + block - 1) / block;
    if (g > 65536 * 4) g = 65536 * 4;
    if (g == 0) g = 1;
    return (unsigned)g;
}

template <template <int, int, bool> class Launcher, typename... A>
hipError_t by_class(int k, int kp, A... args) {
    if (k == 3 && kp == 3) return Launcher<3, 3, true>::run(args...);
    if (k == 5 && kp == 5) return Launcher<5, 5, true>::run(args...);
    if (k == 8 && kp == 8) return Launcher<8, 8, true>::run(args...);
    if (k <= 4 && kp <= 4) return Launcher<4, 4, false>::run(args...);
    if (k <= 8 && kp <= 8) return Launcher<8, 8, false>::run(args...);
    if (k <= 8 && kp <= 12) return Launcher<8, 12, false>::run(args...);
    if (k <= FHE_MAXK && kp <= FHE_MAXKP) return Launcher<FHE_MAXK, FHE_MAXKP, false>::run(args...);
    return hipErrorInvalidValue;
}

template <int MK, int MKP, bool EX>
struct LiftL {
    static hipError_t run(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *E,
                          int npoly, size_t items, hipStream_t s) {
        dim3 grid((c.n + 255) / 256, npoly, (unsigned)items);
        hipLaunchKernelGGL((k_lift<MK, MKP, EX>), grid, dim3(256), 0, s, c, a, b, E, npoly);
        return hipGetLastError();
    }
};

template <int MK, int MKP, bool EX>
struct ScaleL {
    static hipError_t run(const DevCtx &c, const uint64_t *Dt, uint64_t *out, uint64_t *C2,
                          size_t items, int comp0, int ncomp, hipStream_t s) {
        dim3 grid((c.n + 255) / 256, ncomp, (unsigned)items);
        hipLaunchKernelGGL((k_scale<MK, MKP, EX>), grid, dim3(256), 0, s, c, Dt, out, C2, comp0);
        return hipGetLastError();
    }
};

template <int MK, int MKP, bool EX>
struct GammaL {
    static hipError_t run(const DevCtx &c, const uint64_t *x, const uint64_t *E, uint64_t *gam,
                          size_t chains, int tcount, int c0, hipStream_t s) {
        hipLaunchKernelGGL((k_bridge_gamma<MK, MKP, EX>), dim3((unsigned)((chains + 63) / 64)), dim3(64), 0, s,
                           c, x, E, gam, chains, tcount, c0);
        return hipGetLastError();
    }
};

template <int MK, int MKP, bool EX>
struct ScaleChainL {
    static hipError_t run(const DevCtx &c, const uint64_t *Dt, const uint64_t *x, const uint64_t *E,
                          const uint64_t *gam, const uint64_t *R, uint64_t *y, size_t chains, int tcount,
                          hipStream_t s) {
        dim3 grid((c.n + 255) / 256, 2, (unsigned)chains);
        hipLaunchKernelGGL((k_scale_chain<MK, MKP, EX>), grid, dim3(256), 0, s, c, Dt, x, E, gam, R, y, tcount);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_lift(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *E, int npoly,
                       size_t items, hipStream_t s) {
    if (items == 0) return hipSuccess;
    if (c.mx) {
        const int span = mx_span(c.n);
        hipLaunchKernelGGL(k_lift_mx, dim3(c.n / span, npoly, (unsigned)items), dim3(256), 0, s, c, a, b, E, npoly,
                           span);
        return hipGetLastError();
    }
    return by_class<LiftL>(c.k, c.kp, c, a, b, E, npoly, items, s);
}

hipError_t launch_scale(const DevCtx &c, const uint64_t *Dt, uint64_t *out, uint64_t *C2,
                        size_t items, hipStream_t s, int comp0, int ncomp) {
    if (items == 0) return hipSuccess;
    if (c.mx) {
        const int span = mx_span(c.n);
        hipLaunchKernelGGL(k_scale_mx, dim3(c.n / span, ncomp, (unsigned)items), dim3(256), 0, s, c, Dt, out, C2,
                           comp0, span);
        return hipGetLastError();
    }
    return by_class<ScaleL>(c.k, c.kp, c, Dt, out, C2, items, comp0, ncomp, s);
}

hipError_t launch_bridge_gamma(const DevCtx &c, const uint64_t *x, const uint64_t *E, uint64_t *gam,
                               size_t chains, int tcount, int c0, hipStream_t s) {
    if (chains == 0) return hipSuccess;
    return by_class<GammaL>(c.k, c.kp, c, x, E, gam, chains, tcount, c0, s);
}

hipError_t launch_scale_chain(const DevCtx &c, const uint64_t *Dt, const uint64_t *x, const uint64_t *E,
                              const uint64_t *gam, const uint64_t *R, uint64_t *y, size_t chains, int tcount,
                              hipStream_t s) {
    if (chains == 0) return hipSuccess;
    if (c.mx) {
        const int span = mx_span(c.n);
        hipLaunchKernelGGL(k_scale_chain_mx, dim3(c.n / span, 2, (unsigned)chains), dim3(256), 0, s, c, Dt, x, E,
                           gam, R, y, tcount, span);
        return hipGetLastError();
    }
    return by_class<ScaleChainL>(c.k, c.kp, c, Dt, x, E, gam, R, y, chains, tcount, s);
}

hipError_t launch_decrypt_scale(const DevCtx &c, const uint64_t *X, uint64_t *pt, size_t count,
                                hipStream_t s) {
    if (count == 0) return hipSuccess;
    dim3 grid((c.n + 255) / 256, (unsigned)count);
    if (c.k <= 4) hipLaunchKernelGGL((k_decrypt_scale<4>), grid, dim3(256), 0, s, c, X, pt);
    else if (c.k <= 8) hipLaunchKernelGGL((k_decrypt_scale<8>), grid, dim3(256), 0, s, c, X, pt);
    else hipLaunchKernelGGL((k_decrypt_scale<FHE_MAXK>), grid, dim3(256), 0, s, c, X, pt);
    return hipGetLastError();
}

hipError_t launch_addsub(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *out,
                         size_t nrows, int op, hipStream_t s) {
    const size_t words = nrows * c.n;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_addsub, dim3(grid_for(words)), dim3(256), 0, s, c, a, b, out, words, op);
    return hipGetLastError();
}

hipError_t launch_plain_const(const DevCtx &c, const uint64_t *a, uint64_t *out, size_t count,
                              uint64_t cval, int sign, hipStream_t s) {
    const size_t words = count * 2 * c.k * (size_t)c.n;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_plain_const, dim3(grid_for(words)), dim3(256), 0, s, c, a, out, words, cval,
                       sign);
    return hipGetLastError();
}

hipError_t launch_small_to_rns(const DevCtx &c, const void *v, int is8, uint64_t *out, size_t count,
                               hipStream_t s) {
    const size_t words = count * c.k * (size_t)c.n;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_small_to_rns, dim3(grid_for(words)), dim3(256), 0, s, c, v, is8, out, count);
    return hipGetLastError();
}

hipError_t launch_pointwise_mont(const DevCtx &c, const uint64_t *a, const uint64_t *b, uint64_t *out,
                                 size_t nrows, int bcast, hipStream_t s) {
    const size_t words = nrows * c.n;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pointwise_mont, dim3(grid_for(words)), dim3(256), 0, s, c, a, b, out, words,
                       bcast);
    return hipGetLastError();
}

hipError_t launch_key_b(const DevCtx &c, const uint64_t *prod, const uint64_t *e_rns,
                        const uint64_t *s2, int digit, uint64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_key_b, dim3(grid_for((size_t)c.k * c.n)), dim3(256), 0, s, c, prod, e_rns, s2,
                       digit, out);
    return hipGetLastError();
}

hipError_t launch_encrypt_finish(const DevCtx &c, const uint64_t *prod, const int32_t *e,
                                 const uint64_t *pt, uint64_t *ct, size_t count, hipStream_t s) {
    const size_t words = count * 2 * c.k * (size_t)c.n;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_encrypt_finish, dim3(grid_for(words)), dim3(256), 0, s, c, prod, e, pt, ct,
                       count);
    return hipGetLastError();
}

hipError_t launch_bridge_combine(const DevCtx &c, const uint64_t *y, uint64_t *bits, uint64_t *eq,
                                 size_t count, int tcount, int nbits, int c0, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (nbits > FHE_MAXNB) return hipErrorInvalidValue;
    dim3 grid((c.n + 255) / 256, 2 * c.k, (unsigned)count);
    hipLaunchKernelGGL(k_bridge_combine, grid, dim3(256), 0, s, c, y, bits, eq, tcount, nbits, c0);
    return hipGetLastError();
}

hipError_t launch_horner(const DevCtx &c, const uint64_t *bits, int nbits, uint64_t *out,
                         size_t count, int signed_top, hipStream_t s) {
    const size_t words = count * 2 * c.k * (size_t)c.n;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_horner, dim3(grid_for(words)), dim3(256), 0, s, c, bits, nbits, out, count, signed_top);
    return hipGetLastError();
}

hipError_t launch_validate(const DevCtx &c, const uint64_t *a, size_t nrows, int kmod, int off,
                           unsigned int *flag, hipStream_t s) {
    const size_t words = nrows * c.n;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(grid_for(words)), dim3(256), 0, s, c, a, words, kmod, off, flag);
    return hipGetLastError();
}
