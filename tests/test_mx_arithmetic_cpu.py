"""CPU checks of the integer arithmetic the matrix-core kernels rely on
(no GPU): balanced base-256 digits, the biased int32 partial sums and their
recombination, one Montgomery reduction per output, and the carry-free
recombination of the weighted sums.  Each emulation here is plain Python
integer arithmetic following the kernels' steps; it is compared with the
exact value the step must produce (the exact rounding floor((t D + h) / q),
the centred lift, the exact weighted sum), not with the GPU."""
import random
from fractions import Fraction

from oracle import bfv
from paper_2204_12201_amd import inputs

R = 1 << 64
B8 = 0x8080808080808080
BIAS = 1 << 21  # the kernels' accumulator start


def digits(x):
    """Balanced base-256 digits of x, as the kernels form them: the bytes of
    (x + B) xor B read as signed bytes (64-bit words: valid while x + B <
    2^64; every value the kernels decompose is below 2^62)."""
    assert 0 <= x and x + B8 < (1 << 64)
    y = (x + B8) ^ B8
    return [((y >> (8 * u)) & 0xFF) - (256 if (y >> (8 * u)) & 0x80 else 0) for u in range(8)]


def digit_products(sources, weights, m):
    """P_v = sum_{s,u} d_u(x_s) w_v(W_s 256^u mod m), the int32 sums of one
    target over one block of (source, digit) pairs."""
    out = [0] * 8
    for x, w in zip(sources, weights):
        d = digits(x)
        for u in range(8):
            wd = digits(w * (1 << (8 * u)) % m)
            for v in range(8):
                out[v] += d[u] * wd[v]
    return out


def recombine(P):
    return sum(p << (8 * v) for v, p in enumerate(P))


def mx_reduce(T, m):
    """The kernels' reduction of a tile sum T: one Montgomery step (hi +
    floor(m' m / 2^64) + [lo != 0], m' = lo (-m^-1) mod 2^64) and a single
    conditional subtraction, valid because hi = floor(T / 2^64) stays below
    2^16 (sums below 2^79 plus two 64-bit constants) while m >= 2^20."""
    lo, hi = T % R, T >> 64
    assert hi < (1 << 16)
    mp = lo * ((-pow(m, -1, R)) % R) % R
    r = hi + (mp * m >> 64) + (1 if lo else 0)
    assert r < 2 * m
    return r - m if r >= m else r


def test_balanced_digits_recompose():
    rnd = random.Random(1)
    top = (1 << 64) - 1 - B8  # 0x7F7F7F7F7F7F7F7F, the largest word the form covers
    vals = [0, 1, 127, 128, 255, 256, (1 << 55) - 1, (1 << 61) - 1, (1 << 62) - 1, top]
    vals += [rnd.randrange(1 << 62) for _ in range(2000)]
    for x in vals:
        d = digits(x)
        assert all(-128 <= v <= 127 for v in d)
        assert sum(v << (8 * u) for u, v in enumerate(d)) == x
    # one past it: the 64-bit sum x + B wraps and the form no longer holds
    assert (top + 1 + B8) >> 64 == 1


def _bases():
    n = 16384
    qs = inputs.PRIMES[(16384, 55)]
    ps = bfv.ntt_primes(n, 61, 8)
    q = 1
    for v in qs:
        q *= v
    P = 1
    for v in ps:
        P *= v
    return qs, ps, q, P


def test_scale_with_digit_products_is_exact_rounding():
    """The scale's first conversion as two chained digit-product blocks (the
    y_i, then D_p against a block-diagonal weight), bias 2^21, the overflow
    count v and the constant as extra terms, one Montgomery reduction; then
    P -> Q the same way with beta: equal to floor((t D + h) / q) mod q_i."""
    qs, ps, q, P = _bases()
    t, h = 17, (q - 1) // 2
    bias_total = BIAS * sum(1 << (8 * v) for v in range(8))
    rnd = random.Random(2)
    for trial in range(12):
        D = [0, 1, -1][trial] if trial < 3 else rnd.randrange(-(q * P) // (4 * t), (q * P) // (4 * t))
        C = (t * D + h) // q
        dq = [D % qi for qi in qs]
        dp = [D % pj for pj in ps]
        y = [((t * dq[i] + h) * pow(q // qs[i], -1, qs[i])) % qs[i] for i in range(8)]
        v = int(sum(Fraction(y[i], qs[i]) for i in range(8)))
        z = []
        for j, pj in enumerate(ps):
            phinv = pow((P // pj) % pj, -1, pj)
            W = [(-pow(qs[i], -1, pj)) % pj * phinv * R % pj for i in range(8)]
            Wd = [(t * pow(q % pj, -1, pj) * phinv * R % pj) if s == j else 0 for s in range(8)]
            Pv = [BIAS + a + b for a, b in zip(digit_products(y, W, pj), digit_products(dp, Wd, pj))]
            assert all(0 <= x <= (1 << 22) for x in Pv)
            T = recombine(Pv) + v * (phinv * R % pj) + ((h * pow(q % pj, -1, pj) * phinv * R - bias_total) % pj)
            assert T < pj * R
            zj = T * pow(R, -1, pj) % pj
            assert zj == (C % pj) * phinv % pj
            assert mx_reduce(T, pj) == zj
            z.append(zj)
        beta = round(sum(Fraction(z[j], ps[j]) for j in range(8)))
        for i, qi in enumerate(qs):
            W2 = [(P // ps[j]) % qi * R % qi for j in range(8)]
            Pv = [BIAS + a for a in digit_products(z, W2, qi)]
            T = recombine(Pv) + beta * ((-P) % qi * R % qi) + ((-bias_total) % qi)
            assert T * pow(R, -1, qi) % qi == C % qi
            assert mx_reduce(T, qi) == C % qi


def test_lift_with_digit_products_is_centred_lift():
    qs, ps, q, P = _bases()
    bias_total = BIAS * sum(1 << (8 * v) for v in range(8))
    rnd = random.Random(3)
    for X in [0, 1, q - 1, (q - 1) // 2, (q + 1) // 2] + [rnd.randrange(q) for _ in range(10)]:
        xc = X - q if X > q // 2 else X
        y = [(X % qi) * pow((q // qi) % qi, -1, qi) % qi for qi in qs]
        beta = round(sum(Fraction(y[i], qs[i]) for i in range(8)))
        for j, pj in enumerate(ps):
            W = [(q // qs[i]) % pj * R % pj for i in range(8)]
            Pv = [BIAS + a for a in digit_products(y, W, pj)]
            T = recombine(Pv) + beta * ((-q) % pj * R % pj) + ((-bias_total) % pj)
            assert T * pow(R, -1, pj) % pj == xc % pj
            assert mx_reduce(T, pj) == xc % pj


def test_weighted_sum_recombination_is_exact():
    """Weighted sums: P_u = sum_j w_j d_u(x_j) (|w| <= 127, up to 64 inputs),
    biased; x = P'_0 + 2^8 P'_1 + 2^16 P'_2 + 2^24 P'_3, w likewise from
    P'_4..P'_7; A = floor(x / 2^32) + w, B = x mod 2^32; with E the bias
    removal, (A + E_hi) 2^32 + (B + E_lo) = sum_j w_j x_j mod q."""
    rnd = random.Random(4)
    bias_total = BIAS * sum(1 << (8 * v) for v in range(8))
    for q in [(1 << 61) - 1, bfv.ntt_primes(64, 30, 1)[0], inputs.PRIMES[(16384, 55)][0]]:
        for nin in (1, 24, 64):
            xs = [rnd.randrange(q) for _ in range(nin)]
            ws = [rnd.randint(-127, 127) for _ in range(nin)]
            ws[0] = -127
            Pu = [BIAS] * 8
            for x, w in zip(xs, ws):
                for u, d in enumerate(digits(x)):
                    Pu[u] += w * d
            assert all(0 <= p < (1 << 22) for p in Pu)
            x = Pu[0] + (Pu[1] << 8) + (Pu[2] << 16) + (Pu[3] << 24)
            w = Pu[4] + (Pu[5] << 8) + (Pu[6] << 16) + (Pu[7] << 24)
            assert x < (1 << 47) and w < (1 << 47)
            E = (-bias_total) % q
            A = (x >> 32) + w + (E >> 32)
            Bv = (x & 0xFFFFFFFF) + (E & 0xFFFFFFFF)
            assert (A * (1 << 32) + Bv) % q == sum(a * b for a, b in zip(ws, xs)) % q
