"""CPU check (no GPU) of the column-sum Montgomery product the transform
kernels use for a uniform modulus in their tensor products (mont_mul_lazy_u):
Python integers follow its steps (32-bit halves, multiply-adds with 64-bit
addends, the carry masks of the two sums that may pass 2^64, the zero-word
argument for bits 32..63) and the result is compared with a b 2^-64 mod q by
its definition.  Operands cover the kernels' bounds (below 4 q for primes
below 2^64 / 60, below 2 q for primes below 2^61) and a wider first operand
(below 60 q for moduli below 2^56) that drives the middle column's carry."""
import random

R = 1 << 64
M32 = (1 << 32) - 1


def mont_columns(a, b, q):
    qi = (-pow(q, -1, R)) % R
    a0, a1, b0, b1 = a & M32, a >> 32, b & M32, b >> 32
    q0, q1, qi0, qi1 = q & M32, q >> 32, qi & M32, qi >> 32
    assert a1 + b1 + q1 < (1 << 32)
    P00 = a0 * b0
    Mid = a0 * b1
    P11 = a1 * b1
    Mid += a1 * b0
    assert Mid < R  # first block: no carry kept
    t0, t1 = P00 & M32, ((P00 >> 32) + Mid) & M32
    M = t0 * qi0
    m0, m1 = M & M32, ((M >> 32) + t0 * qi1 + t1 * qi0) & M32
    L = P00 + m0 * q0
    cL, L = L >> 64, L % R
    Mid += m0 * q1
    assert Mid < R  # still no carry before the last term
    H = P11 + m1 * q1
    assert H < R
    Mid += m1 * q0
    cM, Mid = Mid >> 64, Mid % R
    assert cL <= 1 and cM <= 1
    ml, mh = Mid & M32, Mid >> 32
    # bits 32..63 of T + m q vanish: hi(L) + lo(Mid) is 0 or 2^32
    assert ((L >> 32) + ml) & M32 == 0
    r = H + mh + cL + (1 if ml else 0) + (cM << 32)
    assert r < R
    return r


def _check(a, b, q):
    r = mont_columns(a, b, q)
    assert a * b < q * R
    assert r < 2 * q
    assert r % q == a * b * pow(R, -1, q) % q


def _prime_like(rnd, bits):
    # odd moduli of the given size (Montgomery needs q odd; primality is not used)
    return rnd.randrange(1 << (bits - 1), 1 << bits) | 1


def test_wide_first_operand_below_2_56():
    rnd = random.Random(11)
    for _ in range(3000):
        q = _prime_like(rnd, rnd.choice([36, 40, 50, 55, 56]))
        a = rnd.choice([0, 1, 60 * q - 1, rnd.randrange(60 * q)])
        b = rnd.choice([0, q - 1, rnd.randrange(q)])
        _check(a, b, q)


def test_tensor_products_lazy_and_canonical_bounds():
    rnd = random.Random(12)
    top = R // 60
    for _ in range(3000):
        q = rnd.choice([_prime_like(rnd, 58), rnd.randrange(top // 2, top) | 1, _prime_like(rnd, 55)])
        a, b = rnd.randrange(4 * q), rnd.randrange(4 * q)
        _check(a, b, q)
        q = _prime_like(rnd, 61)
        a, b = rnd.choice([2 * q - 1, rnd.randrange(2 * q)]), rnd.choice([2 * q - 1, rnd.randrange(2 * q)])
        _check(a, b, q)
