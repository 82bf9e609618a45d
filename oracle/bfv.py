"""Plain CPU oracle for BFV multiply + relinearize and the p-ary bridge.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg may import this module.  It shares no code with the HIP
library: its arithmetic is Python integers plus the textbook C transform in
ref_arith.c.

What it computes (the paper fixes the bridge; it runs BFV through SEAL and says
nothing else about BFV internals, so the scheme is FV12, Fan and Vercauteren,
"Somewhat practical fully homomorphic encryption", the BFV citation of the
paper's introduction):

* Ring R_q = Z_q[X]/(X^n + 1) with q = prod q_i, NTT-friendly primes
  q_i = 1 mod 2n, residue (RNS) form [k][n] per polynomial.
* Keys: s ternary; pk = ([-(a s + e)]_q, a); relinearization digit i
  rlk_i = ([-(a_i s + e_i) + eps_i s^2]_q, a_i), eps_i the CRT idempotent of q_i.
* Enc(m) = ([pk0 u + e1 + Delta m]_q, [pk1 u + e2]_q), Delta = floor(q/t).
* Dec(c) = [round(t [c0 + c1 s]_q / q)]_t.
* Multiply: lift every coefficient to its centred integer, take the exact
  negacyclic products over Z, then C_j = round(t D_j / q) mod q.
* Relinearize: D_i = [C2]_{q_i}; c'_l = C_l + sum_i D_i rlk_i[l] (mod q).
* Bridge (paper, Section 3.2.3, equation for SecureMod -> SecureUint, and the
  pow listing): eq_c = 1 - (x - c)^(t-1) for every c, by the paper's recursive
  repeated-squaring pow; bit j = sum over c in [1, t) with bit j of c set of
  eq_c (the eq_c are one-hot, so the bit-level sum has no carries).
* Recompose (paper, Section 3.2.1, Horner listing): r = b_{S-1}; r = r + r + b_i.
* Weighted sums (the case study's modular stage, Section 4.4): out[m] =
  sum_j w_mj ct_j mod q.  Gates (Section 3.1's expressions over {0, 1}), and
  from them a ripple comparison and a one-hot argmax.
* Bridge from the powers of x (an evaluation of the same bits with fewer
  products): x^1..x^(t-1) by a least-depth product tree, then each bit as a
  weighted sum of the powers with the binomial expansion's weights.
* Signed casts: SecureInt -> SecureMod (Section 3.2.2) as the two's complement
  value, linear; SecureMod -> SecureInt (Section 3.2.4, its equation) as the
  bridge's bits, a constant addition of 2^s - t by a ripple-carry adder of the
  gates, and a MUX on the most significant bit.

Where the paper is silent this oracle takes: Delta = floor(q/t); one key
switching digit per RNS prime, [C2]_{q_i} in [0, q_i), with the CRT idempotent
in the key; sub_plain(c) = c0 - Delta c on the constant coefficient; equality
tests for every c in [0, t) with the bits combining c >= 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import clib

# ----------------------------------------------------------------------------
# Primes and roots (parameter rule: the k largest primes below 2^b that are
# 1 mod 2n, descending; psi_i = x^((q_i - 1)/2n) for the smallest x >= 2 with
# psi_i^n = -1 mod q_i).
# ----------------------------------------------------------------------------

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(m: int) -> bool:
    """Miller-Rabin with the first 12 prime bases: deterministic below 3.3e24."""
    if m < 2:
        return False
    for p in _MR_BASES:
        if m % p == 0:
            return m == p
    d, s = m - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, m)
        if x in (1, m - 1):
            continue
        for _ in range(s - 1):
            x = x * x % m
            if x == m - 1:
                break
        else:
            return False
    return True


def ntt_primes(n: int, bits: int, k: int) -> list:
    """The k largest primes below 2^bits that are 1 mod 2n, descending."""
    step = 2 * n
    c = ((1 << bits) - 2) // step * step + 1
    out = []
    while len(out) < k:
        if c < 2:
            raise ValueError("not enough primes")
        if is_prime(c):
            out.append(c)
        c -= step
    return out


def find_psi(q: int, n: int) -> int:
    """psi = x^((q-1)/2n) mod q for the smallest x >= 2 with psi^n = -1."""
    assert (q - 1) % (2 * n) == 0
    x = 2
    while True:
        psi = pow(x, (q - 1) // (2 * n), q)
        if pow(psi, n, q) == q - 1:
            return psi
        x += 1


def slot_root(t: int, n: int) -> int:
    """psi_t = 3^((t-1)/2n) mod t, the slot-evaluation root for t = 65537."""
    assert (t - 1) % (2 * n) == 0
    return pow(3, (t - 1) // (2 * n), t)


# ----------------------------------------------------------------------------
# Parameters
# ----------------------------------------------------------------------------

@dataclass
class Params:
    n: int
    qs: list
    t: int
    encoding: str = "slots"  # "slots" (t = 1 mod 2n) or "coeff"
    k: int = field(init=False)
    q: int = field(init=False)
    delta: int = field(init=False)
    psis: list = field(init=False)

    def __post_init__(self):
        self.qs = [int(x) for x in self.qs]
        self.k = len(self.qs)
        self.q = math.prod(self.qs)
        self.delta = self.q // self.t
        self.psis = [find_psi(qi, self.n) for qi in self.qs]
        # CRT reconstruction weights: X = sum_i r_i * W_i mod q
        self._crt_w = []
        for qi in self.qs:
            qhat = self.q // qi
            self._crt_w.append(qhat * pow(qhat, -1, qi))


def _obj(a) -> np.ndarray:
    return np.asarray(a).astype(object)


def to_ints(P: Params, rns: np.ndarray) -> np.ndarray:
    """RNS [k][n] -> object array of integers in [0, q) (CRT)."""
    acc = np.zeros(rns.shape[-1], dtype=object)
    for i in range(P.k):
        acc = acc + _obj(rns[i]) * P._crt_w[i]
    return acc % P.q


def centred(P: Params, X: np.ndarray) -> np.ndarray:
    """Map integers in [0, q) to (-q/2, q/2) (q is odd, so no tie)."""
    return np.where(X > (P.q - 1) // 2, X - P.q, X)


def from_ints(P: Params, X) -> np.ndarray:
    """Integers (any sign) -> canonical residues uint64 [k][n]."""
    X = _obj(X)
    return np.stack([(X % qi).astype(np.uint64) for qi in P.qs])


def small_to_rns(P: Params, v) -> np.ndarray:
    return from_ints(P, _obj(np.asarray(v, dtype=np.int64)))


# ----------------------------------------------------------------------------
# Ring products
# ----------------------------------------------------------------------------

def mul_rns(P: Params, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Negacyclic product in R_q, limb by limb (A, B uint64 [k][n])."""
    return clib.polymul_rows(A, B, P.qs, P.psis)


_aux_cache: dict = {}


def _aux_basis(n: int, count: int):
    key = (n, count)
    if key not in _aux_cache:
        ps = ntt_primes(n, 61, count)
        _aux_cache[key] = (ps, [find_psi(p, n) for p in ps])
    return _aux_cache[key]


def mul_int(n: int, A, B, bound: int) -> np.ndarray:
    """Exact negacyclic product over Z of integer polynomials A, B.

    bound must exceed every |coefficient| of the product.  The product is
    taken modulo enough auxiliary 61-bit NTT primes and rebuilt by the CRT.
    """
    count = 1
    while (1 << (60 * count)) <= 2 * bound + 1:
        count += 1
    ps, psis = _aux_basis(n, count)
    M = math.prod(ps)
    assert M > 2 * bound + 1
    A, B = _obj(A), _obj(B)
    ra = np.stack([(A % p).astype(np.uint64) for p in ps])
    rb = np.stack([(B % p).astype(np.uint64) for p in ps])
    rc = clib.polymul_rows(ra, rb, ps, psis)
    acc = np.zeros(n, dtype=object)
    for j, p in enumerate(ps):
        Mj = M // p
        acc = acc + _obj(rc[j]) * (Mj * pow(Mj, -1, p))
    acc = acc % M
    return np.where(acc > M // 2, acc - M, acc)


def schoolbook_negacyclic(A, B, modulus=None):
    """O(n^2) negacyclic product of integer lists (pins only; small n)."""
    n = len(A)
    out = [0] * n
    for i in range(n):
        ai = int(A[i])
        if ai == 0:
            continue
        for j in range(n):
            p = ai * int(B[j])
            if i + j < n:
                out[i + j] += p
            else:
                out[i + j - n] -= p
    if modulus is not None:
        out = [x % modulus for x in out]
    return out


# ----------------------------------------------------------------------------
# Encoding (plaintext polynomials with coefficients in [0, t))
# ----------------------------------------------------------------------------

def encode(P: Params, vals) -> np.ndarray:
    """Slots: m with m(psi_t^(2j+1)) = vals[j] mod t.  Coeff: m = vals."""
    v = np.asarray(vals, dtype=np.uint64) % np.uint64(P.t)
    if P.encoding == "coeff":
        return v.astype(np.uint64)
    psi_t = slot_root(P.t, P.n)
    return clib.ntt_rows(v.reshape(1, -1), [P.t], [psi_t], inverse=True)[0]


def decode(P: Params, pt) -> np.ndarray:
    pt = np.asarray(pt, dtype=np.uint64)
    if P.encoding == "coeff":
        return pt.copy()
    psi_t = slot_root(P.t, P.n)
    return clib.ntt_rows(pt.reshape(1, -1), [P.t], [psi_t])[0]


# ----------------------------------------------------------------------------
# Keys, encryption, decryption
# ----------------------------------------------------------------------------

def _neg_rns(P: Params, A: np.ndarray) -> np.ndarray:
    out = np.empty_like(A)
    for i, qi in enumerate(P.qs):
        out[i] = (np.uint64(qi) - A[i]) % np.uint64(qi)
    return out


def _add_rns(P: Params, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    out = np.empty_like(A)
    for i, qi in enumerate(P.qs):
        out[i] = ((_obj(A[i]) + _obj(B[i])) % qi).astype(np.uint64)
    return out


def _sub_rns(P: Params, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    out = np.empty_like(A)
    for i, qi in enumerate(P.qs):
        out[i] = ((_obj(A[i]) - _obj(B[i])) % qi).astype(np.uint64)
    return out


def keygen(P: Params, s, pk_a, pk_e, rlk_a, rlk_e):
    """Public key [2][k][n] and relinearization key [k digits][2][k][n].

    pk = ([-(a s + e)]_q, a);
    rlk_i = ([-(a_i s + e_i) + eps_i s^2]_q, a_i), eps_i = 1 mod q_i, 0 mod q_j.
    """
    S = small_to_rns(P, s)
    pk_a = np.asarray(pk_a, dtype=np.uint64)
    pk0 = _neg_rns(P, _add_rns(P, mul_rns(P, pk_a, S), small_to_rns(P, pk_e)))
    pk = np.stack([pk0, pk_a])
    S2 = mul_rns(P, S, S)
    rlk = np.empty((P.k, 2, P.k, P.n), dtype=np.uint64)
    for i in range(P.k):
        a_i = np.asarray(rlk_a[i], dtype=np.uint64)
        b = _neg_rns(P, _add_rns(P, mul_rns(P, a_i, S), small_to_rns(P, rlk_e[i])))
        eps_s2 = np.zeros_like(b)
        eps_s2[i] = S2[i]  # eps_i s^2 is s^2 modulo q_i and 0 modulo the other primes
        rlk[i, 0] = _add_rns(P, b, eps_s2)
        rlk[i, 1] = a_i
    return pk, rlk


def encrypt(P: Params, pk: np.ndarray, pt, u, e) -> np.ndarray:
    """([pk0 u + e1 + Delta m]_q, [pk1 u + e2]_q) for pt the plaintext polynomial."""
    U = small_to_rns(P, u)
    dm = from_ints(P, _obj(np.asarray(pt, dtype=np.uint64)) * P.delta)
    c0 = _add_rns(P, _add_rns(P, mul_rns(P, pk[0], U), small_to_rns(P, e[0])), dm)
    c1 = _add_rns(P, mul_rns(P, pk[1], U), small_to_rns(P, e[1]))
    return np.stack([c0, c1])


def phase(P: Params, s, ct: np.ndarray) -> np.ndarray:
    """[c0 + c1 s]_q as integers in [0, q)."""
    S = small_to_rns(P, s)
    return to_ints(P, _add_rns(P, ct[0], mul_rns(P, ct[1], S)))


def decrypt(P: Params, s, ct: np.ndarray) -> np.ndarray:
    """[round(t [c0 + c1 s]_q / q)]_t per coefficient (q odd: no ties)."""
    X = phase(P, s, ct)
    m = (2 * P.t * X + P.q) // (2 * P.q) % P.t
    return m.astype(np.uint64)


def decrypt3(P: Params, s, C) -> np.ndarray:
    """Decryption of a three-component ciphertext: [round(t [C0 + C1 s + C2 s^2]_q / q)]_t."""
    S = small_to_rns(P, s)
    S2 = mul_rns(P, S, S)
    acc = _add_rns(P, _add_rns(P, C[0], mul_rns(P, C[1], S)), mul_rns(P, C[2], S2))
    X = to_ints(P, acc)
    return ((2 * P.t * X + P.q) // (2 * P.q) % P.t).astype(np.uint64)


def noise_ok(P: Params, s, ct: np.ndarray, pt) -> tuple:
    """Noise v = [c0 + c1 s - Delta m]_q (centred) and whether decryption is
    guaranteed correct: |t v - (q mod t) m| < q/2 for every coefficient."""
    X = phase(P, s, ct)
    m = _obj(np.asarray(pt, dtype=np.uint64))
    v = centred(P, (X - P.delta * m) % P.q)
    worst = max(abs(int(x)) for x in (P.t * v - (P.q % P.t) * m))
    vmax = max(abs(int(x)) for x in v)
    return vmax, 2 * worst < P.q


# ----------------------------------------------------------------------------
# Elementwise operations on ciphertexts [2][k][n]
# ----------------------------------------------------------------------------

def add(P: Params, a, b):
    return np.stack([_add_rns(P, a[0], b[0]), _add_rns(P, a[1], b[1])])


def sub(P: Params, a, b):
    return np.stack([_sub_rns(P, a[0], b[0]), _sub_rns(P, a[1], b[1])])


def neg(P: Params, a):
    return np.stack([_neg_rns(P, a[0]), _neg_rns(P, a[1])])


def add_plain(P: Params, a, c: int):
    """c0 + Delta c on the constant coefficient (the constant polynomial c)."""
    out = np.array(a, copy=True)
    for i, qi in enumerate(P.qs):
        out[0, i, 0] = np.uint64((int(a[0, i, 0]) + P.delta * c) % qi)
    return out


def sub_plain(P: Params, a, c: int):
    """c0 - Delta c on the constant coefficient."""
    out = np.array(a, copy=True)
    for i, qi in enumerate(P.qs):
        out[0, i, 0] = np.uint64((int(a[0, i, 0]) - P.delta * c) % qi)
    return out


# ----------------------------------------------------------------------------
# Multiply and relinearize
# ----------------------------------------------------------------------------

def multiply(P: Params, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Tensor then scale: C_j = round(t D_j / q) mod q, returned [3][k][n].

    D0 = A0 B0, D1 = A0 B1 + A1 B0, D2 = A1 B1 over Z[X]/(X^n+1) with A, B the
    centred integer lifts of the inputs.
    """
    A0, A1 = centred(P, to_ints(P, a[0])), centred(P, to_ints(P, a[1]))
    B0, B1 = centred(P, to_ints(P, b[0])), centred(P, to_ints(P, b[1]))
    bound = P.n * ((P.q - 1) // 2) ** 2
    D0 = mul_int(P.n, A0, B0, bound)
    D1 = mul_int(P.n, A0, B1, bound) + mul_int(P.n, A1, B0, bound)
    D2 = mul_int(P.n, A1, B1, bound)
    out = np.empty((3, P.k, P.n), dtype=np.uint64)
    for j, D in enumerate((D0, D1, D2)):
        C = (2 * P.t * D + P.q) // (2 * P.q)
        out[j] = from_ints(P, C)
    return out


def relinearize(P: Params, C: np.ndarray, rlk: np.ndarray) -> np.ndarray:
    """c'_l = C_l + sum_i D_i rlk_i[l] (mod q), D_i = [C2]_{q_i} in [0, q_i)."""
    k = P.k
    rows_a, rows_b, qs, psis = [], [], [], []
    for i in range(k):
        Di = C[2, i].astype(object)  # digit i: the residue of C2 modulo q_i
        for l in range(2):
            for j, qj in enumerate(P.qs):
                rows_a.append((Di % qj).astype(np.uint64))
                rows_b.append(rlk[i, l, j])
                qs.append(qj)
                psis.append(P.psis[j])
    prods = clib.polymul_rows(np.stack(rows_a), np.stack(rows_b), qs, psis)
    prods = prods.reshape(k, 2, k, P.n)
    out = np.empty((2, k, P.n), dtype=np.uint64)
    for l in range(2):
        for j, qj in enumerate(P.qs):
            acc = _obj(C[l, j])
            for i in range(k):
                acc = acc + _obj(prods[i, l, j])
            out[l, j] = (acc % qj).astype(np.uint64)
    return out


class Counter:
    """Counts ciphertext multiplications issued through mul_relin."""

    def __init__(self):
        self.mul = 0


def mul_relin(P: Params, a, b, rlk, counter: Counter | None = None) -> np.ndarray:
    if counter is not None:
        counter.mul += 1
    return relinearize(P, multiply(P, a, b), rlk)


# ----------------------------------------------------------------------------
# Bridge: SecureMod -> SecureUint for a prime plaintext modulus
# ----------------------------------------------------------------------------

def power(P: Params, b, e: int, rlk, counter: Counter | None = None, one=None):
    """Recursive repeated squaring as in the paper's pow listing:
    pow(b, 0) = 1, pow(b, 1) = b, else r = pow(b*b, e >> 1), times b if e odd."""
    if e == 0:
        return one
    if e == 1:
        return b
    r = power(P, mul_relin(P, b, b, rlk, counter), e >> 1, rlk, counter, one)
    if e & 1:
        r = mul_relin(P, r, b, rlk, counter)
    return r


def bridge_eq(P: Params, ct_x: np.ndarray, rlk, c: int, counter: Counter | None = None):
    """eq_c = 1 - (x - c)^(t-1): encrypts 1 if x == c else 0 (t prime)."""
    y = sub_plain(P, ct_x, c)
    y = power(P, y, P.t - 1, rlk, counter)
    return add_plain(P, neg(P, y), 1)


def bridge_bits(P: Params, eqs: list, nbits: int) -> np.ndarray:
    """bit_j = sum_{c in [1, t), (c >> j) & 1} eq_c, returned [nbits][2][k][n]."""
    out = np.zeros((nbits, 2, P.k, P.n), dtype=np.uint64)
    for j in range(nbits):
        for c in range(1, P.t):
            if (c >> j) & 1:
                out[j] = add(P, out[j], eqs[c])
    return out


def bridge_to_bits(P: Params, ct_x, rlk, nbits: int, counter: Counter | None = None):
    """All t equality tests (c = 0..t-1) and the bit combination.

    Returns (bits [nbits][2][k][n], eqs [t][2][k][n])."""
    eqs = [bridge_eq(P, ct_x, rlk, c, counter) for c in range(P.t)]
    return bridge_bits(P, eqs, nbits), np.stack(eqs)


# ----------------------------------------------------------------------------
# Modular linear stage and the bit-level side
# ----------------------------------------------------------------------------

def weighted_sum(P: Params, cts, W) -> np.ndarray:
    """out[m] = sum_j W[m][j] cts[j] (mod q), word by word: the integer-weighted
    sums of the case study's modular stage (paper Section 4.4).  Plain
    definition: Python integers, reduced once per output."""
    X = np.asarray(cts, dtype=np.uint64).astype(object)
    out = np.zeros((len(W), 2, P.k, P.n), dtype=np.uint64)
    for m, row in enumerate(W):
        acc = np.zeros((2, P.k, P.n), dtype=object)
        for j, w in enumerate(row):
            if int(w):
                acc = acc + int(w) * X[j]
        for i, qi in enumerate(P.qs):
            out[m, :, i, :] = np.array([[int(v) % qi for v in acc[l, i]] for l in range(2)],
                                       dtype=np.uint64)
    return out


def gate(P: Params, rlk, op: str, a, b=None, c=None, counter: Counter | None = None):
    """The paper's logic-gate expressions over encrypted bits (Section 3.1):
    AND = ab, NAND = 1 - ab, OR = a + b - ab, NOR = 1 - OR, XOR = a + b - 2ab,
    XNOR = 1 - XOR, NOT = 1 - a, MUX(a, b, c) = a(b - c) + c, each product one
    mul_relin, in this evaluation order."""
    def one_minus(x):
        return add_plain(P, neg(P, x), 1)
    if op == "NOT":
        return one_minus(a)
    if op == "MUX":
        return add(P, mul_relin(P, a, sub(P, b, c), rlk, counter), c)
    p = mul_relin(P, a, b, rlk, counter)
    if op == "AND":
        return p
    if op == "NAND":
        return one_minus(p)
    o = sub(P, add(P, a, b), p)
    if op == "OR":
        return o
    if op == "NOR":
        return one_minus(o)
    x = sub(P, o, p)
    if op == "XOR":
        return x
    if op == "XNOR":
        return one_minus(x)
    raise ValueError(op)


def less_than(P: Params, rlk, a, b, counter: Counter | None = None):
    """[a < b] for bit vectors a, b (least significant first) by the ripple
    circuit of the gates: p = a_i b_i, d = b_i - p (NOT a_i AND b_i),
    e = 1 - ((a_i + b_i) - p - p) (XNOR); lt = d_0, then lt = MUX(e, lt, d)."""
    lt = None
    for i in range(len(a)):
        p = mul_relin(P, a[i], b[i], rlk, counter)
        d = sub(P, b[i], p)
        if i == 0:
            lt = d
            continue
        e = add_plain(P, neg(P, sub(P, sub(P, add(P, a[i], b[i]), p), p)), 1)
        lt = add(P, mul_relin(P, e, sub(P, lt, d), rlk, counter), d)
    return lt


def argmax(P: Params, rlk, scores, counter: Counter | None = None):
    """One-hot argmax of encrypted unsigned scores (ties to the lower class):
    for every pair a < b, l = [s_a < s_b]; class a takes the factor 1 - l and
    class b the factor l, multiplied in as they come."""
    ncls = len(scores)
    out = [None] * ncls
    for a in range(ncls):
        for b in range(a + 1, ncls):
            l = less_than(P, rlk, scores[a], scores[b], counter)
            na = add_plain(P, neg(P, l), 1)
            out[a] = na if out[a] is None else mul_relin(P, out[a], na, rlk, counter)
            out[b] = l if out[b] is None else mul_relin(P, out[b], l, rlk, counter)
    return out


def power_basis(P: Params, ct_x, rlk, e: int, counter: Counter | None = None) -> dict:
    """x^k for k = 1..e, each by one product of lower powers at the least
    depth: x^k = x^h x^(k-h) with h the largest power of two below k (a
    square when k is a power of two); depth ceil(log2 k)."""
    pw = {1: np.array(ct_x, copy=True)}
    for k in range(2, e + 1):
        h = 1 << ((k - 1).bit_length() - 1)
        pw[k] = mul_relin(P, pw[h], pw[k - h], rlk, counter)
    return pw


def bridge_weights(t: int, nbits: int) -> list:
    """The bridge's bits as polynomials in x (mod t): bit_j = sum over c in
    [1, t) with bit j of c set of 1 - (x - c)^(t-1), and (x - c)^(t-1) =
    sum_k C(t-1, k) x^k (-c)^(t-1-k).  Returns W[j][k] (k = 0..t-1, x^0 = 1),
    centred representatives in (-t/2, t/2]."""
    W = []
    for j in range(nbits):
        row = [0] * t
        for c in range(1, t):
            if (c >> j) & 1:
                row[0] += 1
                for k in range(t):
                    row[k] -= math.comb(t - 1, k) * (-c) ** (t - 1 - k)
        row = [w % t for w in row]
        W.append([w - t if w > t // 2 else w for w in row])
    return W


def bridge_to_bits_powers(P: Params, ct_x, rlk, nbits: int, counter: Counter | None = None) -> np.ndarray:
    """The bridge's bits from the powers of x instead of per-test squaring
    chains: the t equality tests share x^1..x^(t-1) (t - 2 products), and
    each bit is one integer-weighted sum of [1, x, ..., x^(t-1)] with the
    weights of bridge_weights (1 = the noiseless encryption (Delta, 0))."""
    pw = power_basis(P, ct_x, rlk, P.t - 1, counter)
    one = np.zeros((2, P.k, P.n), dtype=np.uint64)
    for i, qi in enumerate(P.qs):
        one[0, i, 0] = np.uint64(P.delta % qi)
    return weighted_sum(P, [one] + [pw[k] for k in range(1, P.t)], bridge_weights(P.t, nbits))


def int_to_mod(P: Params, bits) -> np.ndarray:
    """SecureInt -> SecureMod (Section 3.2.2): the two's complement value
    sum_{i < s-1} 2^i x_i - 2^(s-1) x_{s-1}, which modulo t is the paper's
    t - 2^s + sum_i 2^i x_i for a negative x and sum_i 2^i x_i otherwise;
    evaluated linearly as Horner with a negated leading bit:
    r = -x_{s-1}; r = r + r + x_i for i = s-2 .. 0."""
    S = len(bits)
    r = neg(P, bits[S - 1])
    for i in range(S - 2, -1, -1):
        r = add(P, add(P, r, r), bits[i])
    return r


def signed_bits(P: Params, X, rlk, counter: Counter | None = None):
    """The sign adjustment of SecureMod -> SecureInt (Section 3.2.4, its
    equation): from the unsigned bits X (least significant first, 2^s >= t),
    A = X + (2^s - t) in s-bit arithmetic by a ripple-carry adder of the gates
    (constant bit 0: A_i = X_i XOR carry, carry = X_i AND carry; constant bit
    1: A_i = XNOR, carry = OR; a carry known to be zero is not multiplied),
    then Y_i = MUX(X_{s-1}, A_i, X_i) = X_{s-1} (A_i - X_i) + X_i."""
    S = len(X)
    cst = (1 << S) - P.t
    A, carry = [], None
    for i in range(S):
        ci = (cst >> i) & 1
        if carry is None:
            if ci:
                A.append(add_plain(P, neg(P, X[i]), 1))
                carry = np.array(X[i], copy=True)
            else:
                A.append(np.array(X[i], copy=True))
            continue
        p = mul_relin(P, X[i], carry, rlk, counter)
        o = sub(P, add(P, X[i], carry), p)
        x = sub(P, o, p)
        if ci:
            A.append(add_plain(P, neg(P, x), 1))
            carry = o
        else:
            A.append(x)
            carry = p
    msb = X[S - 1]
    return [add(P, mul_relin(P, msb, sub(P, A[i], X[i]), rlk, counter), X[i]) for i in range(S)]


def mod_to_int(P: Params, ct_x, rlk, nbits: int, counter: Counter | None = None):
    """SecureMod -> SecureInt: the bridge's unsigned bits, then signed_bits."""
    X, _ = bridge_to_bits(P, ct_x, rlk, nbits, counter)
    return np.stack(signed_bits(P, list(X), rlk, counter))


def recompose(P: Params, bits) -> np.ndarray:
    """Horner: r = bit_{S-1}; then r = r + r + bit_i for i = S-2 .. 0."""
    S = len(bits)
    r = np.array(bits[S - 1], copy=True)
    for i in range(S - 2, -1, -1):
        r = add(P, add(P, r, r), bits[i])
    return r
