"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle tests.

This module holds random draws and parameter sets only: no ring arithmetic, no
encryption step, nothing that either the HIP library or the CPU oracle computes.
Both sides receive the draws below as explicit inputs (the secret key, the
uniform key polynomials, the error polynomials, the encryption randomness and
the messages), so a mismatch between them can only come from the arithmetic.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-style: output i of a stream with
key K is mix64(K + (i + 1) * 0x9E3779B97F4A7C15).  Every purpose (secret key,
public-key mask, ...) gets its own stream whose key is derived from
(seed, purpose tag).  This is a benchmark harness, not a secure sampler.

Distributions follow the workload descriptions: secret key and encryption mask
ternary uniform in {-1, 0, 1}; errors a discrete Gaussian with sigma = 3.2 cut at
+-19 (= floor(6 sigma)), sampled by a cumulative-distribution table; uniform
ring elements as uniform residues modulo every RNS prime (uniform modulo q by
the CRT).
"""
from __future__ import annotations

import decimal
import functools

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15

SIGMA = 3.2
GAUSS_TAIL = 19


def _mix64_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def _tag_hash(tag: str) -> int:
    """FNV-1a 64 of the purpose tag: a fixed, documented string-to-integer map."""
    h = 0xCBF29CE484222325
    for byte in tag.encode():
        h ^= byte
        h = (h * 0x100000001B3) & MASK64
    return h


class Stream:
    """One counter-based SplitMix64 stream, keyed by (seed, tag)."""

    def __init__(self, seed: int, tag: str):
        self.key = _mix64_int((seed * GOLDEN_GAMMA) ^ _tag_hash(tag))
        self.pos = 0

    def u64(self, count: int) -> np.ndarray:
        idx = np.arange(self.pos + 1, self.pos + 1 + count, dtype=np.uint64)
        self.pos += count
        with np.errstate(over="ignore"):
            z = np.uint64(self.key) + idx * np.uint64(GOLDEN_GAMMA)
        return _mix64_np(z)

    def _accepting(self, count: int, accept, transform) -> np.ndarray:
        """Rejection sampling: draw blocks, keep accepted draws in order.

        Each block consumes need + need/8 + 16 draws whether or not all are
        used, so the stream position after a call depends only on the draws.
        """
        parts = []
        have = 0
        while have < count:
            need = count - have
            raw = self.u64(need + need // 8 + 16)
            take = raw[accept(raw)][:need]
            parts.append(transform(take))
            have += len(take)
        if not parts:
            return np.empty(0, dtype=np.int64)
        return np.concatenate(parts)

    def uniform_mod(self, q: int, count: int) -> np.ndarray:
        """Uniform in [0, q) by rejection on bit_length(q)-bit masked draws."""
        mask = np.uint64((1 << q.bit_length()) - 1)
        qq = np.uint64(q)
        return self._accepting(count, lambda r: (r & mask) < qq,
                               lambda r: (r & mask)).astype(np.uint64)

    def ternary(self, count: int) -> np.ndarray:
        """Uniform in {-1, 0, 1}: r mod 3 with rejection of the top value."""
        limit = np.uint64(MASK64)  # 2^64 - 1 is a multiple of 3: accept r < it
        lut = np.array([0, 1, -1], dtype=np.int8)
        return self._accepting(count, lambda r: r < limit,
                               lambda r: lut[(r % np.uint64(3)).astype(np.int64)]
                               ).astype(np.int8)

    def gaussian(self, count: int) -> np.ndarray:
        """Discrete Gaussian, sigma 3.2, support [-19, 19], by table lookup."""
        thr = np.array(gaussian_thresholds(), dtype=np.uint64)
        r = self.u64(count)
        return (np.searchsorted(thr, r, side="right") - GAUSS_TAIL).astype(np.int32)


@functools.lru_cache(maxsize=None)
def gaussian_thresholds() -> tuple:
    """Cumulative thresholds T_m = floor(2^64 * P(X <= m)) for m = -19..18.

    A draw r maps to the smallest m with r < T_m (else +19).  Computed once in
    60-digit decimal arithmetic so the table is the same on every machine.
    """
    ctx = decimal.Context(prec=60)
    two_sigma_sq = ctx.multiply(decimal.Decimal(2), ctx.power(decimal.Decimal(str(SIGMA)), 2))
    weights = []
    for m in range(-GAUSS_TAIL, GAUSS_TAIL + 1):
        x = ctx.divide(decimal.Decimal(-m * m), two_sigma_sq)
        weights.append(ctx.exp(x))
    total = sum(weights, decimal.Decimal(0))
    out = []
    acc = decimal.Decimal(0)
    for w in weights[:-1]:
        acc = ctx.add(acc, w)
        out.append(int(ctx.multiply(ctx.divide(acc, total), decimal.Decimal(1 << 64))))
    return tuple(out)


# --------------------------------------------------------------------------
# Parameter sets.  Primes: the k largest primes below 2^b that are 1 mod 2n,
# in descending order (the rule is re-derived and checked by the oracle tests).
# --------------------------------------------------------------------------

PRIMES = {
    # n=4096, 36-bit, k=3
    (4096, 36): [68719403009, 68719230977, 68719206401],
    # n=8192, 43-bit, k=5
    (8192, 43): [8796092858369, 8796092792833, 8796092661761, 8796092399617, 8796091957249],
    # n=16384, 55-bit, k=8
    (16384, 55): [36028797017456641, 36028797016178689, 36028797014704129, 36028797014573057,
                  36028797014376449, 36028797014081537, 36028797013327873, 36028797013098497],
}

T_SLOTS = 65537  # 2^16 + 1: prime, 1 mod 2n for every n <= 2^15
P_BRIDGE = 17    # plaintext prime of the bridge workload

CONFIGS = {
    # plain BFV mul+relin: n=4096, 3 x 36-bit primes, t=65537, 64 products
    "bfv_n4096": dict(n=4096, q=PRIMES[(4096, 36)], t=T_SLOTS, encoding="slots", count=64),
    # bridge: n=16384, 8 x 55-bit primes, p=17, 256 inputs -> 5 bit ciphertexts each
    "bridge_n16384": dict(n=16384, q=PRIMES[(16384, 55)], t=P_BRIDGE, encoding="coeff",
                          count=256, nbits=5),
    # mul+relin at n=16384 with t=65537 (batched vs one-pair-per-call)
    "bfv_n16384": dict(n=16384, q=PRIMES[(16384, 55)], t=T_SLOTS, encoding="slots", count=256),
    "bfv_n8192": dict(n=8192, q=PRIMES[(8192, 43)], t=T_SLOTS, encoding="slots", count=341),
}


# --------------------------------------------------------------------------
# Draws.  Purpose tags fix the draw streams; counts are fixed by n and k.
# --------------------------------------------------------------------------

def key_material(n: int, qs, seed: int) -> dict:
    """Randomness of key generation.

    s      int8[n]        ternary secret key
    pk_a   uint64[k][n]   uniform residues of the public-key mask
    pk_e   int32[n]       public-key error
    rlk_a  uint64[k][k][n] mask of relinearization digit i (uniform mod q)
    rlk_e  int32[k][n]    error of relinearization digit i
    """
    k = len(qs)
    s = Stream(seed, "sk").ternary(n)
    st = Stream(seed, "pk.a")
    pk_a = np.stack([st.uniform_mod(int(q), n) for q in qs])
    pk_e = Stream(seed, "pk.e").gaussian(n)
    rlk_a = np.empty((k, k, n), dtype=np.uint64)
    rlk_e = np.empty((k, n), dtype=np.int32)
    for i in range(k):
        sa = Stream(seed, f"rlk.a.{i}")
        rlk_a[i] = np.stack([sa.uniform_mod(int(q), n) for q in qs])
        rlk_e[i] = Stream(seed, f"rlk.e.{i}").gaussian(n)
    return dict(s=s, pk_a=pk_a, pk_e=pk_e, rlk_a=rlk_a, rlk_e=rlk_e)


def encryption_randomness(n: int, count: int, seed: int, first: int = 0) -> dict:
    """u int8[count][n] ternary, e int32[count][2][n] Gaussian (e1, e2)."""
    u = np.empty((count, n), dtype=np.int8)
    e = np.empty((count, 2, n), dtype=np.int32)
    for j in range(count):
        idx = first + j
        u[j] = Stream(seed, f"enc.u.{idx}").ternary(n)
        e[j, 0] = Stream(seed, f"enc.e1.{idx}").gaussian(n)
        e[j, 1] = Stream(seed, f"enc.e2.{idx}").gaussian(n)
    return dict(u=u, e=e)


def slot_messages(n: int, t: int, count: int, seed: int) -> np.ndarray:
    """count x n plaintext slot values uniform in [0, t)."""
    st = Stream(seed, "msg.slots")
    return st.uniform_mod(t, count * n).reshape(count, n)


def bridge_values(p: int, count: int, seed: int) -> np.ndarray:
    """count values uniform in [0, p), one per bridge input."""
    return Stream(seed, "msg.bridge").uniform_mod(p, count)


def uniform_ciphertexts(n: int, qs, count: int, seed: int, tag: str = "ct") -> np.ndarray:
    """count x 2 x k x n uniform residues: RLWE ciphertexts look uniform mod q."""
    k = len(qs)
    out = np.empty((count, 2, k, n), dtype=np.uint64)
    st = Stream(seed, tag)
    for c in range(count):
        for p in range(2):
            for i, q in enumerate(qs):
                out[c, p, i] = st.uniform_mod(int(q), n)
    return out
