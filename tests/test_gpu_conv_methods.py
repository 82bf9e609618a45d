"""The base conversions of the product on both engines.

FV12's product lifts both inputs from q to the auxiliary basis P (centred),
and rounds t D / q in P before bringing the result back to q; both steps are
base conversions, i.e. sums sum_s x_s W[t][s] modulo each target prime.  The
library runs them on the vector ALU (method 0) or, for bases of at most 8
primes each side, as exact int8 matrix products on the matrix cores (method
1, balanced base-256 digits, int32 sums, one Montgomery reduction).  Every
word of both methods is checked against the oracle, on random inputs, on
inputs built to reach the exact (mixed-radix) path, and through the bridge.
"""
import numpy as np
import pytest

from oracle import bfv
from paper_2204_12201_amd import fhe, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-conv] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fhe.lib()
    return torch.device("cuda:0")


def up(a):
    return fhe.from_numpy_u64(np.asarray(a, dtype=np.uint64), "cuda")


def down(t):
    import torch
    torch.cuda.synchronize()
    return fhe.to_numpy_u64(t)


def setup(n, qs, t, enc, seed):
    P = bfv.Params(n, qs, t, enc)
    km = inputs.key_material(n, qs, seed)
    pk, rlk = bfv.keygen(P, km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    ctx = fhe.Context(n, qs, t, enc)
    rlk_dev = ctx.rlk_import(up(rlk))
    return P, km, pk, rlk, ctx, rlk_dev


def put(P, ct, poly, pos, value):
    for i, qi in enumerate(P.qs):
        ct[poly, i, pos] = np.uint64(value % qi)


CASES = [
    # (n, bits, k, t, encoding)
    (16, 30, 2, 17, "coeff"),        # one tile of 16 coefficients per workgroup
    (64, 50, 1, 17, "coeff"),        # one prime of q
    (256, 36, 3, 65537, "slots"),
    (1024, 55, 8, 17, "coeff"),      # eight primes each side: every lane slot in use
    (2048, 61, 3, 65537, "slots"),   # primes right below 2^61
    (4096, 45, 5, 65537, "slots"),   # several workgroups per row
]


@pytest.mark.parametrize("n,bits,k,t,enc", CASES)
def test_both_methods_all_words(dev, n, bits, k, t, enc):
    qs = bfv.ntt_primes(n, bits, k)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, enc, 31)
    assert ctx.conv_mfma, "the matrix-core conversions apply here and are the default"
    count = 3
    a = inputs.uniform_ciphertexts(n, qs, count, 31, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 31, "b")
    want = [bfv.mul_relin(P, a[j], b[j], rlk) for j in range(count)]
    want_sq = [bfv.mul_relin(P, a[j], a[j], rlk) for j in range(count)]
    for mfma in (True, False):
        say(f"n={n} k={k} kp={ctx.aux_primes} t={t} mfma={mfma}")
        ctx.set_conv_method(mfma)
        assert ctx.conv_mfma == mfma
        out = down(ctx.mul_relin(rlk_d, up(a), up(b)))
        da = up(a)
        sq = down(ctx.mul_relin(rlk_d, da, da))
        for j in range(count):
            assert (out[j] == want[j]).all(), f"product {j} mfma={mfma}"
            assert (sq[j] == want_sq[j]).all(), f"square {j} mfma={mfma}"


def test_method_switch_and_limits(dev):
    """Method 1 is the default where it applies; bases of more than 8 primes
    or primes below 2^20 keep the vector ALU (method 1 is refused); the
    switch goes both ways."""
    ctx = fhe.Context(1024, bfv.ntt_primes(1024, 55, 8), 17, "coeff")
    assert ctx.aux_primes == 8 and ctx.conv_mfma
    ctx.set_conv_method(False)
    assert not ctx.conv_mfma
    ctx.set_conv_method(True)
    assert ctx.conv_mfma
    big = fhe.Context(256, bfv.ntt_primes(256, 55, 16), 65537, "slots")
    assert not big.conv_mfma
    with pytest.raises(fhe.FheError):
        big.set_conv_method(True)
    small = fhe.Context(16, bfv.ntt_primes(16, 19, 2), 17, "coeff")  # primes below 2^19
    assert not small.conv_mfma
    with pytest.raises(fhe.FheError):
        small.set_conv_method(True)
    small.set_conv_method(False)


@pytest.mark.parametrize("mfma", [True, False], ids=["mfma", "valu"])
def test_exact_paths_both_methods(dev, mfma):
    """n = 1024, eight 55-bit primes: coefficients at q/2 (centred lift on its
    boundary) and products whose t D / q sits next to a half-integer (the
    rounding boundary) reach the exact path on either engine; every word
    equals the oracle's and the exact-path counter rises."""
    n, k = 1024, 8
    qs = bfv.ntt_primes(n, 55, k)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 33)
    ctx.set_conv_method(mfma)
    q, t = P.q, P.t
    a = inputs.uniform_ciphertexts(n, qs, 1, 33, "a")[0]
    b = inputs.uniform_ciphertexts(n, qs, 1, 33, "b")[0]
    special = [(q - 1) // 2, (q + 1) // 2, (q - 3) // 2, (q + 3) // 2]
    for j, p in enumerate([0, 1, 15, 16, 17, 511, 1022, 1023]):
        for poly in range(2):
            put(P, a, poly, p, special[(j + poly) % 4])
            put(P, b, poly, (p + 16) % n, special[(j + 2 * poly + 1) % 4])
    c0 = ctx.fallback_count()
    out = down(ctx.mul_relin(rlk_d, up(a[None]), up(b[None])))
    c1 = ctx.fallback_count()
    assert c1 > c0, "lift boundary did not reach the exact path"
    assert (out[0] == bfv.mul_relin(P, a, b, rlk)).all()
    A = np.zeros((2, k, n), dtype=np.uint64)
    B = np.zeros((2, k, n), dtype=np.uint64)
    for m in range(8):
        put(P, A, 0, 16 * m + m, ((2 * m + 1) * q + t) // (2 * t))
    put(P, B, 0, 0, 1)
    A[1] = inputs.uniform_ciphertexts(n, qs, 1, 34, "r")[0][1]
    out2 = down(ctx.mul_relin(rlk_d, up(A[None]), up(B[None])))
    assert ctx.fallback_count() > c1, "rounding boundary did not reach the exact path"
    assert (out2[0] == bfv.mul_relin(P, A, B, rlk)).all()


def test_bridge_both_methods(dev):
    """The bridge (shared first squaring with its chain rounding, then three
    squarings) at n = 256 with eight 55-bit primes, p = 17: both methods give
    the same eq and bit words, equal to the oracle's."""
    n = 256
    qs = bfv.ntt_primes(n, 55, 8)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 35)
    xs = [3, 16, 0]
    r = inputs.encryption_randomness(n, len(xs), 35)
    pts = np.zeros((len(xs), n), dtype=np.uint64)
    pts[:, 0] = xs
    cts = np.stack([bfv.encrypt(P, pk, pts[j], r["u"][j], r["e"][j]) for j in range(len(xs))])
    got = {}
    for mfma in (True, False):
        say(f"bridge n={n} mfma={mfma}")
        ctx.set_conv_method(mfma)
        bits, eq = ctx.bridge_to_bits(rlk_d, up(cts), 5, with_eq=True)
        got[mfma] = (down(bits), down(eq))
    assert (got[True][0] == got[False][0]).all() and (got[True][1] == got[False][1]).all()
    bits, eq = got[True]
    for j in range(len(xs)):
        want_bits, want_eq = bfv.bridge_to_bits(P, cts[j], rlk, 5)
        assert (eq[j] == want_eq).all(), f"eq {j}"
        assert (bits[j] == want_bits).all(), f"bits {j}"


@pytest.mark.parametrize("n,bits,k,nin,nout", [(16, 30, 2, 1, 1), (256, 36, 3, 24, 37), (64, 55, 4, 64, 16),
                                               (64, 61, 2, 65, 5), (1024, 55, 8, 130, 20)])
def test_weighted_sum_both_methods(dev, n, bits, k, nin, nout):
    """Integer-weighted sums with weights in [-127, 127]: the matrix-core path
    (one or several passes of 64 inputs, ragged output tiles) and the vector
    ALU path give the same words, equal to the oracle's on every output."""
    qs = bfv.ntt_primes(n, bits, k)
    P = bfv.Params(n, qs, 17, "coeff")
    ctx = fhe.Context(n, qs, 17, "coeff")
    assert ctx.conv_mfma
    rng = np.random.default_rng(nin * 1000 + nout)
    w = rng.integers(-127, 128, size=(nout, nin)).astype(np.int32)
    w[0, 0] = -127
    if nin > 1:
        w[0, 1] = 127
    x = inputs.uniform_ciphertexts(n, qs, nin, 37, "w")
    xd = up(x)
    got = {}
    for mfma in (True, False):
        say(f"weighted sum n={n} k={k} nin={nin} nout={nout} mfma={mfma}")
        ctx.set_conv_method(mfma)
        got[mfma] = down(ctx.weighted_sum(xd, w))
    assert (got[True] == got[False]).all()
    want = bfv.weighted_sum(P, x, w)
    assert (got[True] == want).all()


def test_square_chain_graph_follows_conv_method(dev):
    """A recorded squaring-chain graph holds the conversion kernels it was
    recorded with; switching the engine drops the context's graphs, so the
    next graph call records the other engine's kernels.  Every replay equals
    the eager chain and the oracle."""
    import torch
    n = 1024
    qs = bfv.ntt_primes(n, 55, 8)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 39)
    count, depth = 6, 2
    x0 = inputs.uniform_ciphertexts(n, qs, count, 39, "x")
    xe = up(x0)
    for _ in range(depth):
        ctx.mul_relin(rlk_d, xe, xe, out=xe)
    want = down(xe)
    y = x0[3]
    for _ in range(depth):
        y = bfv.mul_relin(P, y, y, rlk)
    assert (want[3] == y).all()
    src = up(x0)
    xg = up(x0)
    for mfma in (True, False, True):
        say(f"square_chain graph n={n} mfma={mfma}")
        ctx.set_conv_method(mfma)
        for rep in range(2):
            xg.copy_(src)
            torch.cuda.synchronize()
            ctx.square_chain(rlk_d, xg, depth, graph=True)
            assert (down(xg) == want).all(), (mfma, rep)
