"""GPU parity at the exact paths of the configured parameter sets, the bridge
over several groups, and the launch-shape state of the library.

The base conversions decide an overflow count from a floating-point estimate
and recompute a coefficient exactly (mixed radix) when the estimate is within
2^-40 of a decision boundary.  Uniform inputs reach that path with probability
about 2^-40 per coefficient, so the inputs here are built to sit on the
boundaries (FV12's centred lift and its rounding of t D / q):
  * a coefficient at (q - 1)/2 or (q + 1)/2 (and two steps further) makes the
    centred lift's sum_i y_i / q_i land within 1/(2q) of one half;
  * ct_a = (alpha, 0), ct_b = (1, 0) with alpha = round((2m + 1) q / (2t))
    puts t alpha / q within t/(2q) of the half-integer m + 1/2, the rounding
    boundary of the scale step;
  * in the bridge, an input whose constant coefficient minus Delta c equals
    (q - 1)/2 sends the one-coefficient lift of chain c to the exact path, and
    one whose chain value y satisfies t y^2 / q within 2^-200 of a
    half-integer sends that chain's first rounding to it.
Each case checks every compared word against the oracle and that the
library's exact-path counter rose.
"""
import math

import numpy as np
import pytest

from oracle import bfv
from paper_2204_12201_amd import fhe, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-boundaries] {msg}", flush=True)


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
    """Coefficient `pos` of polynomial `poly` of ct [2][k][n] := value mod q."""
    for i, qi in enumerate(P.qs):
        ct[poly, i, pos] = np.uint64(value % qi)


# The configured parameter sets; each has as many auxiliary primes as Q primes,
# so the library runs its exact-size (k, k) conversion kernels on them.
FULL = [("bfv_n4096", 3), ("bfv_n8192", 5), ("bfv_n16384", 8), ("bridge_n16384", 8)]


@pytest.mark.parametrize("mfma", [True, False], ids=["mfma", "valu"])
@pytest.mark.parametrize("name,k", FULL)
def test_exact_path_at_configured_sizes(dev, name, k, mfma):
    """mfma: the base conversions on the matrix cores (the default at these
    sizes), else the exact-size (k, k) vector ALU kernels."""
    cfg = inputs.CONFIGS[name]
    n, qs, t, enc = cfg["n"], cfg["q"], cfg["t"], cfg["encoding"]
    say(f"exact paths {name}: n={n} k={k} t={t} mfma={mfma}")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, enc, 21)
    assert len(qs) == k and ctx.aux_primes == k, "not the exact-size (k, k) instantiation"
    ctx.set_conv_method(mfma)
    q = P.q
    # -- lift boundary: coefficients around q/2 in both polynomials of both
    #    operands, spread over the row (first, last and interior positions)
    a = inputs.uniform_ciphertexts(n, qs, 1, 21, "a")[0]
    b = inputs.uniform_ciphertexts(n, qs, 1, 21, "b")[0]
    special = [(q - 1) // 2, (q + 1) // 2, (q - 3) // 2, (q + 3) // 2, (q - 5) // 2]
    pos = [0, 1, n // 2, n - 2, n - 1] + [17 * j % n for j in range(3, 40)]
    for j, p in enumerate(pos):
        for poly in range(2):
            put(P, a, poly, p, special[(j + poly) % len(special)])
            put(P, b, poly, (p + 5) % n, special[(j + 2 * poly + 1) % len(special)])
    before = ctx.fallback_count()
    out = down(ctx.mul_relin(rlk_d, up(a[None]), up(b[None])))
    after_lift = ctx.fallback_count()
    assert after_lift > before, "lift boundary did not reach the exact path"
    assert (out[0] == bfv.mul_relin(P, a, b, rlk)).all(), "product with lift-boundary inputs"
    # the squaring kernels on the same input
    da = up(a[None])
    sq = down(ctx.mul_relin(rlk_d, da, da))
    assert ctx.fallback_count() > after_lift
    assert (sq[0] == bfv.mul_relin(P, a, a, rlk)).all(), "square with lift-boundary inputs"
    # -- rounding boundary of the scale step: t alpha / q next to m + 1/2
    alpha = [((2 * m + 1) * q + t) // (2 * t) for m in range(8)]
    for m, al in enumerate(alpha):
        assert abs(2 * t * al - (2 * m + 1) * q) <= t  # t alpha / q within t/(2q) of m + 1/2
    A = np.zeros((2, k, n), dtype=np.uint64)
    B = np.zeros((2, k, n), dtype=np.uint64)
    for m, al in enumerate(alpha):
        put(P, A, 0, 3 * m, al)
    put(P, B, 0, 0, 1)
    # keep the second polynomial of A random so the tensor's other rows are not trivial
    A[1] = inputs.uniform_ciphertexts(n, qs, 1, 22, "r")[0][1]
    c0 = ctx.fallback_count()
    out2 = down(ctx.mul_relin(rlk_d, up(A[None]), up(B[None])))
    assert ctx.fallback_count() > c0, "rounding boundary did not reach the exact path"
    assert (out2[0] == bfv.mul_relin(P, A, B, rlk)).all(), "product on the rounding boundary"


@pytest.mark.parametrize("mfma", [True, False], ids=["mfma", "valu"])
def test_bridge_exact_paths_at_full_size(dev, mfma):
    """The bridge at n = 16384, eight 55-bit primes, p = 17, with two crafted
    inputs: (A) chain c* = 5 whose first rounding sits within 2^-200 of a
    half-integer (exact path of the chain-rounding kernel), (B) an input whose
    constant coefficient minus Delta c' (c' = 11) is (q - 1)/2 (exact path of
    the one-coefficient lift of chain c').  The crafted chains and one other
    chain per input equal the oracle word for word, and every bit ciphertext
    equals the oracle's sum of the library's eq outputs."""
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    say(f"bridge exact paths n=16384 k=8 mfma={mfma}")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "coeff", 23)
    assert ctx.aux_primes == 8
    ctx.set_conv_method(mfma)
    q, D = P.q, P.delta
    cs, cb = 5, 11
    # (A) y = x - Delta c*, centred lift y~ = isqrt((2m+1) q / (2t)), m = 3:
    #     t y~^2 / q = m + 1/2 - O(t y~ / q)
    y = math.isqrt((7 * q) // (2 * t))
    assert 0 < y < q // 2
    fr = (t * y * y) % q
    assert abs(2 * fr - q) < q >> 150, "crafted chain is not on the rounding boundary"
    xa = np.zeros((2, 8, n), dtype=np.uint64)
    put(P, xa, 0, 0, y + D * cs)
    # (B) x0[0] - Delta c' = (q - 1)/2
    xb = np.zeros((2, 8, n), dtype=np.uint64)
    put(P, xb, 0, 0, (q - 1) // 2 + D * cb)
    # a random second polynomial keeps the squarings' tensors full
    xb[1] = inputs.uniform_ciphertexts(n, qs, 1, 24, "r")[0][1]
    xs = np.stack([xa, xb])
    before = ctx.fallback_count()
    bits_a, eq_a = ctx.bridge_to_bits(rlk_d, up(xs[:1]), 5, with_eq=True)
    bits_a, eq_a = down(bits_a), down(eq_a)
    after_a = ctx.fallback_count()
    assert after_a > before, "chain rounding boundary did not reach the exact path"
    bits_b, eq_b = ctx.bridge_to_bits(rlk_d, up(xs[1:]), 5, with_eq=True)
    bits_b, eq_b = down(bits_b), down(eq_b)
    assert ctx.fallback_count() > after_a, "chain lift boundary did not reach the exact path"
    for (x, eq, bits, cset) in ((xa, eq_a[0], bits_a[0], (cs, 0)), (xb, eq_b[0], bits_b[0], (cb, 2))):
        for c in cset:
            assert (eq[c] == bfv.bridge_eq(P, x, rlk, c)).all(), c
        assert (bits == bfv.bridge_bits(P, list(eq), 5)).all()


def test_bridge_several_groups_all_words(dev):
    """The bridge runs its inputs in groups of batch_limit / t; with the limit
    at 34 products (groups of two inputs) three inputs take two groups, the
    second one ragged.  n = 1024, eight 55-bit primes (the exact-size (8, 8)
    kernels), p = 17: every eq and bit word against the oracle, and the same
    words as with the default limit (one group)."""
    n = 1024
    qs = bfv.ntt_primes(n, 55, 8)
    say("bridge n=1024 k=8 in groups of 2")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 25)
    assert ctx.aux_primes == 8
    xs = [16, 0, 9]
    r = inputs.encryption_randomness(n, len(xs), 25)
    pts = np.zeros((len(xs), n), dtype=np.uint64)
    pts[:, 0] = xs
    cts = np.stack([bfv.encrypt(P, pk, pts[j], r["u"][j], r["e"][j]) for j in range(len(xs))])
    whole_bits, whole_eq = ctx.bridge_to_bits(rlk_d, up(cts), 5, with_eq=True)
    whole_bits, whole_eq = down(whole_bits), down(whole_eq)
    ctx.set_batch_limit(34)
    bits, eq = ctx.bridge_to_bits(rlk_d, up(cts), 5, with_eq=True)
    bits, eq = down(bits), down(eq)
    bits_noeq = down(ctx.bridge_to_bits(rlk_d, up(cts), 5))
    ctx.set_batch_limit(0)
    assert (bits == whole_bits).all() and (eq == whole_eq).all()
    assert (bits_noeq == bits).all()
    for j in range(len(xs)):
        want_bits, want_eq = bfv.bridge_to_bits(P, cts[j], rlk, 5)
        assert (eq[j] == want_eq).all(), f"eq {j}"
        assert (bits[j] == want_bits).all(), f"bits {j}"
    dec = ctx.decrypt(km["s"], up(bits.reshape(-1, 2, 8, n))).reshape(len(xs), 5, n)
    for j, x in enumerate(xs):
        assert [int(dec[j, b, 0]) for b in range(5)] == [(x >> b) & 1 for b in range(5)]


def test_square_chain_graph_follows_launch_shape(dev):
    """A recorded squaring-chain graph holds the launch shape it was recorded
    with.  After the batch limit is lowered (and the Python workspace cache is
    released, so a smaller workspace may come back at the same address), the
    next graph call must record a new graph: its words equal the eager chain's
    and the oracle's; the same after a fused-threshold change and after the
    autotuner."""
    import torch
    cfg = inputs.CONFIGS["bfv_n4096"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    say("square_chain graph vs launch-shape setters n=4096")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", 43)
    count, depth = 12, 2
    x0 = inputs.uniform_ciphertexts(n, qs, count, 43, "x")
    xe = up(x0)
    for _ in range(depth):
        ctx.mul_relin(rlk_d, xe, xe, out=xe)
    want = down(xe)
    y = x0[5]
    for _ in range(depth):
        y = bfv.mul_relin(P, y, y, rlk)
    assert (want[5] == y).all()
    xg, src = up(x0), up(x0)
    ctx.square_chain(rlk_d, xg, depth, graph=True)
    assert (down(xg) == want).all(), "first graph"
    for step, change in enumerate((lambda: ctx.set_batch_limit(5),
                                   lambda: ctx.set_fused_threshold(True, 10 ** 9),
                                   lambda: ctx.autotune_mul_relin(rlk_d, src, src),
                                   lambda: ctx.set_batch_limit(0))):
        change()
        ctx._ws.clear()
        torch.cuda.synchronize()
        for rep in range(2):
            xg.copy_(src)
            ctx.square_chain(rlk_d, xg, depth, graph=True)
            assert (down(xg) == want).all(), (step, rep)


def test_multi_rejects_cross_part_overlaps(dev):
    """fhe_mul_relin_multi runs parts concurrently, so one part's output or
    workspace overlapping another part's input, output or workspace is
    rejected (FHE_EINVAL) before anything is enqueued; disjoint parts run."""
    import torch
    cfg = inputs.CONFIGS["bfv_n4096"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", 47)
    a = up(inputs.uniform_ciphertexts(n, qs, 4, 47, "a"))
    b = up(inputs.uniform_ciphertexts(n, qs, 4, 47, "b"))
    need = fhe.lib().fhe_workspace_bytes(ctx._h, fhe.OP_MUL_RELIN, 2)
    ws1 = torch.empty(need, dtype=torch.uint8, device="cuda")
    ws2 = torch.empty(need, dtype=torch.uint8, device="cuda")
    o1, o2 = ctx.empty_ct(2), ctx.empty_ct(2)

    def call(parts):
        arr = (fhe.MulPart * len(parts))()
        for i, (aa, bb, oo, ww, wb) in enumerate(parts):
            arr[i] = fhe.MulPart(ctx._h, fhe._dptr(rlk_d), fhe._dptr(aa), fhe._dptr(bb), fhe._dptr(oo), 2,
                                 fhe._dptr(ww), wb)
        return fhe.lib().fhe_mul_relin_multi(arr, len(parts), fhe._stream())

    # output of part 1 is part 0's input
    assert call([(a[:2], b[:2], o1, ws1, need), (a[2:], b[2:], a[:2], ws2, need)]) == -1
    # workspaces overlap partially
    wsb = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    assert call([(a[:2], b[:2], o1, wsb, need), (a[2:], b[2:], o2, wsb[4096:], need)]) == -1
    # workspace of part 0 overlaps part 1's output (both carved from one buffer,
    # so every address the call could touch is allocated)
    ob = o2.numel() * 8
    carve = torch.empty(need + ob, dtype=torch.uint8, device="cuda")
    o_in_ws = carve[need - 4096:need - 4096 + ob].view(torch.int64).view(2, 2, len(qs), n)
    assert call([(a[:2], b[:2], o1, carve, need), (a[2:], b[2:], o_in_ws, ws2, need)]) == -1
    # the workspace overlapping the part's own operand (fhe_mul_relin too)
    big = ctx.empty_ct(40)
    st = fhe.lib().fhe_mul_relin(ctx._h, fhe._dptr(rlk_d), fhe._dptr(big[:2]), fhe._dptr(b[:2]), fhe._dptr(o1), 2,
                                 fhe._dptr(big), big.numel() * 8, fhe._stream())
    assert st == -1
    # disjoint parts run and match single calls
    assert call([(a[:2], b[:2], o1, ws1, need), (a[2:], b[2:], o2, ws2, need)]) == 0
    ctx.sync()
    assert (down(o1) == down(ctx.mul_relin(rlk_d, a[:2], b[:2]))).all()
    assert (down(o2) == down(ctx.mul_relin(rlk_d, a[2:], b[2:]))).all()


# The largest bases: k = 16 primes of q (the most the library takes) and k = 8
# primes of 61 bits (nine auxiliary primes); the generic conversion kernels
# (16, 20) and (8, 12) run here, and key switching sums 16 digit products
# unreduced (the most its bound allows).
@pytest.mark.parametrize("n,bits,k,t,enc", [(256, 55, 16, 65537, "slots"), (16, 30, 16, 17, "coeff"),
                                            (256, 61, 8, 17, "coeff"), (16384, 55, 16, 65537, "slots")])
def test_largest_bases_all_words(dev, n, bits, k, t, enc):
    qs = bfv.ntt_primes(n, bits, k)
    say(f"largest bases n={n} k={k} {bits}-bit")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, enc, 31)
    assert ctx.aux_primes > 8
    q = P.q
    count = 1 if n == 16384 else 3
    a = inputs.uniform_ciphertexts(n, qs, count, 31, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 31, "b")
    special = [(q - 1) // 2, (q + 1) // 2, (q - 3) // 2]
    for j, pos in enumerate([0, n // 2, n - 1]):
        put(P, a[0], 0, pos, special[j])
        put(P, b[0], 1, pos, special[(j + 1) % 3])
    before = ctx.fallback_count()
    out = down(ctx.mul_relin(rlk_d, up(a), up(b)))
    assert ctx.fallback_count() > before
    da = up(a)
    sq = down(ctx.mul_relin(rlk_d, da, da))
    for j in range(count):
        assert (out[j] == bfv.mul_relin(P, a[j], b[j], rlk)).all(), ("product", j)
    assert (sq[0] == bfv.mul_relin(P, a[0], a[0], rlk)).all(), "square"
