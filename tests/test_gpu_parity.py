"""GPU parity: the HIP library against the CPU oracle, word for word.

Every comparison is exact (integer work): each output uint64 word of the
library must equal the oracle's.  Small sizes compare everything; the full
workload sizes (n = 16384, eight 55-bit primes) compare sampled outputs the
oracle can compute one by one, plus properties that hold at any size.
"""
import os

import numpy as np
import pytest

from oracle import bfv
from paper_2204_12201_amd import fhe, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fhe.lib()  # fails loudly when the HIP library is missing
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


SMALL = [
    # (n, bits, k, t, encoding)
    (16, 30, 2, 17, "coeff"),
    (64, 50, 1, 17, "coeff"),        # one prime: trivial base of Q
    (64, 55, 4, 257, "slots"),
    (256, 36, 3, 65537, "slots"),
    (1024, 55, 8, 17, "coeff"),
    (2048, 61, 3, 65537, "slots"),   # primes right below 2^61
]


# ------------------------------------------------------------- transforms ----

@pytest.mark.parametrize("n,bits,k", [(16, 30, 2), (32, 40, 2), (64, 50, 3), (512, 45, 2),
                                      (1024, 55, 3), (4096, 36, 3), (8192, 43, 2), (16384, 55, 2),
                                      (16384, 61, 1)])
def test_ntt_pinned_order(dev, n, bits, k):
    qs = bfv.ntt_primes(n, bits, k)
    say(f"ntt n={n} k={k} bits={bits}")
    ctx = fhe.Context(n, qs, 17, "coeff")
    rng = np.random.default_rng(n + k)
    count = 3
    polys = np.stack([np.stack([rng.integers(0, q, n, dtype=np.uint64) for q in qs]) for _ in range(count)])
    d = up(polys)
    ctx.ntt(d)
    got = down(d)
    psis = [bfv.find_psi(q, n) for q in qs]
    L = n.bit_length() - 1
    rev = np.array([int(format(j, f"0{L}b")[::-1], 2) for j in range(n)])
    for c in range(count):
        want = bfv.clib.ntt_rows(polys[c], qs, psis)  # natural order A_j
        assert (got[c][:, rev] == want).all(), f"poly {c}"
    ctx.ntt(d, inverse=True)
    assert (down(d) == polys).all()


# -------------------------------------------------------- keys, enc, dec ----

@pytest.mark.parametrize("n,bits,k,t,enc", [(64, 55, 4, 257, "slots"), (4096, 36, 3, 65537, "slots"),
                                            (16384, 55, 8, 17, "coeff")])
def test_keygen_encrypt_decrypt_match_oracle(dev, n, bits, k, t, enc):
    qs = bfv.ntt_primes(n, bits, k)
    say(f"keys n={n} k={k}")
    P = bfv.Params(n, qs, t, enc)
    km = inputs.key_material(n, qs, 21)
    pk, rlk = bfv.keygen(P, km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    ctx = fhe.Context(n, qs, t, enc)
    pk_d, rlk_d = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    assert (down(pk_d) == pk).all()
    assert (down(rlk_d) == down(ctx.rlk_import(up(rlk)))).all()
    count = 2
    vals = inputs.slot_messages(n, t, count, 21)
    pts = np.stack([bfv.encode(P, v) for v in vals])
    assert all((ctx.encode(v) == p).all() for v, p in zip(vals, pts))
    assert all((ctx.decode(p) == v).all() for v, p in zip(vals, pts))
    r = inputs.encryption_randomness(n, count, 21)
    ct_d = ctx.encrypt(pk_d, pts, r["u"], r["e"])
    want = np.stack([bfv.encrypt(P, pk, pts[j], r["u"][j], r["e"][j]) for j in range(count)])
    assert (down(ct_d) == want).all()
    dec = ctx.decrypt(km["s"], ct_d)
    assert (dec == pts).all()
    # decrypt of uniform (non-encryption) words still equals the oracle's rounding
    u = inputs.uniform_ciphertexts(n, qs, 2, 5)
    assert (ctx.decrypt(km["s"], up(u)) == np.stack([bfv.decrypt(P, km["s"], c) for c in u])).all()


# ------------------------------------------------------------ multiply -------

@pytest.mark.parametrize("n,bits,k,t,enc", SMALL)
def test_mul_relin_small_all_words(dev, n, bits, k, t, enc):
    qs = bfv.ntt_primes(n, bits, k)
    say(f"mul_relin small n={n} k={k} t={t}")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, enc, 7)
    count = 5
    a = inputs.uniform_ciphertexts(n, qs, count, 1, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 1, "b")
    out = down(ctx.mul_relin(rlk_d, up(a), up(b)))
    sq = down(ctx.mul_relin(rlk_d, up(a), up(a)))  # distinct buffers: general kernels
    da = up(a)
    sq2 = down(ctx.mul_relin(rlk_d, da, da))  # same buffer: squaring kernels
    for j in range(count):
        want = bfv.mul_relin(P, a[j], b[j], rlk)
        assert (out[j] == want).all(), f"product {j}"
        want_sq = bfv.mul_relin(P, a[j], a[j], rlk)
        assert (sq[j] == want_sq).all() and (sq2[j] == want_sq).all(), f"square {j}"


@pytest.mark.parametrize("n,bits,k", [(1024, 36, 3), (2048, 40, 2), (1024, 60, 2)])
def test_mul_relin_fused_batch_all_words(dev, n, bits, k):
    """Batches large enough for the fused product kernel (and squaring): every
    word of every product against the oracle.  n = 1024 runs the transforms
    with one wave per row (and the LDS prefetch inside that wave), n = 2048
    with two.  60-bit primes take the transforms with every conditional
    subtraction (the others skip them)."""
    qs = bfv.ntt_primes(n, bits, k)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 65537, "slots", 13)
    K = k + ctx.aux_primes
    count = -(-512 // K) + 3
    say(f"mul_relin fused n={n} k={k} K={K} x{count}")
    a = inputs.uniform_ciphertexts(n, qs, count, 13, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 13, "b")
    out = down(ctx.mul_relin(rlk_d, up(a), up(b)))
    da = up(a)
    sq = down(ctx.mul_relin(rlk_d, da, da))
    for j in range(count):
        assert (out[j] == bfv.mul_relin(P, a[j], b[j], rlk)).all(), f"product {j}"
        if j % 7 == 0:
            assert (sq[j] == bfv.mul_relin(P, a[j], a[j], rlk)).all(), f"square {j}"


def test_mul_relin_primes_of_mixed_sizes(dev):
    """Q primes of 55 and 40 bits (more than a factor 4 apart): the key
    switching reduces every digit modulo the target prime before its
    transform; all words of products and squares against the oracle."""
    n = 1024
    qs = bfv.ntt_primes(n, 55, 2) + bfv.ntt_primes(n, 40, 1)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 65537, "slots", 17)
    count = 40
    say(f"mul_relin mixed prime sizes n={n} x{count}")
    a = inputs.uniform_ciphertexts(n, qs, count, 17, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 17, "b")
    out = down(ctx.mul_relin(rlk_d, up(a), up(b)))
    da = up(a)
    sq = down(ctx.mul_relin(rlk_d, da, da))
    for j in range(0, count, 3):
        assert (out[j] == bfv.mul_relin(P, a[j], b[j], rlk)).all(), f"product {j}"
        assert (sq[j] == bfv.mul_relin(P, a[j], a[j], rlk)).all(), f"square {j}"


def test_mul_relin_multi_mixed_sizes(dev):
    """One fhe_mul_relin_multi call over parts of three contexts (n = 4096,
    8192, 16384 with their configured primes, t = 65537; one n=4096 part large
    enough for the fused product kernel): every output equals the single-call
    result word for word, and the first product of each part equals the
    oracle's."""
    import torch
    parts, want_single, oracle_checks = [], [], []
    for key, count, seed in (("bfv_n4096", 40, 31), ("bfv_n8192", 5, 32), ("bfv_n16384", 3, 33),
                             ("bfv_n4096", 6, 34)):
        cfg = inputs.CONFIGS[key]
        n, qs, t = cfg["n"], cfg["q"], cfg["t"]
        P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", seed)
        a = inputs.uniform_ciphertexts(n, qs, count, seed, "a")
        b = inputs.uniform_ciphertexts(n, qs, count, seed, "b")
        da, db = up(a), up(b)
        want_single.append(down(ctx.mul_relin(rlk_d, da, db)))
        parts.append((ctx, rlk_d, da, db, ctx.empty_ct(count)))
        oracle_checks.append((P, a[0], b[0], rlk))
    say("mul_relin_multi n=4096/8192/16384/4096")
    outs = fhe.mul_relin_multi(parts)
    for i, o in enumerate(outs):
        assert (down(o) == want_single[i]).all(), f"part {i}"
        P, a0, b0, rlk = oracle_checks[i]
        assert (want_single[i][0] == bfv.mul_relin(P, a0, b0, rlk)).all(), f"part {i} oracle"
    torch.cuda.synchronize()


def test_mul_relin_multi_persistent_key_switching(dev):
    """Key switching of a multi-part call in one persistent launch: parts of
    n = 16384, 8192 and 4096 whose (item, limb) rows leave workgroup tasks with
    idle sub-groups (5 x 3 rows at n = 4096, 3 x 5 at n = 8192), one squaring
    part; the same words as each part's own call (and the oracle on one product
    per ring size), on three calls in a row (the queue starts from zero each
    time) and with the persistent launch switched off."""
    import torch
    specs = (("bfv_n16384", 2, 71, False), ("bfv_n8192", 3, 72, False), ("bfv_n4096", 5, 73, False),
             ("bfv_n4096", 4, 74, True))
    parts, single, checks = [], [], []
    for key, count, seed, square in specs:
        cfg = inputs.CONFIGS[key]
        n, qs, t = cfg["n"], cfg["q"], cfg["t"]
        P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", seed)
        a = inputs.uniform_ciphertexts(n, qs, count, seed, "a")
        b = a if square else inputs.uniform_ciphertexts(n, qs, count, seed, "b")
        da = up(a)
        db = da if square else up(b)
        single.append(down(ctx.mul_relin(rlk_d, da, db)))
        parts.append((ctx, rlk_d, da, db, ctx.empty_ct(count)))
        checks.append((P, a[count - 1], b[count - 1], rlk))
    say("mul_relin_multi with persistent key switching, n=16384/8192/4096/4096(square)")
    lead = parts[0][0]
    lead.set_multi_persistent(True)
    for rep in range(3):
        for p in parts:
            p[4].fill_(0)
        fhe.mul_relin_multi(parts)
        for i, p in enumerate(parts):
            assert (down(p[4]) == single[i]).all(), (rep, i)
    for i, (P, a1, b1, rlk) in enumerate(checks[:3]):
        assert (single[i][-1] == bfv.mul_relin(P, a1, b1, rlk)).all(), i
    lead.set_multi_persistent(False)
    for p in parts:
        p[4].fill_(0)
    fhe.mul_relin_multi(parts)
    for i, p in enumerate(parts):
        assert (down(p[4]) == single[i]).all(), ("per-stream", i)
    # the autotuner times both modes and keeps one; the words stay the same
    fhe.autotune_mul_relin_multi(parts)
    for p in parts:
        p[4].fill_(0)
    fhe.mul_relin_multi(parts)
    for i, p in enumerate(parts):
        assert (down(p[4]) == single[i]).all(), ("autotuned", i)
    lead.set_multi_persistent(False)
    torch.cuda.synchronize()


def test_square_chain_graph_replays(dev):
    """x^(2^3) by the graph-captured squaring chain equals three eager squarings
    (and the oracle on one ciphertext); the graph is replayed three times on
    reset inputs with unrelated eager work and synchronisation in between."""
    import torch
    cfg = inputs.CONFIGS["bfv_n4096"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", 41)
    count, depth = 8, 3
    x0 = inputs.uniform_ciphertexts(n, qs, count, 41, "x")
    xe = up(x0)
    for _ in range(depth):
        ctx.mul_relin(rlk_d, xe, xe, out=xe)
    want = down(xe)
    y = x0[0]
    for _ in range(depth):
        y = bfv.mul_relin(P, y, y, rlk)
    assert (want[0] == y).all()
    say("square_chain graph n=4096 x8 depth 3")
    xg = up(x0)
    src = up(x0)
    junk = up(inputs.uniform_ciphertexts(n, qs, 2, 42, "j"))
    for rep in range(4):
        xg.copy_(src)
        ctx.add(junk, junk, out=junk)  # eager work between replays
        torch.cuda.synchronize()
        ctx.square_chain(rlk_d, xg, depth, graph=True)
        assert (down(xg) == want).all(), f"graph run {rep}"
    xg.copy_(src)
    ctx.square_chain(rlk_d, xg, depth, graph=False)
    assert (down(xg) == want).all(), "eager chain"


def test_serving_results_identical_alone_and_in_mix(dev):
    """The continuous-batching loop with three kinds arriving interleaved and
    faster than service: products at n = 8192 (five 43-bit primes, t = 65537),
    p = 17 bridge conversions, and imputation queries (one target's 3 class
    scores as weighted sums of 24 resident ciphertexts at t = 65537, then that
    target's 3 class scores at p = 17 bridged to 5 bits and reduced to the
    one-hot argmax).  The p = 17 stages run at n = 1024 (eight 55-bit primes)
    so that the oracle can recompute whole conversions.  Every request's
    result equals the same request computed alone; sampled requests of every
    kind equal the oracle word for word; batches formed and kinds were in
    flight together; the bridged bits and the argmax decrypt to the plain
    values."""
    import torch
    from paper_2204_12201_amd import serving
    c8 = inputs.CONFIGS["bfv_n8192"]
    P8, km8, pk8, rlk8_o, ctx8, rlk8 = setup(c8["n"], c8["q"], c8["t"], "slots", 51)
    nb_n, nb_q = 1024, bfv.ntt_primes(1024, 55, 8)
    Pb, kmb, pkb, rlkb_o, ctxb, rlkb = setup(nb_n, nb_q, 17, "coeff", 52)
    # imputation: modular stage at t = 65537, bit-level stage at p = 17 (own
    # contexts: a lane's workspace is its own)
    Pi = bfv.Params(nb_n, nb_q, 65537, "slots")
    ctxi = fhe.Context(nb_n, nb_q, 65537, "slots")
    P2, km2, pk2, rlk2_o, ctx2, rlk2 = setup(nb_n, nb_q, 17, "coeff", 54)
    nm, nb, ni = 24, 6, 6
    a_h = inputs.uniform_ciphertexts(c8["n"], c8["q"], nm, 51, "a")
    b_h = inputs.uniform_ciphertexts(c8["n"], c8["q"], nm, 51, "b")
    a, b = up(a_h), up(b_h)
    xs = inputs.bridge_values(17, nb, 52)
    r = inputs.encryption_randomness(nb_n, nb, 52)
    pts = np.zeros((nb, nb_n), dtype=np.uint64)
    pts[:, 0] = xs
    xb_h = np.stack([bfv.encrypt(Pb, pkb, pts[j], r["u"][j], r["e"][j]) for j in range(nb)])
    xb = up(xb_h)
    g_h = inputs.uniform_ciphertexts(nb_n, nb_q, 24, 53, "g")
    gi = up(g_h)
    wrng = np.random.default_rng(53)
    W = [wrng.integers(-8, 9, size=(3, 24)).astype(np.int32) for _ in range(ni)]
    sv = inputs.bridge_values(17, 3 * ni, 55).reshape(ni, 3)
    sv[0] = [9, 9, 4]  # a tie at the top (ties go to the lower class)
    r2 = inputs.encryption_randomness(nb_n, 3 * ni, 55)
    sc_h = []
    for q_ in range(ni):
        for cl in range(3):
            pt = np.zeros(nb_n, dtype=np.uint64)
            pt[0] = sv[q_, cl]
            sc_h.append(bfv.encrypt(P2, pk2, pt, r2["u"][3 * q_ + cl], r2["e"][3 * q_ + cl]))
    sc_h = np.stack(sc_h).reshape(ni, 3, 2, 8, nb_n)
    sc = up(sc_h)
    torch.cuda.synchronize()
    reqs = []
    for i in range(ni):
        reqs.append(serving.Request(rid=200 + i, kind="impute", arrival=0.00015 * i + 0.00002, w=W[i], s=sc[i]))
    for i in range(nm):
        reqs.append(serving.Request(rid=i, kind="mul", arrival=0.0001 * i, x=a[i:i + 1], y=b[i:i + 1]))
    for i in range(nb):  # arrivals faster than service: later requests queue and batch
        reqs.append(serving.Request(rid=100 + i, kind="bridge", arrival=0.0002 * i + 0.00005, x=xb[i:i + 1]))
    reqs.sort(key=lambda q: q.arrival)
    srv = serving.Server([serving.Lane("mul", ctx8, rlk8, "mul", max_batch=64),
                          serving.Lane("bridge", ctxb, rlkb, "bridge", max_batch=8, nbits=5),
                          serving.Lane("impute", ctxi, None, "impute", max_batch=16, shared=gi, rows=3,
                                       nbits=5, ctx2=ctx2, rlk2=rlk2)],
                         budget_bytes=32 << 30)
    say("serving loop: 24 products n=8192 + 6 bridge conversions + 6 imputation queries (sums, bridge, argmax)")
    done = srv.run(reqs)
    torch.cuda.synchronize()
    assert len(done) == nm + nb + ni
    assert max(q.batch for q in done) > 1
    assert srv.max_concurrent >= 2
    for q in done:  # alone == in the mix
        if q.kind == "mul":
            assert (down(q.result) == down(ctx8.mul_relin(rlk8, q.x, q.y))).all(), q.rid
        elif q.kind == "impute":
            sums = ctxi.weighted_sum(gi, q.w)
            bits = ctx2.bridge_to_bits(rlk2, q.s, 5)
            hot = ctx2.argmax(rlk2, bits.view(3, 1, 5, 2, 8, nb_n))
            assert (down(q.result[0]) == down(sums)).all(), q.rid
            assert (down(q.result[1]) == down(hot)[:, 0]).all(), q.rid
        else:
            assert (down(q.result) == down(ctxb.bridge_to_bits(rlkb, q.x, 5))).all(), q.rid
    # sampled requests of every kind against the oracle
    by = {q.rid: q for q in done}
    for i in (0, 11, 23):
        assert (down(by[i].result)[0] == bfv.mul_relin(P8, a_h[i], b_h[i], rlk8_o)).all(), i
    for i in (0, nb - 1):
        want, _ = bfv.bridge_to_bits(Pb, xb_h[i], rlkb_o, 5)
        assert (down(by[100 + i].result)[0] == want).all(), i
    for i in (0, 3):
        q = by[200 + i]
        assert (down(q.result[0]) == bfv.weighted_sum(Pi, g_h, W[i])).all(), i
        bits_o = [bfv.bridge_to_bits(P2, sc_h[i, cl], rlk2_o, 5)[0] for cl in range(3)]
        want = bfv.argmax(P2, rlk2_o, [list(bo) for bo in bits_o])
        hot = down(q.result[1])
        for cl in range(3):
            assert (hot[cl] == want[cl]).all(), (i, cl)
    # decryptions: bits of x, and the one-hot argmax of the class scores
    dec = ctxb.decrypt(kmb["s"], torch.cat([q.result for q in done if q.kind == "bridge"]).reshape(-1, 2, 8, nb_n))
    got = dec.reshape(nb, 5, nb_n)[:, :, 0]
    order = [q.rid - 100 for q in done if q.kind == "bridge"]
    for row, i in zip(got, order):
        assert [int(v) for v in row] == [(int(xs[i]) >> bit) & 1 for bit in range(5)], i
    for q in done:
        if q.kind != "impute":
            continue
        i = q.rid - 200
        best = max(range(3), key=lambda cl: (int(sv[i, cl]), -cl))
        d = ctx2.decrypt(km2["s"], q.result[1].contiguous())
        assert [int(v) for v in d[:, 0]] == [int(cl == best) for cl in range(3)], i


def test_exact_path_boundary_inputs(dev):
    """Coefficients on the centring boundary (q-1)/2, (q+1)/2 and products whose
    t D / q sits next to a half-integer force the exact mixed-radix path; the
    words must still equal the oracle's."""
    n = 64
    qs = bfv.ntt_primes(n, 55, 4)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 9)
    q = P.q
    before = ctx.fallback_count()
    special = [(q - 1) // 2, (q + 1) // 2, 0, q - 1, 1, (q - 3) // 2, (q + 3) // 2]
    vals = [special[i % len(special)] for i in range(n)]
    rot = vals[3:] + vals[:3]
    a = np.stack([bfv.from_ints(P, vals), bfv.from_ints(P, rot)])[None]
    alpha = [((2 * m + 1) * q + P.t) // (2 * P.t) for m in range(4)]
    a2 = np.stack([bfv.from_ints(P, alpha + [0] * (n - 4)), bfv.from_ints(P, [0] * n)])[None]
    one = np.stack([bfv.from_ints(P, [1] + [0] * (n - 1)), bfv.from_ints(P, [0] * n)])[None]
    A = np.concatenate([a, a2])
    B = np.concatenate([a[:, ::-1].copy(), one])
    out = down(ctx.mul_relin(rlk_d, up(A), up(B)))
    for j in range(2):
        assert (out[j] == bfv.mul_relin(P, A[j], B[j], rlk)).all(), j
    assert ctx.fallback_count() > before


def test_mul_relin_plain_bfv_n4096_workload(dev):
    """n=4096, three 36-bit primes, t=65537: 64 products of fresh encryptions,
    every word against the oracle, and decryption equal to a*b mod t."""
    cfg = inputs.CONFIGS["bfv_n4096"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    count = cfg["count"]
    say("mul_relin n=4096 k=3 x64")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", 0)
    msgs = inputs.slot_messages(n, t, 2 * count, 0)
    r = inputs.encryption_randomness(n, 2 * count, 0)
    pts = np.stack([bfv.encode(P, m) for m in msgs])
    cts = np.stack([bfv.encrypt(P, pk, pts[j], r["u"][j], r["e"][j]) for j in range(2 * count)])
    out = down(ctx.mul_relin(rlk_d, up(cts[:count]), up(cts[count:])))
    for j in range(count):
        want = bfv.mul_relin(P, cts[j], cts[count + j], rlk)
        assert (out[j] == want).all(), f"product {j}"
    dec = ctx.decrypt(km["s"], up(out))
    for j in range(count):
        prod = msgs[j].astype(object) * msgs[count + j].astype(object) % t
        assert (ctx.decode(dec[j]).astype(object) == prod).all(), j


def test_mul_relin_n8192_k5_sampled(dev):
    cfg = inputs.CONFIGS["bfv_n8192"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    say("mul_relin n=8192 k=5 x9 (3 compared)")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", 2)
    a = inputs.uniform_ciphertexts(n, qs, 9, 2, "a")
    b = inputs.uniform_ciphertexts(n, qs, 9, 2, "b")
    out = down(ctx.mul_relin(rlk_d, up(a), up(b)))
    for j in (0, 4, 8):
        assert (out[j] == bfv.mul_relin(P, a[j], b[j], rlk)).all(), j


def test_mul_relin_n16384_batched_equals_single(dev):
    """n=16384, eight 55-bit primes, t=65537: two products against the oracle;
    one batched call equals eight single-pair calls word for word, and a
    repeated call is bitwise identical (determinism)."""
    cfg = inputs.CONFIGS["bfv_n16384"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    say("mul_relin n=16384 k=8 batched vs single")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", 3)
    B = 8
    a = inputs.uniform_ciphertexts(n, qs, B, 3, "a")
    b = inputs.uniform_ciphertexts(n, qs, B, 3, "b")
    da, db = up(a), up(b)
    batched = down(ctx.mul_relin(rlk_d, da, db))
    again = down(ctx.mul_relin(rlk_d, da, db))
    assert (batched == again).all()
    single = np.stack([down(ctx.mul_relin(rlk_d, da[j:j + 1].contiguous(), db[j:j + 1].contiguous()))[0]
                       for j in range(B)])
    assert (batched == single).all()
    for j in (0, B - 1):
        assert (batched[j] == bfv.mul_relin(P, a[j], b[j], rlk)).all(), j
    # chunked execution (batch limit 3 < 8) gives the same words
    ctx.set_batch_limit(3)
    assert (down(ctx.mul_relin(rlk_d, da, db)) == batched).all()


@pytest.mark.parametrize("cfg_name,count", [("bfv_n16384", 17), ("bfv_n8192", 57), ("bfv_n4096", 181)])
def test_products_resident_grid_ragged(dev, cfg_name, count):
    """Squarings and products whose (item, limb) tasks outnumber the
    workgroups the chip holds, by a count that is not a multiple of them: the
    resident grids of the squaring and product kernels, where some workgroups
    take one task more than others and load each next task's rows during the
    previous one.  Every word of the batched calls equals the same squaring or
    product done one ciphertext per call (one task per workgroup, or the
    unfused kernels), and the first and last items equal the oracle."""
    cfg = inputs.CONFIGS[cfg_name]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "slots", 5)
    K = len(qs) + ctx.aux_primes
    say(f"resident grids n={n} K={K} x{count} ({K * count} tasks)")
    a = inputs.uniform_ciphertexts(n, qs, count, 5, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 5, "b")
    da, db = up(a), up(b)
    sq = down(ctx.mul_relin(rlk_d, da, da))
    pr = down(ctx.mul_relin(rlk_d, da, db))
    for j in range(count):
        dj, ej = up(a[j:j + 1]), up(b[j:j + 1])
        assert (down(ctx.mul_relin(rlk_d, dj, dj))[0] == sq[j]).all(), f"square {j}"
        assert (down(ctx.mul_relin(rlk_d, dj, ej))[0] == pr[j]).all(), f"product {j}"
    for j in (0, count - 1):
        assert (sq[j] == bfv.mul_relin(P, a[j], a[j], rlk)).all(), f"oracle square {j}"
        assert (pr[j] == bfv.mul_relin(P, a[j], b[j], rlk)).all(), f"oracle product {j}"


# ----------------------------------------------------------- elementwise ----

def test_elementwise_ops(dev):
    n = 256
    qs = bfv.ntt_primes(n, 55, 3)
    P = bfv.Params(n, qs, 17, "coeff")
    ctx = fhe.Context(n, qs, 17, "coeff")
    say("elementwise n=256")
    a = inputs.uniform_ciphertexts(n, qs, 3, 8, "a")
    b = inputs.uniform_ciphertexts(n, qs, 3, 8, "b")
    da, db = up(a), up(b)
    assert (down(ctx.add(da, db)) == np.stack([bfv.add(P, x, y) for x, y in zip(a, b)])).all()
    assert (down(ctx.sub(da, db)) == np.stack([bfv.sub(P, x, y) for x, y in zip(a, b)])).all()
    assert (down(ctx.neg(da)) == np.stack([bfv.neg(P, x) for x in a])).all()
    for c in (0, 1, 16):
        assert (down(ctx.add_plain(da, c)) == np.stack([bfv.add_plain(P, x, c) for x in a])).all()
        assert (down(ctx.sub_plain(da, c)) == np.stack([bfv.sub_plain(P, x, c) for x in a])).all()
    bits = inputs.uniform_ciphertexts(n, qs, 2 * 5, 8, "bits").reshape(2, 5, 2, 3, n)
    got = down(ctx.bits_to_mod(up(bits.reshape(2, 5, 2, 3, n))))
    for j in range(2):
        assert (got[j] == bfv.recompose(P, list(bits[j]))).all()
    # in place
    ctx.add(da, db, out=da)
    assert (down(da) == np.stack([bfv.add(P, x, y) for x, y in zip(a, b)])).all()


# ----------------------------------------------------------------- bridge ----

def test_bridge_small_all_words(dev):
    """t = 17 at n = 64 (four 55-bit primes): every eq_c and bit word against
    the oracle; decrypted bits are the plain bits of x and recompose to x."""
    n = 64
    qs = bfv.ntt_primes(n, 55, 4)
    say("bridge n=64")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 11)
    xs = [0, 16, 5, 9]
    r = inputs.encryption_randomness(n, len(xs), 11)
    pts = np.zeros((len(xs), n), dtype=np.uint64)
    pts[:, 0] = xs
    cts = np.stack([bfv.encrypt(P, pk, pts[j], r["u"][j], r["e"][j]) for j in range(len(xs))])
    bits, eq = ctx.bridge_to_bits(rlk_d, up(cts), 5, with_eq=True)
    bits, eq = down(bits), down(eq)
    for j, x in enumerate(xs):
        want_bits, want_eq = bfv.bridge_to_bits(P, cts[j], rlk, 5)
        assert (eq[j] == want_eq).all(), f"eq {j}"
        assert (bits[j] == want_bits).all(), f"bits {j}"
    dec = ctx.decrypt(km["s"], up(bits.reshape(-1, 2, 4, n))).reshape(len(xs), 5, n)
    for j, x in enumerate(xs):
        assert [int(dec[j, b, 0]) for b in range(5)] == [(x >> b) & 1 for b in range(5)]
        assert (dec[j, :, 1:] == 0).all()
    rec = ctx.bits_to_mod(up(bits))
    assert [int(v) for v in ctx.decrypt(km["s"], rec)[:, 0]] == xs
    # without eq outputs the c = 0 test is skipped: same bits
    assert (down(ctx.bridge_to_bits(rlk_d, up(cts), 5)) == bits).all()


def test_bridge_full_size_sampled(dev):
    """The bridge workload: n = 16384, eight 55-bit primes, p = 17.  A batch of
    32 encrypted inputs: sampled equality chains against the oracle word for
    word, every bit ciphertext equal to the sum of its eq_c (checked with the
    oracle's addition), and every decrypted bit equal to the plain bit."""
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    say("bridge n=16384 k=8 x32")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "coeff", 0)
    count = 32
    xs = inputs.bridge_values(t, count, 0)
    pk_d = up(pk)
    pts = np.zeros((count, n), dtype=np.uint64)
    pts[:, 0] = xs
    r = inputs.encryption_randomness(n, count, 0)
    ct_d = ctx.encrypt(pk_d, pts, r["u"], r["e"])
    cts = down(ct_d)
    bits, eq = ctx.bridge_to_bits(rlk_d, ct_d, 5, with_eq=True)
    bits_h, eq_h = down(bits), down(eq)
    assert (down(ctx.bridge_to_bits(rlk_d, ct_d, 5)) == bits_h).all()  # c = 0 skipped
    for (j, c) in [(0, int(xs[0])), (1, (int(xs[1]) + 3) % t)]:
        assert (eq_h[j, c] == bfv.bridge_eq(P, cts[j], rlk, c)).all(), (j, c)
    for j in (0, 7):
        want = bfv.bridge_bits(P, list(eq_h[j]), 5)
        assert (bits_h[j] == want).all(), j
    dec = ctx.decrypt(km["s"], bits.reshape(-1, 2, len(qs), n)).reshape(count, 5, n)
    bad = [j for j in range(count)
           if [int(dec[j, b, 0]) for b in range(5)] != [(int(xs[j]) >> b) & 1 for b in range(5)]]
    if bad:  # name the chains that differ from the oracle before failing
        j = bad[0]
        wrong = [c for c in range(t) if not (eq_h[j, c] == bfv.bridge_eq(P, cts[j], rlk, c)).all()]
        pytest.fail(f"items {bad} decrypt wrong; item {j} (x = {int(xs[j])}) chains {wrong} differ")


# ------------------------------------------------------------------ edges ----

def test_edge_cases(dev):
    import torch
    n = 64
    qs = bfv.ntt_primes(n, 55, 3)
    say("edge cases")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 13)
    a = inputs.uniform_ciphertexts(n, qs, 2, 13, "a")
    b = inputs.uniform_ciphertexts(n, qs, 2, 13, "b")
    da, db = up(a), up(b)
    # count 0 is a no-op
    empty = ctx.empty_ct(0)
    assert ctx.mul_relin(rlk_d, empty, empty).shape[0] == 0
    # in place: out == a
    ctx.mul_relin(rlk_d, da, db, out=da)
    assert (down(da) == np.stack([bfv.mul_relin(P, a[j], b[j], rlk) for j in range(2)])).all()
    # workspace too small
    ws = torch.empty(8, dtype=torch.uint8, device="cuda")
    out = ctx.empty_ct(2)
    st = fhe.lib().fhe_mul_relin(ctx._h, fhe._dptr(rlk_d), fhe._dptr(db), fhe._dptr(db), fhe._dptr(out), 2,
                                 fhe._dptr(ws), 8, fhe._stream())
    assert st == -8
    # partial overlap rejected
    big = ctx.empty_ct(3)
    st = fhe.lib().fhe_add(ctx._h, fhe._dptr(big), fhe._dptr(big), fhe._dptr(big[1:]), 2, fhe._stream())
    assert st == -1
    # bridge needs coefficient encoding with t - 1 a power of two
    ctx2 = fhe.Context(n, qs, 257, "slots")
    with pytest.raises(fhe.FheError) as ei:
        ctx2.bridge_to_bits(rlk_d, db, 9)
    assert ei.value.status == -7
    with pytest.raises(fhe.FheError) as ei:
        ctx.bridge_to_bits(rlk_d, db, 4)  # 2^4 < 17
    assert ei.value.status == -1


def test_validate_flags_noncanonical(dev):
    n = 64
    qs = bfv.ntt_primes(n, 55, 3)
    os.environ["FHE_VALIDATE"] = "1"
    try:
        ctx = fhe.Context(n, qs, 17, "coeff")
    finally:
        del os.environ["FHE_VALIDATE"]
    a = inputs.uniform_ciphertexts(n, qs, 1, 2, "a")
    a[0, 1, 2, 5] = np.uint64(qs[2])  # one word equal to its prime
    with pytest.raises(fhe.FheError) as ei:
        ctx.add(up(a), up(a))
    assert ei.value.status == -6


# ------------------------------------- modular linear stage, bit-level side --

@pytest.mark.parametrize("n,bits,k,nin,nout", [(256, 36, 3, 24, 5), (64, 55, 4, 40, 70), (16, 61, 2, 1, 3)])
def test_weighted_sum_all_words(dev, n, bits, k, nin, nout):
    """Every word of every weighted sum against the oracle: weights uniform in
    [-8, 8] plus edge rows (all +8, all -8, zero, one weight near the row
    limit); 40 inputs take two passes, 70 outputs two workgroup rows."""
    qs = bfv.ntt_primes(n, bits, k)
    say(f"weighted_sum n={n} k={k} nin={nin} nout={nout}")
    P = bfv.Params(n, qs, 65537 if n >= 64 else 17, "coeff")
    ctx = fhe.Context(n, qs, P.t, "coeff")
    x = inputs.uniform_ciphertexts(n, qs, nin, 41, "x")
    rng = np.random.default_rng(nin * 1000 + nout)
    W = rng.integers(-8, 9, size=(nout, nin)).astype(np.int32)
    W[0, :] = 8
    W[1 % nout, :] = -8
    if nout > 2:
        W[2, :] = 0
        W[2, nin - 1] = -(1 << 30) + 1
    got = down(ctx.weighted_sum(up(x), W))
    want = bfv.weighted_sum(P, x, W.tolist())
    for m in range(nout):
        assert (got[m] == want[m]).all(), f"output {m}"


def test_weighted_sum_limits_and_empty(dev):
    n = 64
    qs = bfv.ntt_primes(n, 55, 2)
    ctx = fhe.Context(n, qs, 65537, "coeff")
    x = up(inputs.uniform_ciphertexts(n, qs, 2, 42, "x"))
    with pytest.raises(fhe.FheError) as ei:
        ctx.weighted_sum(x, np.array([[1 << 29, 1 << 29]], dtype=np.int32))  # row sum 2^30
    assert ei.value.status == -1
    out = ctx.weighted_sum(x[:0], np.zeros((3, 0), dtype=np.int32))
    assert (down(out) == 0).all()


def test_weighted_sum_imputation_shape_sampled(dev):
    """The imputation-shaped stage at full size (n = 16384, eight 55-bit
    primes, 24 inputs, 1500 outputs) on sampled words."""
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs = cfg["n"], cfg["q"]
    ctx = fhe.Context(n, qs, 65537, "slots")
    nin, nout = 24, 1500
    say(f"weighted_sum imputation shape {nout}x{nin}")
    x = inputs.uniform_ciphertexts(n, qs, nin, 43, "g")
    W = np.random.default_rng(43).integers(-8, 9, size=(nout, nin)).astype(np.int32)
    import torch
    got_d = ctx.weighted_sum(up(x), W)
    rng = np.random.default_rng(44)
    idx = [rng.integers(nout, size=400), rng.integers(2, size=400), rng.integers(len(qs), size=400),
           rng.integers(n, size=400)]
    got = fhe.to_numpy_u64(got_d[tuple(torch.as_tensor(v, device=got_d.device) for v in idx)].contiguous())
    for s_, (m, pl, i, cf) in enumerate(zip(*[v.tolist() for v in idx])):
        want = sum(int(W[m, j]) * int(x[j, pl, i, cf]) for j in range(nin)) % qs[i]
        assert int(got[s_]) == want, (m, pl, i, cf)


@pytest.mark.parametrize("n,bits,k", [(64, 55, 3), (256, 40, 2)])
def test_gates_all_words(dev, n, bits, k):
    """All eight gates against the oracle on uniform ciphertexts (the words
    are defined for any input), including an output aliasing its input."""
    qs = bfv.ntt_primes(n, bits, k)
    say(f"gates n={n} k={k}")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 45)
    count = 3
    a = inputs.uniform_ciphertexts(n, qs, count, 45, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 45, "b")
    c = inputs.uniform_ciphertexts(n, qs, count, 45, "c")
    for op in fhe.GATES:
        got = down(ctx.gate(rlk_d, op, up(a), up(b), up(c)))
        for j in range(count):
            assert (got[j] == bfv.gate(P, rlk, op, a[j], b[j], c[j])).all(), (op, j)
    da = up(a)
    ctx.gate(rlk_d, "XOR", da, up(b), out=da)
    assert (down(da)[1] == bfv.gate(P, rlk, "XOR", a[1], b[1])).all()


def test_less_than_and_argmax_all_words(dev):
    """Comparison and three-class argmax against the oracle on uniform
    ciphertexts, 3-bit vectors, two items."""
    n, qs = 64, bfv.ntt_primes(64, 55, 3)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 46)
    count, nbits, ncls = 2, 3, 3
    s = inputs.uniform_ciphertexts(n, qs, ncls * count * nbits, 46, "s").reshape(ncls, count, nbits, 2, len(qs), n)
    say("less_than / argmax n=64")
    lt = down(ctx.less_than(rlk_d, up(s[0]), up(s[1])))
    for j in range(count):
        assert (lt[j] == bfv.less_than(P, rlk, list(s[0, j]), list(s[1, j]))).all(), j
    oh = down(ctx.argmax(rlk_d, up(s)))
    for j in range(count):
        want = bfv.argmax(P, rlk, [list(s[cl, j]) for cl in range(ncls)])
        for cl in range(ncls):
            assert (oh[cl, j] == want[cl]).all(), (cl, j)


def test_bridge_then_argmax_decrypts_one_hot(dev):
    """End to end at p = 17: encrypted class scores in [0, 17) -> bridge to 5
    bits -> one-hot argmax (ties to the lower class); decryptions equal the
    plain argmax and the words equal the oracle's."""
    n, qs = 256, bfv.ntt_primes(256, 55, 6)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 47)
    scores = [[16, 3], [16, 9], [2, 9]]  # [class][item]: a tie at the top and a tie below
    ncls, count = len(scores), len(scores[0])
    r = inputs.encryption_randomness(n, ncls * count, 47)
    cts = []
    for cl in range(ncls):
        for j in range(count):
            pt = np.zeros(n, dtype=np.uint64)
            pt[0] = scores[cl][j]
            cts.append(bfv.encrypt(P, pk, pt, r["u"][cl * count + j], r["e"][cl * count + j]))
    cts = np.stack(cts)
    say("bridge + argmax n=256")
    bits = ctx.bridge_to_bits(rlk_d, up(cts), 5)  # [ncls*count][5][2][k][n]
    oh = down(ctx.argmax(rlk_d, bits.reshape(ncls, count, 5, 2, len(qs), n)))
    bits_o = np.stack([bfv.bridge_to_bits(P, ct, rlk, 5)[0] for ct in cts])
    assert (down(bits) == bits_o).all()
    bits_o = bits_o.reshape(ncls, count, 5, 2, len(qs), n)
    for j in range(count):
        best = max(range(ncls), key=lambda cl: (scores[cl][j], -cl))
        want = bfv.argmax(P, rlk, [list(bits_o[cl, j]) for cl in range(ncls)])
        for cl in range(ncls):
            assert (oh[cl, j] == want[cl]).all(), (cl, j)
            d = bfv.decrypt(P, km["s"], oh[cl, j])
            assert int(d[0]) == int(cl == best) and (d[1:] == 0).all(), (cl, j)


def test_signed_casts_words_and_round_trip(dev):
    """SecureInt -> SecureMod on uniform bit ciphertexts (words), and
    SecureMod -> SecureInt at p = 17 through the bridge (words, decryptions,
    and the round trip back to x)."""
    n, qs = 64, bfv.ntt_primes(64, 55, 5)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 48)
    u = inputs.uniform_ciphertexts(n, qs, 2 * 5, 48, "u").reshape(2, 5, 2, len(qs), n)
    say("signed casts n=64")
    got = down(ctx.int_to_mod(up(u)))
    for j in range(2):
        assert (got[j] == bfv.int_to_mod(P, list(u[j]))).all(), j
    xs = [16, 5]
    r = inputs.encryption_randomness(n, len(xs), 48)
    cts = []
    for j, x in enumerate(xs):
        pt = np.zeros(n, dtype=np.uint64)
        pt[0] = x
        cts.append(bfv.encrypt(P, pk, pt, r["u"][j], r["e"][j]))
    cts = np.stack(cts)
    Y = ctx.mod_to_int(rlk_d, up(cts), 5)
    Yh = down(Y)
    for j, x in enumerate(xs):
        want = bfv.mod_to_int(P, cts[j], rlk, 5)
        assert (Yh[j] == want).all(), j
        v = x - 17 if x >= 16 else x
        for i in range(5):
            d = bfv.decrypt(P, km["s"], Yh[j, i])
            assert int(d[0]) == ((v % 32) >> i) & 1 and (d[1:] == 0).all(), (x, i)
    back = down(ctx.int_to_mod(Y))
    for j, x in enumerate(xs):
        assert int(bfv.decrypt(P, km["s"], back[j])[0]) == x


def test_unfused_squaring_path_and_autotune(dev):
    """The squaring through the unfused kernels (forced threshold) and the
    product pipeline after the autotuner picked its launch shape: every word
    against the oracle either way."""
    n, qs = 1024, bfv.ntt_primes(1024, 36, 3)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 65537, "slots", 18)
    count = 24
    a = inputs.uniform_ciphertexts(n, qs, count, 18, "a")
    b = inputs.uniform_ciphertexts(n, qs, count, 18, "b")
    say("unfused squaring / autotune n=1024")
    ctx.set_fused_threshold(True, 1 << 40)
    da = up(a)
    sq = down(ctx.mul_relin(rlk_d, da, da))
    ctx.set_fused_threshold(True, 0)
    for j in range(0, count, 5):
        assert (sq[j] == bfv.mul_relin(P, a[j], a[j], rlk)).all(), f"square {j}"
    db = up(b)
    chunk, fused = ctx.autotune_mul_relin(rlk_d, da, db)
    assert chunk in (count, count // 2, count // 4)
    out = down(ctx.mul_relin(rlk_d, da, db))
    for j in range(0, count, 5):
        assert (out[j] == bfv.mul_relin(P, a[j], b[j], rlk)).all(), f"product {j}"
    chunk_s, fused_s = ctx.autotune_mul_relin(rlk_d, da, da)
    sq2 = down(ctx.mul_relin(rlk_d, da, da))
    assert (sq2 == sq).all()


@pytest.mark.parametrize("n,k,limit", [(64, 4, 0), (256, 5, 16), (64, 4, 4)])
def test_bridge_powers_all_words(dev, n, k, limit):
    """The power-basis bridge against the oracle word for word, bits decrypt
    to the plain bits (x = 16, 0, 9); with a batch cap of 16 the inputs run
    in groups of two; with a cap of 4 (below the eight products of the last
    tree level) one input at a time, each level in launches of at most four
    products."""
    qs = bfv.ntt_primes(n, 55, k)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 49)
    if limit:
        ctx.set_batch_limit(limit)
    xs = [16, 0, 9]
    r = inputs.encryption_randomness(n, len(xs), 49)
    cts = []
    for j, x in enumerate(xs):
        pt = np.zeros(n, dtype=np.uint64)
        pt[0] = x
        cts.append(bfv.encrypt(P, pk, pt, r["u"][j], r["e"][j]))
    cts = np.stack(cts)
    say(f"bridge powers n={n} k={k} limit={limit}")
    got = down(ctx.bridge_to_bits_powers(rlk_d, up(cts), 5))
    for j, x in enumerate(xs):
        want = bfv.bridge_to_bits_powers(P, cts[j], rlk, 5)
        assert (got[j] == want).all(), j
        for b in range(5):
            d = bfv.decrypt(P, km["s"], got[j, b])
            assert int(d[0]) == (x >> b) & 1 and (d[1:] == 0).all(), (x, b)


@pytest.mark.parametrize("t,nbits,xs", [(3, 2, [2, 0, 1]), (5, 3, [4, 3]), (7, 3, [6, 5]), (257, 9, [256, 100])])
def test_bridge_powers_other_moduli(dev, t, nbits, xs):
    """The power-basis bridge for other prime plaintext moduli, including the
    degenerate trees (t = 3: one product and no cached power beyond x; t = 5
    and 7: a last level shorter than the one before) and t = 257 (255
    products, depth 8, nine bits): GPU words equal the oracle's, bits decrypt
    to the bits of x."""
    n, k = 64, 4
    qs = bfv.ntt_primes(n, 55, k)
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "coeff", 50)
    r = inputs.encryption_randomness(n, len(xs), 50)
    cts = []
    for j, x in enumerate(xs):
        pt = np.zeros(n, dtype=np.uint64)
        pt[0] = x
        cts.append(bfv.encrypt(P, pk, pt, r["u"][j], r["e"][j]))
    cts = np.stack(cts)
    say(f"bridge powers t={t} nbits={nbits}")
    got = down(ctx.bridge_to_bits_powers(rlk_d, up(cts), nbits))
    for j, x in enumerate(xs):
        want = bfv.bridge_to_bits_powers(P, cts[j], rlk, nbits)
        assert (got[j] == want).all(), (t, j)
        for b in range(nbits):
            d = bfv.decrypt(P, km["s"], got[j, b])
            assert int(d[0]) == (x >> b) & 1 and (d[1:] == 0).all(), (t, x, b)


def test_bridge_powers_full_size_sampled(dev):
    """The power-basis bridge at the benchmark's shape and launch
    configuration: n = 16384, eight 55-bit primes, p = 17, 256 inputs in one
    call.  The last input's five bit ciphertexts against the oracle word for
    word, and every decrypted bit equal to the plain bit."""
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    say("bridge powers n=16384 k=8 x256")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, t, "coeff", 0)
    count = 256
    xs = inputs.bridge_values(t, count, 0)
    pts = np.zeros((count, n), dtype=np.uint64)
    pts[:, 0] = xs
    r = inputs.encryption_randomness(n, count, 0)
    ct_d = ctx.encrypt(up(pk), pts, r["u"], r["e"])
    bits = ctx.bridge_to_bits_powers(rlk_d, ct_d, 5)
    j = count - 1
    last = down(bits[j])
    want = bfv.bridge_to_bits_powers(P, down(ct_d[j]), rlk, 5)
    assert (last == want).all()
    dec = ctx.decrypt(km["s"], bits.reshape(-1, 2, len(qs), n)).reshape(count, 5, n)[:, :, 0]
    plain = (xs[:, None].astype(np.int64) >> np.arange(5)) & 1
    assert (dec.astype(np.int64) == plain).all()


@pytest.mark.parametrize("n,bits,k,count", [(16384, 55, 3, 183), (2048, 55, 5, 1101), (1024, 36, 3, 2731)])
def test_ntt_row_loop_many_rows(dev, n, bits, k, count):
    """Launches with more rows than resident workgroups, so every workgroup
    loops over several rows (prefetching the next one while it transforms
    the current one) and the last pass is ragged: sampled rows in the pinned
    order against the oracle's transform, and every row back after the
    inverse."""
    qs = bfv.ntt_primes(n, bits, k)
    say(f"ntt row loop n={n} k={k} rows={count * k}")
    ctx = fhe.Context(n, qs, 17, "coeff")
    rng = np.random.default_rng(n + count)
    polys = np.stack([np.stack([rng.integers(0, q, n, dtype=np.uint64) for q in qs]) for _ in range(count)])
    d = up(polys)
    ctx.ntt(d)
    got = down(d)
    psis = [bfv.find_psi(q, n) for q in qs]
    L = n.bit_length() - 1
    rev = np.array([int(format(j, f"0{L}b")[::-1], 2) for j in range(n)])
    for c in sorted({0, 1, count // 2, count - 2, count - 1}):
        want = bfv.clib.ntt_rows(polys[c], qs, psis)
        assert (got[c][:, rev] == want).all(), f"poly {c}"
    ctx.ntt(d, inverse=True)
    assert (down(d) == polys).all()


def test_bridge_powers_edges(dev):
    """Argument handling of the power-basis bridge: no inputs is a no-op;
    slot encoding is unsupported; too few bits, a workspace below the
    documented size and an output overlapping the inputs are rejected before
    any launch (the output keeps its contents)."""
    import torch
    n = 64
    qs = bfv.ntt_primes(n, 55, 3)
    say("bridge powers edges")
    P, km, pk, rlk, ctx, rlk_d = setup(n, qs, 17, "coeff", 14)
    x = up(inputs.uniform_ciphertexts(n, qs, 2, 14, "x") % 2)  # canonical words
    assert ctx.bridge_to_bits_powers(rlk_d, ctx.empty_ct(0), 5).shape == (0, 5, 2, 3, n)
    with pytest.raises(fhe.FheError) as ei:
        fhe.Context(n, qs, 257, "slots").bridge_to_bits_powers(rlk_d, x, 9)
    assert ei.value.status == -7
    with pytest.raises(fhe.FheError) as ei:
        ctx.bridge_to_bits_powers(rlk_d, x, 4)  # 2^4 < 17
    assert ei.value.status == -1
    L = fhe.lib()
    out = torch.zeros((2, 5, 2, 3, n), dtype=torch.int64, device="cuda")
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    st = L.fhe_bridge_to_bits_powers(ctx._h, fhe._dptr(rlk_d), fhe._dptr(x), 5, fhe._dptr(out), 2,
                                     fhe._dptr(ws), 64, fhe._stream())
    assert st == -8
    ws, _ = ctx.workspace(fhe.OP_BRIDGE_POWERS, 1)
    buf = torch.zeros((6, 2, 3, n), dtype=torch.int64, device="cuda")
    buf[0].copy_(x[0])
    st = L.fhe_bridge_to_bits_powers(ctx._h, fhe._dptr(rlk_d), fhe._dptr(buf), 5, fhe._dptr(buf), 1,
                                     fhe._dptr(ws), ws.numel(), fhe._stream())
    assert st == -1
    assert (down(out) == 0).all() and (down(buf[1:]) == 0).all()
