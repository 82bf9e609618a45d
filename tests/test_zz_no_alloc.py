"""The product entry point that allocates nothing (fhe_mul_relin_static),
called through the C ABI, against fhe_mul_relin with a caller workspace:
the same words on two calls in a row, the second with fewer products, at
n = 16384 (eight 55-bit primes, the static array holds four products) and
n = 4096; the squaring path; a call needing more than the static array is
rejected before anything is enqueued, and runs once the batch limit is
lowered."""
import numpy as np
import pytest

from paper_2204_12201_amd import fhe, inputs

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20  # FHE_STATIC_WS_BYTES


def say(msg):
    print(f"[no-alloc] {msg}", flush=True)


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


def static_call(ctx, rlk, a, b, out):
    return fhe.lib().fhe_mul_relin_static(ctx._h, fhe._dptr(rlk), fhe._dptr(a), fhe._dptr(b), fhe._dptr(out),
                                          a.shape[0], fhe._stream())


def context(name, seed):
    cfg = inputs.CONFIGS[name]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    km = inputs.key_material(n, qs, seed)
    ctx = fhe.Context(n, qs, t, cfg["encoding"])
    _, rlk = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    return ctx, rlk, n, qs


@pytest.mark.parametrize("name,counts", [("bfv_n16384", (4, 3)), ("bfv_n4096", (40, 7))])
def test_static_workspace_product_matches_workspace_product(dev, name, counts):
    ctx, rlk, n, qs = context(name, 51)
    per = fhe.lib().fhe_workspace_bytes(ctx._h, fhe.OP_MUL_RELIN, 1)
    assert counts[0] * per <= STATIC_BYTES
    for call, count in enumerate(counts):
        say(f"{name}: call {call} with {count} products")
        a = up(inputs.uniform_ciphertexts(n, qs, count, 52 + call, "a"))
        b = up(inputs.uniform_ciphertexts(n, qs, count, 52 + call, "b"))
        want = down(ctx.mul_relin(rlk, a, b))
        out = ctx.empty_ct(count)
        assert static_call(ctx, rlk, a, b, out) == 0
        assert (down(out) == want).all(), (name, call)
        # squaring path (a == b), in place
        wsq = down(ctx.mul_relin(rlk, a, a))
        assert static_call(ctx, rlk, a, a, a) == 0
        assert (down(a) == wsq).all(), (name, call, "square")
    ctx.sync()


def test_static_workspace_limit(dev):
    ctx, rlk, n, qs = context("bfv_n16384", 53)
    per = fhe.lib().fhe_workspace_bytes(ctx._h, fhe.OP_MUL_RELIN, 1)
    count = STATIC_BYTES // per + 1  # one product more than the array holds
    a = up(inputs.uniform_ciphertexts(n, qs, count, 54, "a"))
    b = up(inputs.uniform_ciphertexts(n, qs, count, 54, "b"))
    out = ctx.empty_ct(count)
    out.fill_(7)
    say(f"n=16384: {count} products, over the static array")
    assert static_call(ctx, rlk, a, b, out) == -8  # FHE_EWORKSPACE
    assert (down(out) == 7).all()  # nothing was enqueued
    ctx.set_batch_limit(2)
    assert static_call(ctx, rlk, a, b, out) == 0
    got = down(out)
    ctx.set_batch_limit(0)
    assert (got == down(ctx.mul_relin(rlk, a, b))).all()
    ctx.sync()
