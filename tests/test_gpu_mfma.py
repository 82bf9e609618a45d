"""The first radix-16 pass of the forward transform on the int8 matrix cores
against the same pass on the vector ALU (fhe_ntt_pass0): every output word
equal, both equal to the pass's definition on sampled groups (the four
butterfly levels of the negacyclic transform reduce a(X) modulo
X^(n/16) - zeta^(2 bitrev4(j) + 1), zeta = psi^(n/16): slot j of group g is
sum_e a[g + e n/16] zeta^(e (2 bitrev4(j) + 1))), at n = 1024 .. 16384 with
the configured primes, on uniform residues plus the edge words 0 and q - 1."""
import numpy as np
import pytest

from oracle import bfv
from paper_2204_12201_amd import fhe, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-mfma] {msg}", flush=True)


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


def brev4(j):
    return int(f"{j:04b}"[::-1], 2)


@pytest.mark.parametrize("n,bits,k,count", [(1024, 55, 8, 3), (4096, 36, 3, 5), (8192, 43, 5, 2),
                                            (16384, 55, 8, 2)])
def test_pass0_matrix_cores_equal_valu_and_definition(dev, n, bits, k, count):
    qs = bfv.ntt_primes(n, bits, k)
    say(f"pass 0 n={n} k={k} x{count}")
    ctx = fhe.Context(n, qs, 17, "coeff")
    x = inputs.uniform_ciphertexts(n, qs, count, 61, "p0")[:, 0].copy()  # [count][k][n]
    S = n // 16
    for i, q in enumerate(qs):  # edge words: a whole group of q - 1, and zeros
        x[0, i, [3 + e * S for e in range(16)]] = q - 1
        x[-1, i, [S - 1 + e * S for e in range(16)]] = 0
        x[-1, i, 5] = q - 1
    a, b = up(x), up(x)
    ctx.ntt_pass0(a, mfma=False)
    ctx.ntt_pass0(b, mfma=True)
    va, vb = down(a), down(b)
    assert (va == vb).all()
    # three passes back to back on the chip (M^3 x): the same words again
    a3, b3 = up(x), up(x)
    ctx.ntt_pass0(a3, mfma=False, reps=3)
    ctx.ntt_pass0(b3, mfma=True, reps=3)
    a1 = up(x)
    for _ in range(3):
        ctx.ntt_pass0(a1, mfma=True)
    v3 = down(a3)
    assert (v3 == down(b3)).all() and (v3 == down(a1)).all()
    rng = np.random.default_rng(n)
    for r in range(count):
        for i, q in enumerate(qs):
            zeta = pow(bfv.find_psi(q, n), S, q)
            for g in [0, 3, 5, S - 1] + [int(v) for v in rng.integers(0, S, 4)]:
                xs = [int(x[r, i, g + e * S]) for e in range(16)]
                for j in range(16):
                    ex = 2 * brev4(j) + 1
                    want = sum(xe * pow(zeta, e * ex, q) for e, xe in enumerate(xs)) % q
                    assert int(va[r, i, g + j * S]) == want, (r, i, g, j)


def test_pass0_rejections(dev):
    n = 1024
    ctx61 = fhe.Context(n, bfv.ntt_primes(n, 61, 2), 17, "coeff")
    t = up(np.zeros((1, 2, n), dtype=np.uint64))
    with pytest.raises(fhe.FheError) as ei:
        ctx61.ntt_pass0(t, mfma=True)
    assert ei.value.status == -7
    ctx61.ntt_pass0(t, mfma=False)  # the vector ALU pass takes any prime
    small = fhe.Context(512, bfv.ntt_primes(512, 40, 2), 17, "coeff")
    with pytest.raises(fhe.FheError) as ei:
        small.ntt_pass0(up(np.zeros((1, 2, 512), dtype=np.uint64)), mfma=False)
    assert ei.value.status == -7
