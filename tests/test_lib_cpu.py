"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects bad parameter sets before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2204_12201_amd import fhe, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fhe.LIBPATH):
        from paper_2204_12201_amd import build
        build.build(verbose=False)
    return fhe.lib()


def header_functions():
    text = open(os.path.join(ROOT, "include", "fhe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fhe_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported(L):
    names = header_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(L, name), name
    assert sorted(fhe.EXPORTED) == names


def _create(L, n, q, t, enc=fhe.ENC_SLOTS, k=None):
    arr = (ctypes.c_uint64 * max(1, len(q)))(*q)
    p = fhe._Params(n, len(q) if k is None else k, t, ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint64)), enc)
    h = ctypes.c_void_p()
    st = L.fhe_ctx_create(ctypes.byref(p), 0, ctypes.byref(h))
    if st == 0:
        L.fhe_ctx_destroy(h)
    return st


Q4096 = inputs.PRIMES[(4096, 36)]


@pytest.mark.parametrize("case", [
    dict(n=4095, q=Q4096, t=65537),                      # n not a power of two
    dict(n=32768, q=Q4096, t=65537),                     # n too large
    dict(n=8, q=Q4096, t=65537),                         # n too small
    dict(n=4096, q=Q4096 + [Q4096[0]], t=65537),         # repeated prime
    dict(n=4096, q=[68719403009 + 8192], t=65537),       # 1 mod 2n but composite
    dict(n=8192, q=Q4096, t=65537),                      # q_i != 1 mod 2n
    dict(n=4096, q=[(1 << 62) + 1], t=65537),            # q_i >= 2^62
    dict(n=4096, q=[2305843009213800449], t=65537),     # prime, 1 mod 2n, but >= 2^61
    dict(n=4096, q=Q4096, t=Q4096[1]),                   # gcd(t, q) != 1
    dict(n=4096, q=Q4096, t=65539),                      # slots need t = 1 mod 2n
    dict(n=4096, q=Q4096, t=1),                          # t < 2
    dict(n=4096, q=Q4096, t=65537, k=0),                 # k = 0
    dict(n=4096, q=Q4096, t=65537, enc=7),               # unknown encoding
])
def test_bad_params_rejected(L, case):
    st = _create(L, case["n"], case["q"], case["t"], case.get("enc", fhe.ENC_SLOTS), case.get("k"))
    assert st == -2, fhe.STATUS.get(st, st)


def test_null_arguments(L):
    assert L.fhe_ctx_create(None, 0, None) == -1
    assert L.fhe_mul_relin(None, None, None, None, None, 1, None, 0, None) == -1
    assert L.fhe_status_str(-8) == b"workspace too small"


def test_valid_params_pass_validation(L):
    # A valid set gets past the parameter checks: OK with a device, else a HIP error.
    st = _create(L, 4096, Q4096, 65537)
    assert st in (0, -4)
    st = _create(L, 16384, inputs.PRIMES[(16384, 55)], 17, fhe.ENC_COEFF)
    assert st in (0, -4)


def test_shoup_sum_form_host(tmp_path):
    """The transforms form the lazy Shoup remainder a w - h q as
    a w + h (2^64 - q) (equal modulo 2^64, no borrow chain).  The header's
    host build checks both forms against each other and against a w mod q
    (below 4q) for the configured primes and moduli at the extremes of the
    supported range, on edge operands and 200,000 random pairs each."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "host_modarith")
    src = os.path.join(ROOT, "tests", "host_modarith.cpp")
    inc = os.path.join(ROOT, "paper_2204_12201_amd", "csrc")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", inc, src, "-o", exe], check=True)
    qs = sorted({q for cfg in inputs.CONFIGS.values() for q in cfg["q"]})
    qs += [3, (1 << 36) + 1, (1 << 61) - 1]
    r = subprocess.run([exe, *map(str, qs)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
