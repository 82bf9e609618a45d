"""Thin ctypes binding of libfhe.so (include/fhe.h).

Argument marshalling only: every homomorphic step runs in the library's HIP
kernels.  Device buffers are torch int64 tensors used as raw uint64 storage
(no torch arithmetic touches them); torch supplies device memory and the
current stream.  Host arrays are numpy.  If the library is not built this
module raises FheError on first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libfhe.so")

ENC_SLOTS, ENC_COEFF = 0, 1
OP_MUL_RELIN, OP_SQUARE_RELIN, OP_BRIDGE, OP_KEYGEN, OP_ENCRYPT, OP_DECRYPT, OP_RLK_IMPORT = range(1, 8)
OP_WEIGHTED_SUM, OP_GATE, OP_COMPARE, OP_ARGMAX, OP_MOD_TO_INT, OP_BRIDGE_POWERS = range(8, 14)
GATES = {"AND": 0, "NAND": 1, "OR": 2, "NOR": 3, "XOR": 4, "XNOR": 5, "NOT": 6, "MUX": 7}

STATUS = {0: "ok", -1: "invalid argument", -2: "parameter set rejected", -3: "device allocation failed",
          -4: "HIP error", -5: "shape mismatch", -6: "non-canonical input word",
          -7: "operation not supported for these parameters", -8: "workspace too small"}


class FheError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status})")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("k", ctypes.c_uint32), ("t", ctypes.c_uint64),
                ("q", ctypes.POINTER(ctypes.c_uint64)), ("encoding", ctypes.c_uint32)]


class MulPart(ctypes.Structure):
    """One part of fhe_mul_relin_multi (include/fhe.h)."""
    _fields_ = [("ctx", ctypes.c_void_p), ("rlk_dev", ctypes.c_void_p), ("a", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("out", ctypes.c_void_p), ("count", ctypes.c_size_t),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


_lib = None

# (name, restype, argtypes); c_void_p stands for pointers and the stream.
_P, _Z, _U64, _U32, _I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
_SIGS = [
    ("fhe_ctx_create", _I, [ctypes.POINTER(_Params), _I, ctypes.POINTER(_P)]),
    ("fhe_ctx_destroy", None, [_P]),
    ("fhe_ct_words", _Z, [_P]),
    ("fhe_pk_words", _Z, [_P]),
    ("fhe_rlk_words", _Z, [_P]),
    ("fhe_aux_primes", _U32, [_P]),
    ("fhe_workspace_bytes", _Z, [_P, _I, _Z]),
    ("fhe_set_batch_limit", _I, [_P, _Z]),
    ("fhe_set_fused_threshold", _I, [_P, _I, _Z]),
    ("fhe_set_conv_method", _I, [_P, _I]),
    ("fhe_conv_method", _I, [_P]),
    ("fhe_autotune_mul_relin", _I, [_P, _P, _P, _P, _P, _Z, _P, _Z, _P, ctypes.POINTER(_Z),
                                    ctypes.POINTER(ctypes.c_int)]),
    ("fhe_keygen", _I, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _Z, _P]),
    ("fhe_rlk_import", _I, [_P, _P, _P, _P, _Z, _P]),
    ("fhe_encode", _I, [_P, _P, _P]),
    ("fhe_decode", _I, [_P, _P, _P]),
    ("fhe_encrypt", _I, [_P, _P, _P, _P, _P, _P, _Z, _P, _Z, _P]),
    ("fhe_decrypt", _I, [_P, _P, _P, _P, _Z, _P, _Z, _P]),
    ("fhe_add", _I, [_P, _P, _P, _P, _Z, _P]),
    ("fhe_sub", _I, [_P, _P, _P, _P, _Z, _P]),
    ("fhe_neg", _I, [_P, _P, _P, _Z, _P]),
    ("fhe_add_plain_const", _I, [_P, _P, _U64, _P, _Z, _P]),
    ("fhe_sub_plain_const", _I, [_P, _P, _U64, _P, _Z, _P]),
    ("fhe_mul_relin", _I, [_P, _P, _P, _P, _P, _Z, _P, _Z, _P]),
    ("fhe_mul_relin_multi", _I, [ctypes.POINTER(MulPart), _Z, _P]),
    ("fhe_set_multi_persistent", _I, [_P, _I]),
    ("fhe_autotune_mul_relin_multi", _I, [ctypes.POINTER(MulPart), _Z, _P, ctypes.POINTER(ctypes.c_int)]),
    ("fhe_mul_relin_static", _I, [_P, _P, _P, _P, _P, _Z, _P]),
    ("fhe_square_chain", _I, [_P, _P, _P, _U32, _Z, _P, _Z, _I, _P]),
    ("fhe_bridge_to_bits", _I, [_P, _P, _P, _U32, _P, _P, _Z, _P, _Z, _P]),
    ("fhe_bits_to_mod", _I, [_P, _P, _U32, _P, _Z, _P]),
    ("fhe_weighted_sum", _I, [_P, _P, _Z, _P, _Z, _P, _P, _Z, _P]),
    ("fhe_gate", _I, [_P, _P, _I, _P, _P, _P, _P, _Z, _P, _Z, _P]),
    ("fhe_less_than", _I, [_P, _P, _P, _P, _U32, _P, _Z, _P, _Z, _P]),
    ("fhe_argmax", _I, [_P, _P, _P, _U32, _U32, _P, _Z, _P, _Z, _P]),
    ("fhe_int_to_mod", _I, [_P, _P, _U32, _P, _Z, _P]),
    ("fhe_mod_to_int", _I, [_P, _P, _P, _U32, _P, _Z, _P, _Z, _P]),
    ("fhe_bridge_to_bits_powers", _I, [_P, _P, _P, _U32, _P, _Z, _P, _Z, _P]),
    ("fhe_ntt", _I, [_P, _I, _P, _Z, _P]),
    ("fhe_ntt_pass0", _I, [_P, _I, _U32, _P, _Z, _P]),
    ("fhe_set_timing", _I, [_P, _I]),
    ("fhe_kernel_kinds", _I, []),
    ("fhe_kernel_name", ctypes.c_char_p, [_I]),
    ("fhe_kernel_stats", _I, [_P, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)]),
    ("fhe_reset_kernel_stats", _I, [_P]),
    ("fhe_fallback_count", _I, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    ("fhe_sync", _I, [_P, _P]),
    ("fhe_status_str", ctypes.c_char_p, [_I]),
]

EXPORTED = [s[0] for s in _SIGS]


def lib():
    """Load libfhe.so; raises FheError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise FheError(-4, f"HIP library missing at {LIBPATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIBPATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise FheError(status, where)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t) -> ctypes.c_void_p:
    assert t.is_cuda and t.is_contiguous(), "device tensor must be a contiguous CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray, dtype) -> tuple:
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def to_numpy_u64(t) -> np.ndarray:
    """Device int64 tensor (raw uint64 words) -> numpy uint64 copy."""
    return t.detach().cpu().numpy().view(np.uint64)


def from_numpy_u64(a: np.ndarray, device):
    """numpy uint64 words -> device int64 tensor holding the same bits."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64).copy()).to(device)


class Context:
    """One parameter set on one HIP device (not thread safe)."""

    def __init__(self, n: int, q, t: int, encoding: str = "slots", device: int = 0):
        import torch
        self.n, self.q, self.t = int(n), [int(x) for x in q], int(t)
        self.k = len(self.q)
        self.encoding = encoding
        self.device = torch.device("cuda", device)
        qarr = (ctypes.c_uint64 * self.k)(*self.q)
        p = _Params(self.n, self.k, self.t, ctypes.cast(qarr, ctypes.POINTER(ctypes.c_uint64)),
                    ENC_SLOTS if encoding == "slots" else ENC_COEFF)
        h = ctypes.c_void_p()
        _check(lib().fhe_ctx_create(ctypes.byref(p), device, ctypes.byref(h)), "fhe_ctx_create")
        self._h = h
        self.ct_words = lib().fhe_ct_words(h)
        self.rlk_words = lib().fhe_rlk_words(h)
        self.aux_primes = lib().fhe_aux_primes(h)
        self._ws = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().fhe_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- buffers ---
    def empty_ct(self, count: int):
        import torch
        return torch.empty((count, 2, self.k, self.n), dtype=torch.int64, device=self.device)

    def workspace(self, op: int, count: int):
        """Cached device workspace of at least fhe_workspace_bytes(op, count)."""
        import torch
        need = lib().fhe_workspace_bytes(self._h, op, count)
        cur = self._ws.get("buf")
        if cur is None or cur.numel() < need:
            self._ws["buf"] = None
            cur = torch.empty(max(need, 8), dtype=torch.uint8, device=self.device)
            self._ws["buf"] = cur
        return cur, need

    def set_batch_limit(self, items: int):
        _check(lib().fhe_set_batch_limit(self._h, items), "fhe_set_batch_limit")
        self._ws.clear()

    # -------------------------------------------------------------- keys ---
    def keygen(self, s, pk_a, pk_e, rlk_a, rlk_e):
        import torch
        s, ps = _hptr(s, np.int8)
        pk_a, ppa = _hptr(pk_a, np.uint64)
        pk_e, ppe = _hptr(pk_e, np.int32)
        rlk_a, pra = _hptr(rlk_a, np.uint64)
        rlk_e, pre = _hptr(rlk_e, np.int32)
        pk = torch.empty((2, self.k, self.n), dtype=torch.int64, device=self.device)
        rlk = torch.empty(self.rlk_words, dtype=torch.int64, device=self.device)
        ws, need = self.workspace(OP_KEYGEN, 1)
        _check(lib().fhe_keygen(self._h, ps, ppa, ppe, pra, pre, _dptr(pk), _dptr(rlk), _dptr(ws),
                                ws.numel(), _stream()), "fhe_keygen")
        return pk, rlk

    def rlk_import(self, rlk_coeff):
        """rlk_coeff: device tensor [k][2][k][n] (coefficient form)."""
        import torch
        rlk = torch.empty(self.rlk_words, dtype=torch.int64, device=self.device)
        _check(lib().fhe_rlk_import(self._h, _dptr(rlk_coeff.contiguous()), _dptr(rlk), None, 0,
                                    _stream()), "fhe_rlk_import")
        return rlk

    # ---------------------------------------------------------- encoding ---
    def encode(self, vals) -> np.ndarray:
        v, pv = _hptr(vals, np.uint64)
        out = np.empty(self.n, dtype=np.uint64)
        _check(lib().fhe_encode(self._h, pv, out.ctypes.data_as(ctypes.c_void_p)), "fhe_encode")
        return out

    def decode(self, pt) -> np.ndarray:
        p, pp = _hptr(pt, np.uint64)
        out = np.empty(self.n, dtype=np.uint64)
        _check(lib().fhe_decode(self._h, pp, out.ctypes.data_as(ctypes.c_void_p)), "fhe_decode")
        return out

    # -------------------------------------------------------- enc / dec ---
    def encrypt(self, pk, pts, u, e):
        """pts uint64 [count][n], u int8 [count][n], e int32 [count][2][n]."""
        pts, pp = _hptr(pts, np.uint64)
        count = pts.shape[0]
        u, pu = _hptr(u, np.int8)
        e, pe = _hptr(e, np.int32)
        ct = self.empty_ct(count)
        ws, need = self.workspace(OP_ENCRYPT, count)
        _check(lib().fhe_encrypt(self._h, _dptr(pk), pp, pu, pe, _dptr(ct), count, _dptr(ws), ws.numel(),
                                 _stream()), "fhe_encrypt")
        return ct

    def decrypt(self, s, ct) -> np.ndarray:
        s, ps = _hptr(s, np.int8)
        count = ct.shape[0]
        out = np.empty((count, self.n), dtype=np.uint64)
        ws, need = self.workspace(OP_DECRYPT, count)
        _check(lib().fhe_decrypt(self._h, ps, _dptr(ct), out.ctypes.data_as(ctypes.c_void_p), count,
                                 _dptr(ws), ws.numel(), _stream()), "fhe_decrypt")
        return out

    # ------------------------------------------------------- elementwise ---
    def _out(self, out, like):
        return self.empty_ct(like.shape[0]) if out is None else out

    def add(self, a, b, out=None):
        out = self._out(out, a)
        _check(lib().fhe_add(self._h, _dptr(a), _dptr(b), _dptr(out), a.shape[0], _stream()), "fhe_add")
        return out

    def sub(self, a, b, out=None):
        out = self._out(out, a)
        _check(lib().fhe_sub(self._h, _dptr(a), _dptr(b), _dptr(out), a.shape[0], _stream()), "fhe_sub")
        return out

    def neg(self, a, out=None):
        out = self._out(out, a)
        _check(lib().fhe_neg(self._h, _dptr(a), _dptr(out), a.shape[0], _stream()), "fhe_neg")
        return out

    def add_plain(self, a, c: int, out=None):
        out = self._out(out, a)
        _check(lib().fhe_add_plain_const(self._h, _dptr(a), c, _dptr(out), a.shape[0], _stream()),
               "fhe_add_plain_const")
        return out

    def sub_plain(self, a, c: int, out=None):
        out = self._out(out, a)
        _check(lib().fhe_sub_plain_const(self._h, _dptr(a), c, _dptr(out), a.shape[0], _stream()),
               "fhe_sub_plain_const")
        return out

    # ---------------------------------------------------------- hot path ---
    def mul_relin(self, rlk, a, b, out=None):
        out = self._out(out, a)
        count = a.shape[0]
        op = OP_SQUARE_RELIN if a.data_ptr() == b.data_ptr() else OP_MUL_RELIN
        ws, need = self.workspace(op, count)
        _check(lib().fhe_mul_relin(self._h, _dptr(rlk), _dptr(a), _dptr(b), _dptr(out), count, _dptr(ws),
                                   ws.numel(), _stream()), "fhe_mul_relin")
        return out

    def autotune_mul_relin(self, rlk, a, b):
        """Time the product pipeline on these inputs at the candidate launch
        shapes and keep the fastest in the context; returns (chunk, fused)."""
        count = a.shape[0]
        op = OP_SQUARE_RELIN if a.data_ptr() == b.data_ptr() else OP_MUL_RELIN
        ws, _ = self.workspace(op, count)
        out = self.empty_ct(count)
        chunk, fused = _Z(0), ctypes.c_int(0)
        _check(lib().fhe_autotune_mul_relin(self._h, _dptr(rlk), _dptr(a), _dptr(b), _dptr(out), count, _dptr(ws),
                                            ws.numel(), _stream(), ctypes.byref(chunk), ctypes.byref(fused)),
               "fhe_autotune_mul_relin")
        return chunk.value, bool(fused.value)

    def set_multi_persistent(self, enable: bool):
        """Key switching of multi-part products led by this context in one
        persistent launch where it applies (fhe_set_multi_persistent)."""
        _check(lib().fhe_set_multi_persistent(self._h, 1 if enable else 0), "fhe_set_multi_persistent")

    def set_conv_method(self, mfma: bool):
        """Base conversions of the product on the int8 matrix cores (True,
        the default where the bases allow it) or on the vector ALU (False);
        same words (fhe_set_conv_method)."""
        _check(lib().fhe_set_conv_method(self._h, 1 if mfma else 0), "fhe_set_conv_method")

    @property
    def conv_mfma(self) -> bool:
        return lib().fhe_conv_method(self._h) == 1

    def set_fused_threshold(self, square: bool, min_rows: int):
        _check(lib().fhe_set_fused_threshold(self._h, 1 if square else 0, min_rows), "fhe_set_fused_threshold")

    def square_chain(self, rlk, x, depth: int, graph: bool = False):
        """x <- x^(2^depth) in place (device [count][2][k][n]); graph: record
        the launches once into a HIP graph and replay it on later calls with
        the same buffers (the workspace is kept per (count, depth) for that)."""
        import torch
        count = x.shape[0]
        key = ("chain", count, depth)
        need = lib().fhe_workspace_bytes(self._h, OP_SQUARE_RELIN, count)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 8), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        _check(lib().fhe_square_chain(self._h, _dptr(rlk), _dptr(x), depth, count, _dptr(ws), ws.numel(),
                                      1 if graph else 0, _stream()), "fhe_square_chain")
        return x

    def bridge_to_bits(self, rlk, x, nbits: int, with_eq: bool = False):
        import torch
        count = x.shape[0]
        bits = torch.empty((count, nbits, 2, self.k, self.n), dtype=torch.int64, device=self.device)
        eq = (torch.empty((count, self.t, 2, self.k, self.n), dtype=torch.int64, device=self.device)
              if with_eq else None)
        ws, need = self.workspace(OP_BRIDGE, count)
        _check(lib().fhe_bridge_to_bits(self._h, _dptr(rlk), _dptr(x), nbits, _dptr(bits),
                                        _dptr(eq) if eq is not None else None, count, _dptr(ws),
                                        ws.numel(), _stream()), "fhe_bridge_to_bits")
        return (bits, eq) if with_eq else bits

    def bits_to_mod(self, bits, out=None):
        count, nbits = bits.shape[0], bits.shape[1]
        out = self.empty_ct(count) if out is None else out
        _check(lib().fhe_bits_to_mod(self._h, _dptr(bits), nbits, _dptr(out), count, _stream()),
               "fhe_bits_to_mod")
        return out

    def weighted_sum(self, x, w, out=None):
        """out[m] = sum_j w[m][j] x[j]: x device [nin][2][k][n], w host int32
        [nout][nin] (row sums of |w| below 2^30)."""
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.int32)
        nout, nin = w.shape
        out = self.empty_ct(nout) if out is None else out
        ws, _ = self.workspace(OP_WEIGHTED_SUM, nout * nin)
        _check(lib().fhe_weighted_sum(self._h, _dptr(x), nin, w.ctypes.data, nout, _dptr(out), _dptr(ws),
                                      ws.numel(), _stream()), "fhe_weighted_sum")
        return out

    def gate(self, rlk, op: str, a, b=None, c=None, out=None):
        """The paper's gate `op` (AND, NAND, OR, NOR, XOR, XNOR, NOT, MUX) on
        batches of bit ciphertexts (device [count][2][k][n])."""
        out = self._out(out, a)
        count = a.shape[0]
        ws, _ = self.workspace(OP_GATE, count)
        _check(lib().fhe_gate(self._h, _dptr(rlk), GATES[op], _dptr(a), _dptr(b) if b is not None else None,
                              _dptr(c) if c is not None else None, _dptr(out), count, _dptr(ws), ws.numel(),
                              _stream()), "fhe_gate")
        return out

    def less_than(self, rlk, a, b, out=None):
        """[a < b] per item: a, b device [count][nbits][2][k][n], least
        significant bit first."""
        count, nbits = a.shape[0], a.shape[1]
        out = self.empty_ct(count) if out is None else out
        ws, _ = self.workspace(OP_COMPARE, count)
        _check(lib().fhe_less_than(self._h, _dptr(rlk), _dptr(a), _dptr(b), nbits, _dptr(out), count,
                                   _dptr(ws), ws.numel(), _stream()), "fhe_less_than")
        return out

    def argmax(self, rlk, scores, out=None):
        """One-hot argmax: scores device [ncls][count][nbits][2][k][n] ->
        [ncls][count][2][k][n]."""
        import torch
        ncls, count, nbits = scores.shape[0], scores.shape[1], scores.shape[2]
        if out is None:
            out = torch.empty((ncls, count, 2, self.k, self.n), dtype=torch.int64, device=self.device)
        ws, _ = self.workspace(OP_ARGMAX, count)
        _check(lib().fhe_argmax(self._h, _dptr(rlk), _dptr(scores), ncls, nbits, _dptr(out), count, _dptr(ws),
                                ws.numel(), _stream()), "fhe_argmax")
        return out

    def bridge_to_bits_powers(self, rlk, x, nbits: int, out=None):
        """The bridge's bits from the powers of x (t - 2 products per input):
        x device [count][2][k][n] -> [count][nbits][2][k][n]."""
        import torch
        count = x.shape[0]
        if out is None:
            out = torch.empty((count, nbits, 2, self.k, self.n), dtype=torch.int64, device=self.device)
        ws, _ = self.workspace(OP_BRIDGE_POWERS, count)
        _check(lib().fhe_bridge_to_bits_powers(self._h, _dptr(rlk), _dptr(x), nbits, _dptr(out), count, _dptr(ws),
                                               ws.numel(), _stream()), "fhe_bridge_to_bits_powers")
        return out

    def int_to_mod(self, bits, out=None):
        """SecureInt -> SecureMod: bits device [count][nbits][2][k][n]
        (two's complement, least significant first) -> [count][2][k][n]."""
        count, nbits = bits.shape[0], bits.shape[1]
        out = self.empty_ct(count) if out is None else out
        _check(lib().fhe_int_to_mod(self._h, _dptr(bits), nbits, _dptr(out), count, _stream()), "fhe_int_to_mod")
        return out

    def mod_to_int(self, rlk, x, nbits: int, out=None):
        """SecureMod -> SecureInt: x device [count][2][k][n] -> two's
        complement bits [count][nbits][2][k][n]."""
        import torch
        count = x.shape[0]
        if out is None:
            out = torch.empty((count, nbits, 2, self.k, self.n), dtype=torch.int64, device=self.device)
        ws, _ = self.workspace(OP_MOD_TO_INT, count)
        _check(lib().fhe_mod_to_int(self._h, _dptr(rlk), _dptr(x), nbits, _dptr(out), count, _dptr(ws),
                                    ws.numel(), _stream()), "fhe_mod_to_int")
        return out

    def ntt(self, polys, inverse: bool = False):
        """In place on a device tensor [count][k][n]."""
        _check(lib().fhe_ntt(self._h, 1 if inverse else 0, _dptr(polys), polys.shape[0], _stream()),
               "fhe_ntt")
        return polys

    # ------------------------------------------------------------ timing ---
    def ntt_pass0(self, polys, mfma: bool, reps: int = 1):
        """Levels 0..3 of the forward transform, `reps` times, in place
        ([count][k][n]); mfma: on the int8 matrix cores, else on the vector
        ALU (same words)."""
        _check(lib().fhe_ntt_pass0(self._h, 1 if mfma else 0, reps, _dptr(polys), polys.shape[0], _stream()),
               "fhe_ntt_pass0")
        return polys

    def set_timing(self, on: bool):
        _check(lib().fhe_set_timing(self._h, 1 if on else 0), "fhe_set_timing")

    def kernel_stats(self) -> dict:
        out = {}
        for kind in range(lib().fhe_kernel_kinds()):
            ms, cnt = ctypes.c_double(), ctypes.c_uint64()
            _check(lib().fhe_kernel_stats(self._h, kind, ctypes.byref(ms), ctypes.byref(cnt)),
                   "fhe_kernel_stats")
            out[lib().fhe_kernel_name(kind).decode()] = (ms.value, cnt.value)
        return out

    def reset_kernel_stats(self):
        _check(lib().fhe_reset_kernel_stats(self._h), "fhe_reset_kernel_stats")

    def fallback_count(self) -> int:
        v = ctypes.c_uint64()
        _check(lib().fhe_fallback_count(self._h, ctypes.byref(v)), "fhe_fallback_count")
        return v.value

    def sync(self):
        """Wait for the current stream; raises FheError on a device fault."""
        _check(lib().fhe_sync(self._h, _stream()), "fhe_sync")


def _multi_parts(parts):
    import torch
    arr = (MulPart * len(parts))()
    keep = []
    for i, (ctx, rlk, a, b, out) in enumerate(parts):
        count = a.shape[0]
        op = OP_SQUARE_RELIN if a.data_ptr() == b.data_ptr() else OP_MUL_RELIN
        need = lib().fhe_workspace_bytes(ctx._h, op, count)
        ws = torch.empty(max(need, 8), dtype=torch.uint8, device=ctx.device)
        keep.append(ws)
        arr[i] = MulPart(ctx._h, _dptr(rlk), _dptr(a), _dptr(b), _dptr(out), count, _dptr(ws), ws.numel())
    return arr, keep


def autotune_mul_relin_multi(parts) -> bool:
    """fhe_autotune_mul_relin_multi on parts as for mul_relin_multi: keeps the
    faster key-switching mode in the first part's context; returns True for the
    persistent launch."""
    arr, keep = _multi_parts(parts)
    mode = ctypes.c_int(0)
    _check(lib().fhe_autotune_mul_relin_multi(arr, len(parts), _stream(), ctypes.byref(mode)),
           "fhe_autotune_mul_relin_multi")
    return bool(mode.value)


def mul_relin_multi(parts):
    """parts: list of (Context, rlk, a, b, out) with device tensors; every part
    gets its own workspace.  One fhe_mul_relin_multi call on the current
    stream; returns the list of outputs.  The workspaces are released to
    torch's allocator on return: the current stream waits for every part, and
    the allocator hands a freed block only to later work on that stream."""
    arr, keep = _multi_parts(parts)
    _check(lib().fhe_mul_relin_multi(arr, len(parts), _stream()), "fhe_mul_relin_multi")
    return [p[4] for p in parts]
