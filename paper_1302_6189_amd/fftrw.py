"""ctypes binding for libfftrw.so (include/fftrw.h): argument marshalling only.

Every computation runs in the native library: the host integer functions in
C++, the transforms and transposes in HIP kernels on the GPU.  There is no
Python or CPU fallback; if the library is missing, ``lib()`` raises.

Orders and permutations may be given as sequences of axis indices or as
strings in the paper's notation ("abc->acb->bca").  Device buffers are torch
tensors (complex64 or complex128, contiguous) or raw integer pointers.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfftrw.so")

OK, E_ARG, E_SIZE, E_ORDER, E_ROWSPLIT, E_NOMEM, E_DEVICE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
C64, C128 = 1, 2
PREC_NATIVE, PREC_SPLIT_F16, PREC_SPLIT_BF16, PREC_SPLIT_BF16X3 = 0, 1, 2, 3
OWN_LITERAL, OWN_MATCHED = 0, 1
FLAG_LEAVE_PERMUTED, FLAG_STAGED, FLAG_COUNT_MOVED, FLAG_OWN_MATCHED, FLAG_FUSED_FFT = 1, 2, 4, 8, 16
FLAG_BATCH_NO_GRAPH = 32
FLAG_BATCH_NO_FUSE = 64
FLAG_SEPARATE = 128

LETTERS = "abcdefgh"

_lib = None


class FftrwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fftrw error {code}: {msg}")
        self.code = code


class ItemDesc(ctypes.Structure):
    """fft_item_desc"""
    _fields_ = [("M", ctypes.c_int), ("dims", ctypes.c_int64 * 5), ("P", ctypes.c_int64),
                ("order", ctypes.c_int8 * 25), ("has_order", ctypes.c_int)]


_i64p = ctypes.POINTER(ctypes.c_int64)
_i8p = ctypes.POINTER(ctypes.c_int8)
_vp = ctypes.c_void_p

_SIGNATURES = {
    "fft_decomp": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, _i8p, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_int), _i64p, _i64p, _i64p, _i64p]),
    "fft_comm_volume": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, _i8p, ctypes.c_int,
                                       _i64p, _i64p, _i64p]),
    "fft_rowsplit_volume": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, _i8p, _i64p, _i64p]),
    "fft_fused_unit_shape": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "fft_pair_counts": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, _i8p, _i8p, _i64p]),
    "fft_transpose_volumes": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, _i64p]),
    "fft_order_count": (ctypes.c_int64, [ctypes.c_int]),
    "fft_order_at": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, _i8p]),
    "fft_order_index": (ctypes.c_int, [ctypes.c_int, _i8p, _i64p]),
    "fft_order_search": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int,
                                        _i64p, _i64p, _i64p, _i64p, _i64p, _i64p, _i8p, _i8p]),
    "fft_order_volumes": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, ctypes.c_int, _i64p]),
    "fft_compare_models": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "fft_plan": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _i64p, ctypes.c_int64, _i8p,
                                ctypes.c_int, ctypes.c_int, ctypes.c_uint]),
    "fft_exec_noalloc": (ctypes.c_int, [ctypes.c_int, _i64p, ctypes.c_int64, _i8p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint, ctypes.c_int, _vp, _vp, _vp]),
    "fft_exec_fwd": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "fft_exec_inv": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "fft_exec_fft_step": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "fft_exec_transpose": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "fft_plan_stats": (ctypes.c_int, [_vp, _i64p, _i64p]),
    "fft_plan_messages": (ctypes.c_int, [_vp, _i64p]),
    "fft_plan_rowsplit_stats": (ctypes.c_int, [_vp, _i64p, _i64p]),
    "fft_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "fft_plan_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "fft_plan_timings": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "fft_plan_describe": (ctypes.c_int, [_vp, _i8p, ctypes.c_char_p, ctypes.c_size_t]),
    "fft_destroy": (ctypes.c_int, [_vp]),
    "fft_batch_plan": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_char_p, ctypes.c_uint]),
    "fft_batch_exec_fwd": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "fft_batch_exec_inv": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "fft_batch_stats": (ctypes.c_int, [_vp, _i64p, _i64p, _i64p, ctypes.POINTER(ctypes.c_int)]),
    "fft_batch_destroy": (ctypes.c_int, [_vp]),
    "fft_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_uint]),
    "fft_last_error": (ctypes.c_char_p, []),
    "fft_version": (ctypes.c_char_p, []),
}


def lib():
    """Load libfftrw.so (built by ``paper_1302_6189_amd.build``); no fallback."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime and loads it by a different file name
        # than the one this library links against; loading torch first makes
        # both resolve to that single runtime (two runtimes in one process do
        # not share devices).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise FftrwError(E_DEVICE, f"{LIB_PATH} is missing: run `python -m paper_1302_6189_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(rc: int):
    if rc != OK:
        raise FftrwError(rc, lib().fft_last_error().decode())


# ---- marshalling helpers ---------------------------------------------------------
def perm_from(p, M=None):
    if isinstance(p, str):
        return tuple(LETTERS.index(c) for c in p.strip())
    return tuple(int(a) for a in p)


def order_from(order, M=None):
    """Order as a tuple of permutations from a string or a sequence."""
    if isinstance(order, str):
        parts = order.replace("→", "->").split("->")
        return tuple(perm_from(s) for s in parts)
    arr = np.asarray(order)
    if arr.ndim == 1 and M is not None:
        arr = arr.reshape(M, M)
    return tuple(tuple(int(x) for x in row) for row in arr)


def order_to_str(order) -> str:
    return "->".join("".join(LETTERS[a] for a in p) for p in order)


def _dims(dims):
    return (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])


def _perm(p):
    return (ctypes.c_int8 * len(p))(*p)


def _order(order):
    flat = [a for p in order for a in p]
    return (ctypes.c_int8 * len(flat))(*flat)


# ---- host integer functions ------------------------------------------------------
def fft_decomp(dims, P, perm, myid):
    M = len(dims)
    perm = perm_from(perm)
    lev = ctypes.c_int()
    xs, xe = ctypes.c_int64(), ctypes.c_int64()
    st, en = (ctypes.c_int64 * M)(), (ctypes.c_int64 * M)()
    _check(lib().fft_decomp(M, _dims(dims), int(P), _perm(perm), int(myid), ctypes.byref(lev),
                            ctypes.byref(xs), ctypes.byref(xe), st, en))
    return lev.value, xs.value, xe.value, tuple(st), tuple(en)


def fft_comm_volume(dims, P, order, ownership=OWN_LITERAL, allow_rowsplit=False):
    """(per_step list, total, return_volume) of a transpose order."""
    M = len(dims)
    order = order_from(order, M)
    per = (ctypes.c_int64 * (M - 1))()
    tot, ret = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().fft_comm_volume(M, _dims(dims), int(P), _order(order), int(ownership), per,
                               ctypes.byref(tot), ctypes.byref(ret))
    if not (allow_rowsplit and rc == E_ROWSPLIT):
        _check(rc)
    return list(per), tot.value, ret.value


def fft_rowsplit_volume(dims, P, order):
    """(per FFT step list, total): points the split rows' own 1-D FFTs would
    exchange at level M under the binary-exchange reading (0 below level M)."""
    M = len(dims)
    order = order_from(order, M)
    per = (ctypes.c_int64 * M)()
    tot = ctypes.c_int64()
    _check(lib().fft_rowsplit_volume(M, _dims(dims), int(P), _order(order), per, ctypes.byref(tot)))
    return list(per), tot.value


def fft_fused_unit_shape(N, Nv, nslices, esz=8):
    """(rw, G) of the fused FFT + transpose unit for rows of N points."""
    rw, G = ctypes.c_int(), ctypes.c_int()
    _check(lib().fft_fused_unit_shape(int(N), int(esz), int(Nv), int(nslices), ctypes.byref(rw), ctypes.byref(G)))
    return rw.value, G.value


def fft_pair_counts(dims, P, perm_a, perm_b):
    M = len(dims)
    C = np.zeros(int(P) * int(P), dtype=np.int64)
    _check(lib().fft_pair_counts(M, _dims(dims), int(P), _perm(perm_from(perm_a)), _perm(perm_from(perm_b)),
                                 C.ctypes.data_as(_i64p)))
    return C.reshape(int(P), int(P))


def fft_transpose_volumes(dims, P, ownership=OWN_LITERAL):
    """(M!, M!) int64 table of single-transpose amounts over the permutations
    in lexicographic order; -1 where no order contains the pair."""
    M = len(dims)
    n = math.factorial(M)
    out = np.zeros(n * n, dtype=np.int64)
    _check(lib().fft_transpose_volumes(M, _dims(dims), int(P), int(ownership), out.ctypes.data_as(_i64p)))
    return out.reshape(n, n)


def fft_order_count(M):
    return int(lib().fft_order_count(int(M)))


def fft_order_at(M, index):
    buf = (ctypes.c_int8 * (M * M))()
    _check(lib().fft_order_at(int(M), int(index), buf))
    return order_from(list(buf), M)


def fft_order_index(order):
    order = order_from(order)
    M = len(order)
    idx = ctypes.c_int64()
    _check(lib().fft_order_index(M, _order(order), ctypes.byref(idx)))
    return idx.value


def fft_order_search(dims, P, ownership=OWN_LITERAL):
    """dict with best/worst canonical index, volume, tie count and order."""
    M = len(dims)
    v = [ctypes.c_int64() for _ in range(6)]
    bo, wo = (ctypes.c_int8 * (M * M))(), (ctypes.c_int8 * (M * M))()
    _check(lib().fft_order_search(M, _dims(dims), int(P), int(ownership), *[ctypes.byref(x) for x in v], bo, wo))
    return {"best_index": v[0].value, "best_volume": v[1].value, "n_best": v[2].value,
            "worst_index": v[3].value, "worst_volume": v[4].value, "n_worst": v[5].value,
            "best_order": order_from(list(bo), M), "worst_order": order_from(list(wo), M)}


def fft_order_volumes(dims, P, ownership=OWN_LITERAL):
    M = len(dims)
    # past five axes the library refuses before writing (one entry per order
    # would be 2.99e12 entries)
    out = np.zeros(fft_order_count(M) if M <= 5 else 1, dtype=np.int64)
    _check(lib().fft_order_volumes(M, _dims(dims), int(P), int(ownership), out.ctypes.data_as(_i64p)))
    return out


def fft_compare_models(N, P):
    out = (ctypes.c_double * 5)()
    _check(lib().fft_compare_models(float(N), float(P), out))
    return tuple(out)


# ---- device plans ---------------------------------------------------------------
def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def fft_exec_noalloc(dims, P, order, direction, x, y, dtype: int = C64, precision: int = PREC_NATIVE,
                     flags: int = 0, stream=None):
    """fft_exec_noalloc: plan and run one transform without device allocation
    (workspace in the library's fixed device array)."""
    dims = tuple(int(d) for d in dims)
    M = len(dims)
    ordp = _order(order_from(order, M)) if order is not None else None
    _check(lib().fft_exec_noalloc(M, _dims(dims), int(P), ordp, int(dtype), int(precision), ctypes.c_uint(int(flags)),
                                  int(direction), _ptr(x), _ptr(y), _stream(stream)))


class Plan:
    """fft_plan_t: one M-D transform of fixed sizes, process count and order."""

    def __init__(self, dims: Sequence[int], P: int, order=None, dtype: int = C64,
                 precision: int = PREC_NATIVE, flags: int = 0):
        self.dims = tuple(int(d) for d in dims)
        self.M = len(self.dims)
        self.P = int(P)
        self.dtype = dtype
        self.flags = int(flags)
        h = _vp()
        ordp = _order(order_from(order, self.M)) if order is not None else None
        _check(lib().fft_plan(ctypes.byref(h), self.M, _dims(self.dims), self.P, ordp, int(dtype),
                              int(precision), ctypes.c_uint(self.flags)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def exec_fwd(self, x, y, stream=None):
        _check(lib().fft_exec_fwd(self._h, _ptr(x), _ptr(y), _stream(stream)))

    def exec_inv(self, x, y, stream=None):
        _check(lib().fft_exec_inv(self._h, _ptr(x), _ptr(y), _stream(stream)))

    def exec_fft_step(self, t, direction, x, y, stream=None):
        _check(lib().fft_exec_fft_step(self._h, int(t), int(direction), _ptr(x), _ptr(y), _stream(stream)))

    def exec_transpose(self, t, x, y, stream=None):
        _check(lib().fft_exec_transpose(self._h, int(t), _ptr(x), _ptr(y), _stream(stream)))

    def stats(self):
        """(analytic amounts [M], device-counted moved points [M] or -1)."""
        a, m = (ctypes.c_int64 * self.M)(), (ctypes.c_int64 * self.M)()
        _check(lib().fft_plan_stats(self._h, a, m))
        return list(a), list(m)

    def set_timing(self, enable=True):
        _check(lib().fft_plan_set_timing(self._h, 1 if enable else 0))

    def rowsplit_stats(self):
        """(per-step split-row exchange amounts, device-counted copies of the last exec)."""
        a = (ctypes.c_int64 * self.M)()
        m = (ctypes.c_int64 * self.M)()
        _check(lib().fft_plan_rowsplit_stats(self._h, a, m))
        return list(a), list(m)

    def messages(self):
        """Messages of each staged transpose: (p, q) pairs, p != q, that exchange points."""
        out = (ctypes.c_int64 * self.M)()
        _check(lib().fft_plan_messages(self._h, out))
        return list(out)

    def timings(self):
        """Per-stage durations (ms) of the last exec: FFT 1, transpose 1, ...
        (a staged transpose is three stages: pack, exchange, unpack)."""
        buf = (ctypes.c_float * (4 * self.M + 1))()
        n = ctypes.c_int()
        _check(lib().fft_plan_timings(self._h, buf, 4 * self.M + 1, ctypes.byref(n)))
        return list(buf)[:n.value]

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        _check(lib().fft_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def describe(self):
        o = (ctypes.c_int8 * (self.M * self.M))()
        txt = ctypes.create_string_buffer(256)
        _check(lib().fft_plan_describe(self._h, o, txt, 256))
        return order_from(list(o), self.M), txt.value.decode()

    def destroy(self):
        if getattr(self, "_h", None):
            lib().fft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _item_array(items):
    arr = (ItemDesc * len(items))()
    for i, it in enumerate(items):
        dims, P = tuple(int(d) for d in it[0]), int(it[1])
        order = it[2] if len(it) > 2 else None
        d = arr[i]
        d.M = len(dims)
        for a, n in enumerate(dims):
            d.dims[a] = n
        d.P = P
        if order is not None:
            flat = [a for p in order_from(order, len(dims)) for a in p]
            for k, a in enumerate(flat):
                d.order[k] = a
            d.has_order = 1
    return arr


def fft_autotune(items, cache_path: str):
    """Time kernel parameters for the items' row lengths and transposes on the
    current device and write the winners to cache_path (JSON)."""
    arr = _item_array(items)
    _check(lib().fft_autotune(len(items), ctypes.cast(arr, ctypes.c_void_p), cache_path.encode(), 0))


class Batch:
    """fft_batch_t: many complex64 transforms in one persistent launch.

    items: sequence of (dims, P) or (dims, P, order); order None = best."""

    def __init__(self, items, flags: int = 0, tune_cache: str | None = None):
        arr = _item_array(items)
        self.items = [(tuple(int(d) for d in it[0]), int(it[1])) for it in items]
        self.n = len(items)
        self.flags = int(flags)
        h = _vp()
        _check(lib().fft_batch_plan(ctypes.byref(h), self.n, ctypes.cast(arr, ctypes.c_void_p), PREC_NATIVE,
                                    tune_cache.encode() if tune_cache else None, ctypes.c_uint(self.flags)))
        self._h = h

    def _ptrs(self, bufs):
        return (_vp * self.n)(*[_ptr(b) for b in bufs])

    def exec_fwd(self, ins, outs, stream=None):
        _check(lib().fft_batch_exec_fwd(self._h, self._ptrs(ins), self._ptrs(outs), _stream(stream)))

    def exec_inv(self, ins, outs, stream=None):
        _check(lib().fft_batch_exec_inv(self._h, self._ptrs(ins), self._ptrs(outs), _stream(stream)))

    def stats(self):
        """dict: per-item lists of device-counted and analytic amounts, units, error flag."""
        tot = sum(len(d) for d, _ in self.items)
        mv, an = (ctypes.c_int64 * tot)(), (ctypes.c_int64 * tot)()
        units, err = ctypes.c_int64(), ctypes.c_int()
        _check(lib().fft_batch_stats(self._h, mv, an, ctypes.byref(units), ctypes.byref(err)))
        out_m, out_a, off = [], [], 0
        for dims, _ in self.items:
            M = len(dims)
            out_m.append(list(mv)[off:off + M])
            out_a.append(list(an)[off:off + M])
            off += M
        return {"moved": out_m, "analytic": out_a, "units": units.value, "error": err.value}

    def destroy(self):
        if getattr(self, "_h", None):
            lib().fft_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
