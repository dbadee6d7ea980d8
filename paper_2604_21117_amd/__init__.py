"""Python binding of libgtree.so, the MI355X batched B+-tree library.

Argument marshalling only: every step of build, lookup, insert and range
runs in the library's HIP kernels.  The functions keep the C names
(``tree_build``, ``tree_lookup_batch``, ``tree_insert_batch``,
``tree_range_batch``, ...) and take torch tensors on a HIP device; torch
supplies device memory and streams.  If the library has not been built the
import of a function raises -- there is no fallback path.

Keys and values are uint32 or uint64.  torch stores them in int32 / int64
tensors with the same bits; :func:`to_device` and :func:`to_numpy` convert
from and to numpy's unsigned types.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgtree.so")

GT_OK, GT_ERR_INVALID, GT_ERR_DUPLICATE, GT_ERR_CAPACITY, GT_ERR_ADMISSION, GT_ERR_HIP, GT_ERR_DEVICE = range(7)
INSERTED, UPDATED = 0, 1


class GtError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


class gt_params(C.Structure):
    _fields_ = [("key_bytes", C.c_uint32), ("fanout", C.c_uint32), ("leaf_cap", C.c_uint32),
                ("fill", C.c_float), ("lanes_per_query", C.c_uint32), ("lds_levels", C.c_uint32),
                ("sorted_mode", C.c_uint32), ("queries_per_group", C.c_uint32), ("max_batch", C.c_uint64),
                ("value_coload", C.c_uint32), ("xcd_split", C.c_uint32), ("leaf_stream", C.c_uint32),
                ("reserved", C.c_uint32)]


class gt_tree_stats(C.Structure):
    _fields_ = [("n_keys", C.c_uint64), ("height", C.c_uint32), ("root", C.c_uint32),
                ("inner_used", C.c_uint64), ("inner_cap", C.c_uint64),
                ("leaf_used", C.c_uint64), ("leaf_cap", C.c_uint64),
                ("arena_bytes", C.c_uint64), ("max_batch", C.c_uint64),
                ("error_word", C.c_uint32), ("key_bytes", C.c_uint32)]


_lib = None


def lib():
    """Load libgtree.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2604_21117_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        L.gt_status_str.argtypes = [C.c_int]
        L.gt_status_str.restype = C.c_char_p
        L.tree_arena_bytes.argtypes = [C.POINTER(gt_params), u64, u64]
        L.tree_arena_bytes.restype = u64
        L.tree_build.argtypes = [C.POINTER(gt_params), vp, vp, u64, vp, u64, vp, C.POINTER(vp)]
        L.tree_lookup_batch.argtypes = [vp, vp, u64, vp, vp, vp]
        L.tree_insert_batch.argtypes = [vp, vp, vp, u64, vp, vp]
        L.tree_range_batch.argtypes = [vp, vp, vp, vp, vp, u64, vp, vp, vp, vp]
        L.tree_destroy.argtypes = [vp]
        L.tree_stats.argtypes = [vp, C.POINTER(gt_tree_stats), vp]
        L.tree_device_error.argtypes = [vp, vp]
        L.tree_export.argtypes = [vp, vp, C.POINTER(u64), vp]
        for f in ("tree_build", "tree_lookup_batch", "tree_insert_batch", "tree_range_batch",
                  "tree_destroy", "tree_stats", "tree_device_error", "tree_export"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().gt_status_str(int(s)).decode()


def _check(st: int, what: str):
    if st != GT_OK:
        raise GtError(st, what)


# --------------------------------------------------------------- marshalling

def _torch():
    import torch
    return torch


def to_device(a: np.ndarray, device="cuda"):
    """numpy uint32/uint64/uint8 array -> torch tensor with the same bits."""
    torch = _torch()
    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32}.get(a.dtype)
    t = torch.from_numpy(a.view(view) if view is not None else a)
    return t.to(device)


def to_numpy(t, unsigned_dtype=None) -> np.ndarray:
    a = t.detach().cpu().numpy()
    if unsigned_dtype is not None:
        a = a.view(unsigned_dtype)
    return a


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else 0


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def key_dtype(key_bytes: int):
    torch = _torch()
    return torch.int64 if key_bytes == 8 else torch.int32


# ------------------------------------------------------------------ C names

def make_params(key_bytes: int, fill: float = 1.0, lanes_per_query: int = 0, lds_levels: int = 0,
                queries_per_group: int = 0, max_batch: int = 0, value_coload: int = 0, xcd_split: int = 0,
                leaf_stream: int = 0) -> gt_params:
    return gt_params(key_bytes=key_bytes, fanout=16, leaf_cap=16, fill=fill, lanes_per_query=lanes_per_query,
                     lds_levels=lds_levels, sorted_mode=0, queries_per_group=queries_per_group,
                     max_batch=max_batch, value_coload=value_coload, xcd_split=xcd_split,
                     leaf_stream=leaf_stream, reserved=0)


def tree_arena_bytes(params: gt_params, n: int, leaf_slack: int = 0) -> int:
    return int(lib().tree_arena_bytes(C.byref(params), n, leaf_slack))


def tree_build(params: gt_params, keys, values, arena, stream=None) -> int:
    """Build a tree in `arena` (torch uint8 device tensor); returns the handle."""
    h = C.c_void_p()
    n = 0 if keys is None else keys.numel()
    _check(lib().tree_build(C.byref(params), _ptr(keys) if n else None, _ptr(values) if n else None, n,
                            _ptr(arena), arena.numel(), _stream(stream), C.byref(h)), "tree_build")
    return h.value


def tree_lookup_batch(h, keys, values_out, found_out, stream=None):
    _check(lib().tree_lookup_batch(h, _ptr(keys), keys.numel(), _ptr(values_out), _ptr(found_out),
                                   _stream(stream)), "tree_lookup_batch")


def tree_insert_batch(h, keys, values, status_out, stream=None):
    _check(lib().tree_insert_batch(h, _ptr(keys), _ptr(values), keys.numel(), _ptr(status_out),
                                   _stream(stream)), "tree_insert_batch")


def tree_range_batch(h, lo, hi, max_out, out_offsets, out_keys, out_values, count_out, stream=None):
    _check(lib().tree_range_batch(h, _ptr(lo), _ptr(hi), _ptr(max_out), _ptr(out_offsets), lo.numel(),
                                  _ptr(out_keys), _ptr(out_values), _ptr(count_out), _stream(stream)),
           "tree_range_batch")


def tree_destroy(h):
    _check(lib().tree_destroy(h), "tree_destroy")


def tree_stats(h, stream=None) -> dict:
    s = gt_tree_stats()
    _check(lib().tree_stats(h, C.byref(s), _stream(stream)), "tree_stats")
    return {f: getattr(s, f) for f, _ in gt_tree_stats._fields_}


def tree_device_error(h, stream=None) -> int:
    return int(lib().tree_device_error(h, _stream(stream)))


def tree_export(h, stream=None) -> np.ndarray:
    n = C.c_uint64(0)
    _check(lib().tree_export(h, None, C.byref(n), _stream(stream)), "tree_export")
    buf = np.zeros(n.value, dtype=np.uint8)
    _check(lib().tree_export(h, buf.ctypes.data_as(C.c_void_p), C.byref(n), _stream(stream)), "tree_export")
    return buf


# ------------------------------------------------------------ convenience

class Tree:
    """Owns an arena tensor and a tree handle; methods allocate outputs."""

    def __init__(self, keys: np.ndarray, values: np.ndarray, key_bytes: int, leaf_slack: int = 0,
                 arena_bytes: int | None = None, device="cuda", **param_kw):
        torch = _torch()
        self.kb = key_bytes
        self.udtype = np.uint64 if key_bytes == 8 else np.uint32
        self.tdtype = key_dtype(key_bytes)
        self.device = device
        self.params = make_params(key_bytes, **param_kw)
        n = len(keys)
        need = arena_bytes if arena_bytes is not None else tree_arena_bytes(self.params, n, leaf_slack)
        if need == 0:
            raise GtError(GT_ERR_INVALID, "tree_arena_bytes")
        self.arena = torch.empty(need, dtype=torch.uint8, device=device)
        k = to_device(np.asarray(keys, dtype=self.udtype), device) if n else None
        v = to_device(np.asarray(values, dtype=self.udtype), device) if n else None
        self.h = tree_build(self.params, k, v, self.arena)

    def close(self):
        if getattr(self, "h", None):
            tree_destroy(self.h)
            self.h = None

    __del__ = close

    def dev(self, a: np.ndarray):
        return to_device(np.asarray(a, dtype=self.udtype), self.device)

    def lookup_dev(self, q, stream=None):
        torch = _torch()
        vo = torch.empty(q.numel(), dtype=self.tdtype, device=self.device)
        fo = torch.empty(q.numel(), dtype=torch.uint8, device=self.device)
        tree_lookup_batch(self.h, q, vo, fo, stream)
        return vo, fo

    def lookup(self, q: np.ndarray):
        vo, fo = self.lookup_dev(self.dev(q))
        return to_numpy(vo, self.udtype), to_numpy(fo)

    def insert(self, k: np.ndarray, v: np.ndarray, check: bool = True):
        torch = _torch()
        kd, vd = self.dev(k), self.dev(v)
        st = torch.empty(kd.numel(), dtype=torch.uint8, device=self.device)
        tree_insert_batch(self.h, kd, vd, st)
        if check:
            _check(tree_device_error(self.h), "tree_insert_batch (device)")
        return to_numpy(st)

    def range(self, lo: np.ndarray, hi: np.ndarray, maxc: np.ndarray):
        torch = _torch()
        mc = np.asarray(maxc, dtype=np.uint32)
        off = np.zeros(len(mc), dtype=np.uint64)
        if len(mc) > 1:
            off[1:] = np.cumsum(mc.astype(np.uint64))[:-1]
        tot = int(mc.astype(np.uint64).sum())
        ok = torch.empty(max(tot, 1), dtype=self.tdtype, device=self.device)
        ov = torch.empty(max(tot, 1), dtype=self.tdtype, device=self.device)
        cnt = torch.empty(len(mc), dtype=torch.int32, device=self.device)
        tree_range_batch(self.h, self.dev(lo), self.dev(hi), to_device(mc, self.device),
                         to_device(off, self.device), ok, ov, cnt)
        return (to_numpy(cnt, np.uint32), off, to_numpy(ok, self.udtype)[:tot], to_numpy(ov, self.udtype)[:tot])

    def stats(self):
        return tree_stats(self.h)

    def export(self):
        return tree_export(self.h)
