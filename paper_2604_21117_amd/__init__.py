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


class gt_li_params(C.Structure):
    _fields_ = [("models", C.c_uint32), ("kind", C.c_uint32), ("max_window", C.c_uint32), ("search", C.c_uint32),
                ("gate", C.c_uint32), ("reserved", C.c_uint32 * 2)]


class gt_li_stats(C.Structure):
    _fields_ = [("trained_leaves", C.c_uint64), ("trained_keys", C.c_uint64), ("lookups", C.c_uint64),
                ("fallbacks", C.c_uint64), ("models", C.c_uint32), ("linear_models", C.c_uint32),
                ("mlp_models", C.c_uint32), ("tree_models", C.c_uint32), ("max_window", C.c_uint32),
                ("declined", C.c_uint32), ("mean_window", C.c_double)]


class gt_srv_params(C.Structure):
    _fields_ = [("read_streams", C.c_uint32), ("slots", C.c_uint32), ("mem_cap", C.c_uint64),
                ("max_batch", C.c_uint32), ("max_range", C.c_uint32), ("use_graphs", C.c_uint32),
                ("retrain_log2", C.c_uint32)]


class gt_request(C.Structure):
    _fields_ = [("op", C.c_uint32), ("B", C.c_uint32), ("keys", C.c_void_p), ("values", C.c_void_p),
                ("max_out", C.c_void_p), ("out0", C.c_void_p), ("out1", C.c_void_p), ("count_out", C.c_void_p),
                ("arrival_s", C.c_double)]


class gt_srv_stats(C.Structure):
    _fields_ = [("done", C.c_uint64 * 4), ("ops", C.c_uint64 * 4), ("refused", C.c_uint64),
                ("graph_launches", C.c_uint64), ("direct_launches", C.c_uint64), ("wall_s", C.c_double),
                ("p50_us", C.c_double), ("p99_us", C.c_double), ("p50_us_op", C.c_double * 4),
                ("p99_us_op", C.c_double * 4), ("busy_frac", C.c_double), ("retrains", C.c_uint64),
                ("retrain_s", C.c_double), ("captures", C.c_uint64), ("capture_s", C.c_double),
                ("precaptured", C.c_uint64)]


OP_LOOKUP, OP_INSERT, OP_RANGE, OP_DELETE = 0, 1, 2, 3
REQ_QUEUED, REQ_INFLIGHT, REQ_DONE, REQ_REFUSED = 0, 1, 2, 3

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
        L.tree_lookup_levelwise_workspace_bytes.argtypes = [vp, u64, u32]
        L.tree_lookup_levelwise_workspace_bytes.restype = u64
        L.tree_lookup_levelwise.argtypes = [vp, vp, u64, u32, vp, vp, vp, u64, vp]
        L.tree_lookup_levelwise_noalloc.argtypes = [vp, vp, u64, u32, vp, vp, vp]
        L.gt_probe_empty.argtypes = [vp]
        L.gt_probe_xcc.argtypes = [vp, u32, vp]
        L.gt_probe_chase.argtypes = [vp, u64, u64, vp, vp]
        L.gt_probe_gather.argtypes = [vp, u64, u64, u32, u64, vp, vp]
        L.gt_probe_batch.argtypes = [vp, u64, vp, u64, u32, vp, u64, u32, u32, vp, vp]
        L.tree_insert_batch.argtypes = [vp, vp, vp, u64, vp, vp]
        L.tree_delete_batch.argtypes = [vp, vp, u64, vp, vp]
        L.tree_range_batch.argtypes = [vp, vp, vp, vp, vp, u64, vp, vp, vp, vp]
        L.tree_destroy.argtypes = [vp]
        L.tree_stats.argtypes = [vp, C.POINTER(gt_tree_stats), vp]
        L.tree_device_error.argtypes = [vp, vp]
        L.tree_export.argtypes = [vp, vp, C.POINTER(u64), vp]
        L.gt_set_sort_spin_limit.argtypes = [u32]
        L.gt_set_sort_spin_limit.restype = u32
        L.gt_set_single_key_insert.argtypes = [C.c_int]
        L.gt_set_single_key_insert.restype = C.c_int
        L.gt_set_one_launch_insert.argtypes = [C.c_int]
        L.gt_set_one_launch_insert.restype = C.c_int
        L.gt_set_one_launch_delete.argtypes = [C.c_int]
        L.gt_set_one_launch_delete.restype = C.c_int
        L.li_arena_bytes.argtypes = [vp, C.POINTER(gt_li_params)]
        L.li_arena_bytes.restype = u64
        L.li_create.argtypes = [vp, C.POINTER(gt_li_params), vp, u64, C.POINTER(vp)]
        L.li_train.argtypes = [vp, vp]
        L.li_lookup_batch.argtypes = [vp, vp, u64, vp, vp, vp]
        L.li_predict.argtypes = [vp, vp, u64, vp, vp, vp, vp, vp, vp]
        L.li_set_bounds.argtypes = [vp, C.c_int32, C.c_int32, vp]
        L.li_stats.argtypes = [vp, C.POINTER(gt_li_stats), vp]
        L.li_destroy.argtypes = [vp]
        L.srv_create.argtypes = [vp, vp, C.POINTER(gt_srv_params), C.POINTER(vp)]
        L.srv_submit.argtypes = [vp, C.POINTER(gt_request), C.POINTER(u64)]
        L.srv_poll.argtypes = [vp, u64, C.POINTER(u32)]
        L.srv_wait.argtypes = [vp, u64]
        L.srv_replay.argtypes = [vp, vp, u64]
        L.srv_stats.argtypes = [vp, C.POINTER(gt_srv_stats)]
        L.srv_latencies.argtypes = [vp, vp, u64]
        L.srv_destroy.argtypes = [vp]
        for f in ("tree_build", "tree_lookup_batch", "tree_insert_batch", "tree_delete_batch", "tree_range_batch",
                  "tree_destroy", "tree_stats", "tree_device_error", "tree_export", "li_create", "li_train",
                  "li_lookup_batch", "li_predict", "li_set_bounds", "li_stats", "li_destroy", "srv_create",
                  "srv_submit", "srv_poll", "srv_wait", "srv_replay", "srv_stats", "srv_latencies",
                  "srv_destroy"):
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


GT_LW_PRESORTED = 1
GT_LW_NOALLOC_SCRATCH_BYTES = 16 << 20


def tree_lookup_levelwise_workspace_bytes(h, B: int, flags: int = 0) -> int:
    return lib().tree_lookup_levelwise_workspace_bytes(h, B, flags)


def tree_lookup_levelwise(h, keys, flags, values_out, found_out, workspace, stream=None):
    _check(lib().tree_lookup_levelwise(h, _ptr(keys), keys.numel(), flags, _ptr(values_out), _ptr(found_out),
                                       _ptr(workspace), workspace.numel(), _stream(stream)),
           "tree_lookup_levelwise")


def tree_lookup_levelwise_noalloc(h, keys, flags, values_out, found_out, stream=None):
    _check(lib().tree_lookup_levelwise_noalloc(h, _ptr(keys), keys.numel(), flags, _ptr(values_out),
                                               _ptr(found_out), _stream(stream)),
           "tree_lookup_levelwise_noalloc")


def tree_insert_batch(h, keys, values, status_out, stream=None):
    _check(lib().tree_insert_batch(h, _ptr(keys), _ptr(values), keys.numel(), _ptr(status_out),
                                   _stream(stream)), "tree_insert_batch")


def tree_delete_batch(h, keys, status_out, stream=None):
    _check(lib().tree_delete_batch(h, _ptr(keys), keys.numel(), _ptr(status_out), _stream(stream)),
           "tree_delete_batch")


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


def set_sort_spin_limit(limit: int) -> int:
    """Testing hook: the device sort's look-back limit (0 makes every sort
    of more than 4096 keys fail); returns the previous value."""
    return int(lib().gt_set_sort_spin_limit(limit))


def set_single_key_insert(enable: bool) -> bool:
    """Testing switch: a one-key insert batch runs in its own kernel (True,
    the default) or through the batch path (False); returns the previous
    setting."""
    return bool(lib().gt_set_single_key_insert(1 if enable else 0))


def set_one_launch_insert(enable: bool) -> bool:
    """Testing switch: an insert batch of 2 to 64 keys runs in one launch
    (True, the default) or through the small-batch path's four kernels
    (False); returns the previous setting."""
    return bool(lib().gt_set_one_launch_insert(1 if enable else 0))


def set_one_launch_delete(enable: bool) -> bool:
    """Testing switch: a delete batch of at most 64 keys runs in one launch
    (True, the default) or through the batch path's kernels (False); returns
    the previous setting."""
    return bool(lib().gt_set_one_launch_delete(1 if enable else 0))


def tree_export(h, stream=None) -> np.ndarray:
    n = C.c_uint64(0)
    _check(lib().tree_export(h, None, C.byref(n), _stream(stream)), "tree_export")
    buf = np.zeros(n.value, dtype=np.uint8)
    _check(lib().tree_export(h, buf.ctypes.data_as(C.c_void_p), C.byref(n), _stream(stream)), "tree_export")
    return buf


def li_params(models: int = 0, kind: int = 0, max_window: int = 0, search: int = 0, gate: int = 0) -> gt_li_params:
    return gt_li_params(models=models, kind=kind, max_window=max_window, search=search, gate=gate)


def li_arena_bytes(h, params: gt_li_params) -> int:
    return int(lib().li_arena_bytes(h, C.byref(params)))


def li_create(h, params: gt_li_params, arena) -> int:
    out = C.c_void_p()
    _check(lib().li_create(h, C.byref(params), _ptr(arena), arena.numel(), C.byref(out)), "li_create")
    return out.value


def li_train(li, stream=None):
    _check(lib().li_train(li, _stream(stream)), "li_train")


def li_lookup_batch(li, keys, values_out, found_out, stream=None):
    _check(lib().li_lookup_batch(li, _ptr(keys), keys.numel(), _ptr(values_out), _ptr(found_out),
                                 _stream(stream)), "li_lookup_batch")


def li_predict(li, keys, model_out, pred_out, lo_out, hi_out, kind_out, stream=None):
    _check(lib().li_predict(li, _ptr(keys), keys.numel(), _ptr(model_out), _ptr(pred_out), _ptr(lo_out),
                            _ptr(hi_out), _ptr(kind_out), _stream(stream)), "li_predict")


def li_set_bounds(li, lo: int, hi: int, stream=None):
    _check(lib().li_set_bounds(li, lo, hi, _stream(stream)), "li_set_bounds")


def li_stats(li, stream=None) -> dict:
    s = gt_li_stats()
    _check(lib().li_stats(li, C.byref(s), _stream(stream)), "li_stats")
    return {f: getattr(s, f) for f, _ in gt_li_stats._fields_}


def li_destroy(li):
    _check(lib().li_destroy(li), "li_destroy")


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
        h = getattr(self, "h", None)
        if h:
            self.h = None
            tree_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

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

    def levelwise_workspace(self, B: int, presorted: bool = False):
        torch = _torch()
        flags = GT_LW_PRESORTED if presorted else 0
        n = tree_lookup_levelwise_workspace_bytes(self.h, B, flags)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)

    def lookup_levelwise_dev(self, q, presorted: bool = False, workspace=None, stream=None):
        torch = _torch()
        vo = torch.empty(q.numel(), dtype=self.tdtype, device=self.device)
        fo = torch.empty(q.numel(), dtype=torch.uint8, device=self.device)
        ws = workspace if workspace is not None else self.levelwise_workspace(q.numel(), presorted)
        tree_lookup_levelwise(self.h, q, GT_LW_PRESORTED if presorted else 0, vo, fo, ws, stream)
        return vo, fo

    def lookup_levelwise(self, q: np.ndarray, presorted: bool = False):
        vo, fo = self.lookup_levelwise_dev(self.dev(q), presorted)
        return to_numpy(vo, self.udtype), to_numpy(fo)

    def insert(self, k: np.ndarray, v: np.ndarray, check: bool = True):
        torch = _torch()
        kd, vd = self.dev(k), self.dev(v)
        st = torch.empty(kd.numel(), dtype=torch.uint8, device=self.device)
        tree_insert_batch(self.h, kd, vd, st)
        if check:
            _check(tree_device_error(self.h), "tree_insert_batch (device)")
        return to_numpy(st)

    def delete(self, k: np.ndarray, check: bool = True):
        torch = _torch()
        kd = self.dev(k)
        st = torch.empty(kd.numel(), dtype=torch.uint8, device=self.device)
        tree_delete_batch(self.h, kd, st)
        if check:
            _check(tree_device_error(self.h), "tree_delete_batch (device)")
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


# ------------------------------------------------ memory-system probes

def probe_empty(stream=None):
    _check(lib().gt_probe_empty(_stream(stream)), "gt_probe_empty")


def probe_xcc(out, workgroups: int, stream=None):
    _check(lib().gt_probe_xcc(_ptr(out), workgroups, _stream(stream)), "gt_probe_xcc")


def probe_chase(next_idx, steps: int, start: int, out, stream=None):
    _check(lib().gt_probe_chase(_ptr(next_idx), steps, start, _ptr(out), _stream(stream)), "gt_probe_chase")


def probe_gather(region, lines: int, n: int, per_group: int, seed: int, out, stream=None):
    _check(lib().gt_probe_gather(_ptr(region), lines, n, per_group, seed, _ptr(out), _stream(stream)),
           "gt_probe_gather")


def probe_batch(q, table, table_lines: int, table_rounds: int, region, region_lines: int, region_rounds: int,
                lines_per_round: int, out, stream=None):
    _check(lib().gt_probe_batch(_ptr(q), q.numel(), _ptr(table), table_lines, table_rounds, _ptr(region),
                                region_lines, region_rounds, lines_per_round, _ptr(out), _stream(stream)),
           "gt_probe_batch")


def make_static_params(key_bytes: int, fanout: int, fill: float = 1.0) -> gt_params:
    """Parameters of the static tree of the paper's key and node variants:
    key_bytes 32 with fanout 16, 32 or 64, or key_bytes 8 with fanout 32 or
    64 (leaves of fanout - 1 keys)."""
    return gt_params(key_bytes=key_bytes, fanout=fanout, leaf_cap=0, fill=fill, lanes_per_query=0, lds_levels=0,
                     sorted_mode=0, queries_per_group=0, max_batch=0, value_coload=0, xcd_split=0, leaf_stream=0,
                     reserved=0)


class StaticTree:
    """A static tree of 32-byte keys (orders 16, 32, 64) or 8-byte keys
    (orders 32, 64) with 8-byte values, through the same C calls as
    :class:`Tree`.  32-byte keys are numpy (n, 32) uint8 arrays; 8-byte keys
    uint64 arrays.  Owns its arena tensor and handle."""

    def __init__(self, keys: np.ndarray, values: np.ndarray, key_bytes: int, fanout: int, fill: float = 1.0,
                 device="cuda"):
        torch = _torch()
        self.kb, self.m, self.device = key_bytes, fanout, device
        self.params = make_static_params(key_bytes, fanout, fill)
        k = self._rows(keys)
        n = len(k)
        need = tree_arena_bytes(self.params, n)
        if need == 0:
            raise GtError(GT_ERR_INVALID, "tree_arena_bytes")
        self.arena = torch.empty(need, dtype=torch.uint8, device=device)
        kd = self.dev_keys(k) if n else None
        vd = to_device(np.asarray(values, dtype=np.uint64), device) if n else None
        h = C.c_void_p()
        _check(lib().tree_build(C.byref(self.params), _ptr(kd), _ptr(vd), n, _ptr(self.arena), self.arena.numel(),
                                _stream(None), C.byref(h)), "tree_build")
        self.h = h.value

    def _rows(self, a) -> np.ndarray:
        if self.kb == 8:
            return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
        a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8))
        return a.reshape(-1, self.kb)

    def dev_keys(self, a):
        """Keys to a device tensor of len(a) * key_bytes bytes."""
        r = self._rows(a)
        return to_device(r.view(np.uint8).reshape(-1) if self.kb == 32 else r, self.device)

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            tree_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

    def lookup_dev(self, qd, B: int, stream=None):
        torch = _torch()
        vo = torch.empty(B, dtype=torch.int64, device=self.device)
        fo = torch.empty(B, dtype=torch.uint8, device=self.device)
        _check(lib().tree_lookup_batch(self.h, _ptr(qd), B, _ptr(vo), _ptr(fo), _stream(stream)), "tree_lookup_batch")
        return vo, fo

    def lookup(self, q: np.ndarray):
        r = self._rows(q)
        vo, fo = self.lookup_dev(self.dev_keys(r), len(r))
        return to_numpy(vo, np.uint64), to_numpy(fo)

    def range(self, lo: np.ndarray, hi: np.ndarray, maxc: np.ndarray):
        torch = _torch()
        lo, hi = self._rows(lo), self._rows(hi)
        mc = np.asarray(maxc, dtype=np.uint32)
        B = len(mc)
        off = np.zeros(B, dtype=np.uint64)
        if B > 1:
            off[1:] = np.cumsum(mc.astype(np.uint64))[:-1]
        tot = int(mc.astype(np.uint64).sum())
        ok = torch.empty(max(tot, 1) * self.kb, dtype=torch.uint8, device=self.device)
        ov = torch.empty(max(tot, 1), dtype=torch.int64, device=self.device)
        cnt = torch.empty(max(B, 1), dtype=torch.int32, device=self.device)
        # the input tensors stay referenced until the call has enqueued its
        # kernel (a freed block could be handed to the next allocation)
        lod, hid = self.dev_keys(lo), self.dev_keys(hi)
        mcd, offd = to_device(mc, self.device), to_device(off, self.device)
        _check(lib().tree_range_batch(self.h, _ptr(lod), _ptr(hid), _ptr(mcd), _ptr(offd), B,
                                      _ptr(ok), _ptr(ov), _ptr(cnt), _stream(None)), "tree_range_batch")
        keys = to_numpy(ok)[:tot * self.kb]
        keys = keys.reshape(tot, self.kb) if self.kb == 32 else keys.view(np.uint64)
        return to_numpy(cnt, np.uint32)[:B], off, keys, to_numpy(ov, np.uint64)[:tot]

    def stats(self):
        return tree_stats(self.h)

    def export(self):
        return tree_export(self.h)


class Learned:
    """A learned index over a :class:`Tree` (owns its arena tensor)."""

    def __init__(self, tree: Tree, models: int = 0, kind: int = 0, max_window: int = 0, search: int = 0,
                 gate: int = 0):
        torch = _torch()
        self.tree = tree
        self.params = li_params(models, kind, max_window, search, gate)
        n = li_arena_bytes(tree.h, self.params)
        if n == 0:
            raise GtError(GT_ERR_INVALID, "li_arena_bytes")
        self.arena = torch.empty(n, dtype=torch.uint8, device=tree.device)
        self.h = li_create(tree.h, self.params, self.arena)

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            li_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

    def train(self):
        li_train(self.h)

    def lookup_dev(self, q, stream=None):
        torch = _torch()
        vo = torch.empty(q.numel(), dtype=self.tree.tdtype, device=self.tree.device)
        fo = torch.empty(q.numel(), dtype=torch.uint8, device=self.tree.device)
        li_lookup_batch(self.h, q, vo, fo, stream)
        return vo, fo

    def lookup(self, q: np.ndarray):
        vo, fo = self.lookup_dev(self.tree.dev(q))
        return to_numpy(vo, self.tree.udtype), to_numpy(fo)

    def predict(self, q: np.ndarray):
        torch = _torch()
        qd = self.tree.dev(q)
        n, dev = qd.numel(), self.tree.device
        mo = torch.empty(n, dtype=torch.int32, device=dev)
        po = torch.empty(n, dtype=torch.int32, device=dev)
        lo = torch.empty(n, dtype=torch.int32, device=dev)
        hi = torch.empty(n, dtype=torch.int32, device=dev)
        ko = torch.empty(n, dtype=torch.uint8, device=dev)
        li_predict(self.h, qd, mo, po, lo, hi, ko)
        return to_numpy(mo), to_numpy(po), to_numpy(lo), to_numpy(hi), to_numpy(ko)

    def set_bounds(self, lo: int, hi: int):
        li_set_bounds(self.h, lo, hi)

    def stats(self):
        return li_stats(self.h)


# ----------------------------------------------------------------- serving

def srv_params(read_streams=0, slots=0, mem_cap=0, max_batch=0, max_range=0, use_graphs=0,
               retrain_log2=0) -> gt_srv_params:
    return gt_srv_params(read_streams=read_streams, slots=slots, mem_cap=mem_cap, max_batch=max_batch,
                         max_range=max_range, use_graphs=use_graphs, retrain_log2=retrain_log2)


class Batch:
    """One serving request with its host buffers (numpy arrays kept alive)."""

    def __init__(self, op: int, keys: np.ndarray, values: np.ndarray | None = None,
                 max_out: np.ndarray | None = None, arrival_s: float = 0.0):
        self.op = op
        self.keys = np.ascontiguousarray(keys)
        dt = self.keys.dtype
        B = len(self.keys)
        self.values = None if values is None else np.ascontiguousarray(values, dtype=dt)
        self.max_out = None if max_out is None else np.ascontiguousarray(max_out, dtype=np.uint32)
        self.count = None
        if op == OP_LOOKUP:
            self.out0 = np.empty(B, dtype=dt)
            self.out1 = np.empty(B, dtype=np.uint8)
        elif op in (OP_INSERT, OP_DELETE):
            self.out0 = np.empty(B, dtype=np.uint8)
            self.out1 = None
        else:
            tot = int(self.max_out.astype(np.uint64).sum())
            self.out0 = np.zeros(max(tot, 1), dtype=dt)
            self.out1 = np.zeros(max(tot, 1), dtype=dt)
            self.count = np.empty(B, dtype=np.uint32)
        self.arrival_s = arrival_s

    def struct(self) -> gt_request:
        p = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None  # noqa: E731
        return gt_request(op=self.op, B=len(self.keys), keys=p(self.keys), values=p(self.values),
                          max_out=p(self.max_out), out0=p(self.out0), out1=p(self.out1),
                          count_out=p(self.count), arrival_s=self.arrival_s)


class Server:
    def __init__(self, tree: Tree, learned: "Learned | None" = None, **kw):
        self.tree, self.learned = tree, learned
        self.params = srv_params(**kw)
        h = C.c_void_p()
        _check(lib().srv_create(tree.h, learned.h if learned is not None else None, C.byref(self.params),
                                C.byref(h)), "srv_create")
        self.h = h.value

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            lib().srv_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may be gone
            pass

    def submit(self, b: Batch) -> int:
        t = C.c_uint64()
        b._s = b.struct()
        _check(lib().srv_submit(self.h, C.byref(b._s), C.byref(t)), "srv_submit")
        return t.value

    def wait(self, ticket: int) -> int:
        return int(lib().srv_wait(self.h, ticket))

    def poll(self, ticket: int) -> int:
        s = C.c_uint32()
        _check(lib().srv_poll(self.h, ticket, C.byref(s)), "srv_poll")
        return s.value

    def replay(self, batches: list) -> int:
        arr = (gt_request * len(batches))(*[b.struct() for b in batches])
        return int(lib().srv_replay(self.h, C.cast(arr, C.c_void_p), len(batches)))

    def stats(self) -> dict:
        s = gt_srv_stats()
        _check(lib().srv_stats(self.h, C.byref(s)), "srv_stats")
        d = {f: getattr(s, f) for f, _ in gt_srv_stats._fields_}
        for f in ("done", "ops", "p50_us_op", "p99_us_op"):
            d[f] = list(d[f])
        return d

    def latencies(self, n: int) -> np.ndarray:
        out = np.empty(n, dtype=np.float64)
        _check(lib().srv_latencies(self.h, out.ctypes.data_as(C.c_void_p), n), "srv_latencies")
        return out
