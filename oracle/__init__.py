"""CPU oracle for the batched B+-tree: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links, loads or
calls it, and the two share no code: the oracle is C compiled with gcc
(``oracle.c``), wrapped here with ctypes and numpy for marshalling only.

Parts (each cited in ``oracle.c``):

* :class:`SortedArray` -- the plain definitions: lookup by binary search,
  an insert or delete batch as its sequential application in batch order,
  range as a sorted slice (paper Section III for the structure, Section IV-D for the
  -1 "not found" result).
* :class:`PointerTree` -- a textbook pointer B+-tree (Section III), the
  timed CPU baseline; lookup batches split evenly over threads (Section V-F).
  Its ``lookup_levelwise`` is the paper's level-by-level search of a sorted
  batch with a FIFO of (node, count) entries (Sections IV-A, IV-F).
* :func:`check_export` -- invariant checker over the flat tree export
  format (sorted leaves, equal depth, fill of at least half, separator
  bounds, leaf chain, reachability, padding).
* :mod:`oracle.brute` -- linear-scan brute force for tiny inputs, which pins
  the two above.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

INSERTED, UPDATED = 0, 1

# violation bits returned by check_export
V_FORMAT, V_SORTED, V_DEPTH, V_FILL, V_COUNT, V_SEPARATOR, V_CHAIN, V_REACH, V_PADDING = \
    (1 << i for i in range(9))
V_NAMES = {V_FORMAT: "format", V_SORTED: "I1 sorted", V_DEPTH: "I2 depth", V_FILL: "I3 fill",
           V_COUNT: "I4 count", V_SEPARATOR: "I5 separator", V_CHAIN: "I6 chain",
           V_REACH: "I7 reach", V_PADDING: "padding"}


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp,
                               SRC_PATH, "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        u64, i32, vp = C.c_uint64, C.c_int, C.c_void_p
        L.ora_lookup.argtypes = [_u64p, _u64p, u64, _u64p, u64, i32, _u64p, _u8p]
        L.ora_insert.argtypes = [_u64p, _u64p, u64, _u64p, _u64p, u64, _u64p, _u64p, _u8p]
        L.ora_insert.restype = u64
        L.ora_delete.argtypes = [_u64p, _u64p, u64, _u64p, u64, _u64p, _u64p, _u8p]
        L.ora_delete.restype = u64
        L.ora_range.argtypes = [_u64p, _u64p, u64, _u64p, _u64p, _u32p, _u64p, u64, _u64p, _u64p, _u32p]
        L.orb_sort.argtypes = [_u8p, _u64p, u64, i32, _u8p, _u64p]
        L.orb_sort.restype = i32
        L.orb_lookup.argtypes = [_u8p, _u64p, u64, i32, _u8p, u64, _u64p, _u8p]
        L.orb_range.argtypes = [_u8p, _u64p, u64, i32, _u8p, _u8p, _u32p, _u64p, u64, _u8p, _u64p, _u32p]
        L.orb_check_export.argtypes = [_u8p, u64, _u8p, _u64p, u64, C.POINTER(u64)]
        L.orb_check_export.restype = C.c_uint32
        L.bpt_create.argtypes = [i32, i32, i32]
        L.bpt_create.restype = vp
        L.bpt_free.argtypes = [vp]
        L.bpt_bulk_load.argtypes = [vp, _u64p, _u64p, u64, C.c_double]
        L.bpt_bulk_load.restype = i32
        L.bpt_insert_batch.argtypes = [vp, _u64p, _u64p, u64, _u8p]
        L.bpt_lookup_batch.argtypes = [vp, _u64p, u64, _u64p, _u8p, i32]
        L.bpt_lookup_batches_timed.argtypes = [vp, _u64p, u64, u64, _u64p, _u8p, i32, _u64p]
        L.bpt_lookup_batches_timed.restype = i32
        L.bpt_range_batch.argtypes = [vp, _u64p, _u64p, _u32p, _u64p, u64, _u64p, _u64p, _u32p]
        L.bpt_stats.argtypes = [vp, _u64p]
        L.bpt_levelwise.argtypes = [vp, _u64p, u64, _u64p, _u8p, _u32p, _u64p, _u64p, _u64p, u64]
        L.bpt_levelwise.restype = C.c_longlong
        L.bpt_export_bytes.argtypes = [vp]
        L.bpt_export_bytes.restype = u64
        L.bpt_export.argtypes = [vp, _u8p, u64]
        L.bpt_export.restype = u64
        L.ora_check_export.argtypes = [_u8p, u64, _u64p, _u64p, u64, C.POINTER(u64)]
        L.ora_check_export.restype = C.c_uint32
        _lib = L
    return _lib


def _w(x) -> np.ndarray:
    if isinstance(x, np.ndarray):
        return np.ascontiguousarray(x.astype(np.uint64))
    # Python ints up to 2^64-1 convert exactly only with an explicit dtype
    return np.ascontiguousarray(np.array([int(v) for v in x], dtype=np.uint64))


def _narrow(x: np.ndarray, width: int) -> np.ndarray:
    return x.astype(np.uint32) if width == 32 else x


def _offsets(maxc) -> np.ndarray:
    m = np.asarray(maxc, dtype=np.uint64)
    off = np.zeros(len(m), dtype=np.uint64)
    if len(m) > 1:
        off[1:] = np.cumsum(m)[:-1]
    return off


def _kb_rows(keys, kb: int) -> np.ndarray:
    """Packed kb-byte keys as a C-contiguous (n, kb) uint8 array."""
    a = np.ascontiguousarray(np.asarray(keys, dtype=np.uint8))
    return a.reshape(-1, kb) if a.size else np.zeros((0, kb), dtype=np.uint8)


class SortedBytes:
    """State S over keys of kb bytes (the paper's 32-byte keys) compared as
    byte strings, byte 0 first, with 8-byte values: sorted distinct keys,
    lookup by binary search, range as a sorted slice (plain definitions)."""

    def __init__(self, keys=None, vals=(), kb: int = 32):
        self.kb = kb
        k = _kb_rows(keys if keys is not None else np.zeros((0, kb), np.uint8), kb)
        v = np.ascontiguousarray(np.asarray(vals, dtype=np.uint64))
        n = len(k)
        self.keys = np.zeros((max(n, 1), kb), dtype=np.uint8)
        self.vals = np.zeros(max(n, 1), dtype=np.uint64)
        if lib().orb_sort(k.reshape(-1) if n else np.zeros(1, np.uint8), v if n else np.zeros(1, np.uint64), n, kb,
                          self.keys.reshape(-1), self.vals):
            raise ValueError("duplicate keys")
        self.keys, self.vals = self.keys[:n], self.vals[:n]

    def __len__(self):
        return len(self.keys)

    def _flat(self):
        return (self.keys.reshape(-1) if len(self.keys) else np.zeros(1, np.uint8),
                self.vals if len(self.vals) else np.zeros(1, np.uint64))

    def lookup(self, q):
        q = _kb_rows(q, self.kb)
        B = len(q)
        vo = np.empty(max(B, 1), dtype=np.uint64)
        fo = np.empty(max(B, 1), dtype=np.uint8)
        k, v = self._flat()
        lib().orb_lookup(k, v, len(self.keys), self.kb, q.reshape(-1) if B else np.zeros(1, np.uint8), B, vo, fo)
        return vo[:B], fo[:B]

    def range(self, lo, hi, maxc):
        lo, hi = _kb_rows(lo, self.kb), _kb_rows(hi, self.kb)
        mc = np.ascontiguousarray(np.asarray(maxc, dtype=np.uint32))
        off = _offsets(mc)
        tot = int(mc.astype(np.uint64).sum())
        ok = np.zeros((max(tot, 1), self.kb), dtype=np.uint8)
        ov = np.zeros(max(tot, 1), dtype=np.uint64)
        cnt = np.zeros(max(len(mc), 1), dtype=np.uint32)
        k, v = self._flat()
        z = np.zeros(1, np.uint8)
        lib().orb_range(k, v, len(self.keys), self.kb, lo.reshape(-1) if len(lo) else z,
                        hi.reshape(-1) if len(hi) else z, mc if len(mc) else np.zeros(1, np.uint32),
                        off if len(off) else np.zeros(1, np.uint64), len(mc), ok.reshape(-1), ov, cnt)
        return cnt[:len(mc)], off, ok, ov


class SortedArray:
    """State S as sorted distinct keys with values (plain definitions)."""

    def __init__(self, keys=(), vals=(), width: int = 64):
        self.width = width
        k = _w(keys)
        v = _w(vals)
        order = np.argsort(k, kind="stable")
        self.keys, self.vals = k[order], v[order]
        if len(self.keys) > 1 and np.any(self.keys[1:] == self.keys[:-1]):
            raise ValueError("duplicate keys")

    def __len__(self):
        return len(self.keys)

    def lookup(self, q):
        q = _w(q)
        vo = np.empty(len(q), dtype=np.uint64)
        fo = np.empty(len(q), dtype=np.uint8)
        lib().ora_lookup(self.keys, self.vals, len(self.keys), q, len(q), self.width, vo, fo)
        return _narrow(vo, self.width), fo

    def insert(self, k, v):
        k, v = _w(k), _w(v)
        n, B = len(self.keys), len(k)
        ok = np.empty(n + B, dtype=np.uint64)
        ov = np.empty(n + B, dtype=np.uint64)
        st = np.empty(B, dtype=np.uint8)
        m = lib().ora_insert(self.keys, self.vals, n, k, v, B, ok, ov, st)
        self.keys, self.vals = ok[:m].copy(), ov[:m].copy()
        return st

    def delete(self, k):
        """Delete batch in batch order; per key 1 (DELETED) or 0 (ABSENT)."""
        k = _w(k)
        n, B = len(self.keys), len(k)
        ok = np.empty(max(n, 1), dtype=np.uint64)
        ov = np.empty(max(n, 1), dtype=np.uint64)
        st = np.empty(B, dtype=np.uint8)
        m = lib().ora_delete(self.keys, self.vals, n, k, B, ok, ov, st)
        self.keys, self.vals = ok[:m].copy(), ov[:m].copy()
        return st

    def range(self, lo, hi, maxc):
        """Returns (count[B], offsets[B], out_keys, out_vals) in CSR form."""
        lo, hi = _w(lo), _w(hi)
        mc = np.ascontiguousarray(np.asarray(maxc, dtype=np.uint32))
        off = _offsets(mc)
        tot = int(mc.astype(np.uint64).sum())
        ok = np.zeros(max(tot, 1), dtype=np.uint64)
        ov = np.zeros(max(tot, 1), dtype=np.uint64)
        cnt = np.empty(len(lo), dtype=np.uint32)
        lib().ora_range(self.keys, self.vals, len(self.keys), lo, hi, mc, off, len(lo), ok, ov, cnt)
        return cnt, off, _narrow(ok[:tot], self.width), _narrow(ov[:tot], self.width)

    def items(self):
        return _narrow(self.keys, self.width), _narrow(self.vals, self.width)


class PointerTree:
    """Textbook pointer B+-tree (order ``fanout``, leaf capacity ``cap``)."""

    def __init__(self, fanout: int = 16, cap: int = 16, width: int = 64):
        self.width = width
        self.h = lib().bpt_create(fanout, cap, width)
        if not self.h:
            raise ValueError("bad tree parameters")

    def __del__(self):
        if getattr(self, "h", None):
            lib().bpt_free(self.h)
            self.h = None

    def bulk_load(self, keys, vals, fill: float = 1.0):
        k, v = _w(keys), _w(vals)
        o = np.argsort(k, kind="stable")
        if lib().bpt_bulk_load(self.h, k[o], v[o], len(k), fill) != 0:
            raise ValueError("duplicate keys")

    def insert(self, k, v):
        k, v = _w(k), _w(v)
        st = np.empty(len(k), dtype=np.uint8)
        lib().bpt_insert_batch(self.h, k, v, len(k), st)
        return st

    def lookup(self, q, threads: int = 1):
        q = _w(q)
        vo = np.empty(len(q), dtype=np.uint64)
        fo = np.empty(len(q), dtype=np.uint8)
        lib().bpt_lookup_batch(self.h, q, len(q), vo, fo, threads)
        return _narrow(vo, self.width), fo

    def lookup_batches_timed(self, q, B: int, threads: int = 1):
        """len(q) // B batches of B queries, each split evenly over
        `threads` threads created once (a barrier before and after every
        batch).  Returns (values, found, seconds per batch)."""
        q = _w(q)
        nb = len(q) // B
        q = np.ascontiguousarray(q[:nb * B])
        vo = np.empty(max(1, nb * B), dtype=np.uint64)
        fo = np.empty(max(1, nb * B), dtype=np.uint8)
        tn = np.zeros(max(1, nb), dtype=np.uint64)
        if lib().bpt_lookup_batches_timed(self.h, q, nb, B, vo, fo, threads, tn) != 0:
            raise RuntimeError("could not start the lookup threads")
        return _narrow(vo[:nb * B], self.width), fo[:nb * B], tn[:nb].astype(np.float64) * 1e-9

    def lookup_levelwise(self, sorted_q):
        """Level-wise search of an ascending batch (Sections IV-A, IV-F).

        Returns (values, found, runs): results in processing order, and the
        FIFO entries as a dict of arrays level / first / count / node.
        """
        q = _w(sorted_q)
        B = len(q)
        vo = np.empty(max(B, 1), dtype=np.uint64)
        fo = np.empty(max(B, 1), dtype=np.uint8)
        cap = max(1, B * int(self.stats()["height"]))
        lv = np.empty(cap, dtype=np.uint32)
        fi, co, no = (np.empty(cap, dtype=np.uint64) for _ in range(3))
        w = lib().bpt_levelwise(self.h, q, B, vo, fo, lv, fi, co, no, cap)
        if w < 0:
            raise ValueError("batch not in ascending order")
        runs = {"level": lv[:w].copy(), "first": fi[:w].copy(), "count": co[:w].copy(), "node": no[:w].copy()}
        return _narrow(vo[:B], self.width), fo[:B], runs

    def range(self, lo, hi, maxc):
        lo, hi = _w(lo), _w(hi)
        mc = np.ascontiguousarray(np.asarray(maxc, dtype=np.uint32))
        off = _offsets(mc)
        tot = int(mc.astype(np.uint64).sum())
        ok = np.zeros(max(tot, 1), dtype=np.uint64)
        ov = np.zeros(max(tot, 1), dtype=np.uint64)
        cnt = np.empty(len(lo), dtype=np.uint32)
        lib().bpt_range_batch(self.h, lo, hi, mc, off, len(lo), ok, ov, cnt)
        return cnt, off, _narrow(ok[:tot], self.width), _narrow(ov[:tot], self.width)

    def stats(self):
        s = np.zeros(4, dtype=np.uint64)
        lib().bpt_stats(self.h, s)
        return {"height": int(s[0]), "n_keys": int(s[1]), "n_inner": int(s[2]), "n_leaves": int(s[3])}

    def export(self) -> np.ndarray:
        n = lib().bpt_export_bytes(self.h)
        buf = np.zeros(n, dtype=np.uint8)
        if lib().bpt_export(self.h, buf, n) != n:
            raise RuntimeError("export failed")
        return buf


def check_export(buf: np.ndarray, expect_n: int | None = None):
    """Check a flat tree export.  Returns (violation_bits, keys, vals) where
    keys/vals is the in-order sequence: keys as u64 for 4- and 8-byte keys,
    as an (n, 32) uint8 array for 32-byte keys; values as u64."""
    buf = np.ascontiguousarray(np.asarray(buf, dtype=np.uint8))
    if len(buf) >= 48:
        nk = int(np.frombuffer(buf[40:48].tobytes(), dtype=np.uint64)[0])
        kb = int(np.frombuffer(buf[4:8].tobytes(), dtype=np.uint32)[0])
    else:
        nk, kb = 0, 8
    cap = max(nk, expect_n or 0) + 1
    if kb > 8:
        okb = np.zeros(cap * kb, dtype=np.uint8)
        ov = np.zeros(cap, dtype=np.uint64)
        nout = C.c_uint64(0)
        v = lib().orb_check_export(buf, len(buf), okb, ov, cap, C.byref(nout))
        m = min(int(nout.value), cap)
        return int(v), okb.reshape(cap, kb)[:m], ov[:m]
    ok = np.zeros(cap, dtype=np.uint64)
    ov = np.zeros(cap, dtype=np.uint64)
    nout = C.c_uint64(0)
    v = lib().ora_check_export(buf, len(buf), ok, ov, cap, C.byref(nout))
    m = min(int(nout.value), cap)
    return int(v), ok[:m], ov[:m]


def violations(bits: int) -> list[str]:
    return [name for b, name in V_NAMES.items() if bits & b]


def iqm(x) -> float:
    """Interquartile mean: the arithmetic mean of the central half of the
    sorted sample (Section V-C defines it in words; its printed 1/n factor
    would halve that mean, so the mean over n/2 values is taken).  Requires
    n divisible by 4."""
    s = np.sort(np.asarray(x, dtype=np.float64))
    n = len(s)
    if n == 0 or n % 4:
        raise ValueError("IQM needs a sample size divisible by 4")
    return float(s[n // 4: 3 * n // 4].mean())


def iqr(x) -> float:
    """Interquartile range (upper minus lower quartile, numpy's default
    linear interpolation)."""
    q1, q3 = np.percentile(np.asarray(x, dtype=np.float64), [25, 75])
    return float(q3 - q1)
