"""Pins for the oracle's 32-byte keys (Section IV-C's search keys, compared
bytewise with the most significant byte deciding, Section IV-E) and for the
tree orders m = 16, 32, 64 (Section V-C), CPU only.

* The sorted-array reference over byte keys against a pure-Python brute
  force whose order is Python's own bytes comparison.
* Closed forms: a 32-byte big-endian encoding of an integer orders like the
  integer; keys that differ only in byte j order by that byte.
* The invariant checker on hand-written 32-byte exports (valid trees of
  orders 16, 32 and 64 accepted with their in-order content; planted
  mistakes flagged), and on the textbook pointer tree of orders 32 and 64
  with 8-byte keys, whose bulk load at fill 1 has Section III's N_max nodes.
"""
import numpy as np
import pytest

import oracle
from oracle.brute import BruteBytes

KB = 32


def _keys_with_prefixes(rng, n):
    """n distinct 32-byte keys drawn from {0, 1, 0x7f, 0x80, 0xff} on a few
    positions spread over the key and a shared background, so that most
    comparisons run deep into the key and cross the sign of a byte."""
    alphabet = np.array([0, 1, 0x7F, 0x80, 0xFF], dtype=np.uint8)
    pos = np.array([0, 7, 8, 15, 16, 24, 31])
    out = set()
    base = np.full(KB, 0x55, dtype=np.uint8)
    while len(out) < n:
        k = base.copy()
        k[pos] = alphabet[rng.integers(0, len(alphabet), len(pos))]
        out.add(k.tobytes())
    return np.frombuffer(b"".join(sorted(out, key=lambda b: rng.random())), dtype=np.uint8).reshape(n, KB).copy()


@pytest.mark.parametrize("seed", range(10))
def test_sorted_bytes_vs_brute(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 120))
    keys = _keys_with_prefixes(rng, n) if n else np.zeros((0, KB), np.uint8)
    if n >= 2:
        keys[0] = 0          # the smallest and the largest key value
        keys[1] = 0xFF
        keys = np.unique(keys, axis=0)[rng.permutation(len(np.unique(keys, axis=0)))]
    vals = rng.integers(0, 1 << 63, len(keys), dtype=np.uint64) * 2 + 1
    sb = oracle.SortedBytes(keys, vals)
    br = BruteBytes(keys, vals)
    q = np.concatenate([keys[rng.integers(0, max(1, len(keys)), 40)] if len(keys) else np.zeros((0, KB), np.uint8),
                        _keys_with_prefixes(rng, 40), np.zeros((1, KB), np.uint8),
                        np.full((1, KB), 0xFF, np.uint8)])
    v, f = sb.lookup(q)
    bv, bf = br.lookup(q)
    assert list(f) == bf and [int(x) for x in v] == bv
    lo = q[:30]
    hi = np.concatenate([q[30:55], q[:5]])
    mc = rng.integers(0, 9, 30).astype(np.uint32)
    cnt, off, ok, ov = sb.range(lo, hi, mc)
    want = br.range(lo, hi, mc)
    for i, w in enumerate(want):
        got = [(ok[off[i] + j].tobytes(), int(ov[off[i] + j])) for j in range(int(cnt[i]))]
        assert got == w, i
    assert [bytes(k) for k in sb.keys] == [p[0] for p in br.items()]


def test_byte_order_closed_forms():
    """Big-endian encodings order like the integers they encode; a key
    difference in byte j is decided by byte j alone, whatever follows."""
    rng = np.random.default_rng(3)
    xs = sorted({int(rng.integers(0, 1 << 62)) << int(rng.integers(0, 190)) for _ in range(300)})
    enc = np.frombuffer(b"".join(x.to_bytes(KB, "big") for x in xs), dtype=np.uint8).reshape(-1, KB)
    perm = rng.permutation(len(xs))
    sb = oracle.SortedBytes(enc[perm], np.arange(len(xs), dtype=np.uint64)[perm])
    assert np.array_equal(sb.keys, enc)
    assert np.array_equal(sb.vals, np.arange(len(xs), dtype=np.uint64))
    for j in range(KB):
        a = np.full(KB, 0x80, dtype=np.uint8)
        b = a.copy()
        b[j] = 0x81
        a[j + 1:] = 0xFF       # larger tail on the smaller key
        b[j + 1:] = 0x00
        s2 = oracle.SortedBytes(np.stack([b, a]), np.array([2, 1], dtype=np.uint64))
        assert s2.keys[0].tobytes() == a.tobytes() and list(s2.vals) == [1, 2]


def test_sorted_bytes_rejects_duplicates():
    k = np.zeros((3, KB), dtype=np.uint8)
    k[1, 5] = 1
    with pytest.raises(ValueError):
        oracle.SortedBytes(k, np.arange(3, dtype=np.uint64))


def test_sorted_bytes_empty():
    sb = oracle.SortedBytes(None, [])
    v, f = sb.lookup(np.zeros((2, KB), np.uint8))
    assert list(f) == [0, 0] and (v == np.uint64((1 << 64) - 1)).all()


# ---------------------------------------------------------------- exports

def _key32(i: int) -> bytes:
    """The i-th key of a hand-written tree: a shared 24-byte prefix, then
    10 * (i + 1) big-endian, so separators are decided in the last bytes."""
    return bytes([0xA5] * 24) + (10 * (i + 1)).to_bytes(8, "big")


def hand_export(shape, F, C, kb=KB):
    """A flat export written by hand from a nested shape (a list is an inner
    node, an int a leaf with that many keys), in the library's format:
    header with the value width in its last u32 (8 for 32-byte keys), inner
    records key[F] + child[F], leaf records key[C] + value[C] + count +
    next, unused entries padded with the largest key, leaf slots past the
    count repeating the last key, the chain linking plain leaf indices."""
    maxk = b"\xff" * kb
    inner, leaves = [], []
    nxt = [0]

    def depth(s):
        return 1 if isinstance(s, int) else 1 + depth(s[0])

    def make(s):
        if isinstance(s, int):
            ks = [_key32(nxt[0] + i) for i in range(s)]
            nxt[0] += s
            leaves.append(ks)
            return (len(leaves) - 1) | 0x80000000, ks[-1]
        me = len(inner)
        inner.append(None)
        refs, tops = zip(*[make(c) for c in s])
        inner[me] = (list(refs), list(tops))
        return me, tops[-1]

    root, _ = make(shape)
    out = bytearray()
    nk = sum(len(k) for k in leaves)
    out += np.array([0x58455447, kb, F, C, depth(shape), root, 0, len(inner), len(leaves), 8],
                    dtype=np.uint32).tobytes()
    out += np.array([nk], dtype=np.uint64).tobytes()
    for refs, tops in inner:
        seps = tops[:-1] + [maxk] * (F - len(tops) + 1)
        out += b"".join(seps)
        out += np.array(refs + [0xFFFFFFFF] * (F - len(refs)), dtype=np.uint32).tobytes()
    for j, ks in enumerate(leaves):
        out += b"".join(ks + [ks[-1]] * (C - len(ks)))
        out += np.array([int.from_bytes(k[-8:], "big") + 1 for k in ks] + [0] * (C - len(ks)),
                        dtype=np.uint64).tobytes()
        out += np.array([len(ks), j + 1 if j + 1 < len(leaves) else 0xFFFFFFFF], dtype=np.uint32).tobytes()
    return np.frombuffer(bytes(out), dtype=np.uint8).copy()


def _leaf_at(buf, leaf):
    h = np.frombuffer(buf[:40].tobytes(), dtype=np.uint32)
    kb, F, Cc, ni = int(h[1]), int(h[2]), int(h[3]), int(h[7])
    return 48 + ni * F * (kb + 4) + leaf * (Cc * (kb + 8) + 8), Cc


@pytest.mark.parametrize("m", [16, 32, 64])
def test_checker_accepts_valid_32byte_trees(m):
    half = m // 2
    shape = [[m - 1] * m, [half] * half]      # a full parent and a half-full one
    buf = hand_export(shape, m, m - 1)
    bits, ek, ev = oracle.check_export(buf)
    assert bits == 0, oracle.violations(bits)
    n = (m - 1) * m + half * half
    assert ek.shape == (n, KB)
    assert [bytes(k) for k in ek] == [_key32(i) for i in range(n)]
    assert list(ev) == [10 * (i + 1) + 1 for i in range(n)]


@pytest.mark.parametrize("m", [16, 32, 64])
def test_checker_flags_32byte_mistakes(m):
    half = m // 2
    good = [[half] * half, [half] * half]
    # Section III's m/2 rule for a non-root inner node, at each order
    assert oracle.check_export(hand_export([[half] * half, [half] * (half - 1)], m, m - 1))[0] == oracle.V_FILL
    # a leaf below half full (leaf capacity m - 1: at least m/2 keys)
    assert oracle.check_export(hand_export([[half] * half, [half] * (half - 1) + [half - 1]], m, m - 1))[0] \
        & oracle.V_FILL
    # two keys of a leaf swapped: the order check must look past the shared
    # 24-byte prefix
    b = hand_export(good, m, m - 1)
    o, _ = _leaf_at(b, 3)
    k0 = b[o:o + KB].copy()
    b[o:o + KB] = b[o + KB:o + 2 * KB]
    b[o + KB:o + 2 * KB] = k0
    assert oracle.check_export(b)[0] & oracle.V_SORTED
    # a separator one below the largest key of its child: that key now lies
    # outside its interval
    b = hand_export(good, m, m - 1)
    sep = 48 + 1 * m * (KB + 4)               # inner node 1 = first parent, entry 0
    b[sep + KB - 1] -= 1
    assert oracle.check_export(b)[0] & oracle.V_SEPARATOR
    # a padded leaf slot that does not repeat the last key
    b = hand_export(good, m, m - 1)
    o, Cc = _leaf_at(b, 0)
    b[o + (Cc - 1) * KB] ^= 0x01
    assert oracle.check_export(b)[0] & oracle.V_PADDING


def test_checker_rejects_bad_value_width():
    b = hand_export([8, 8], 16, 15)
    b[36:40] = np.frombuffer(np.uint32(32).tobytes(), dtype=np.uint8)
    assert oracle.check_export(b)[0] == oracle.V_FORMAT


@pytest.mark.parametrize("m,h", [(32, 2), (32, 3), (64, 2), (64, 3)])
def test_pointer_tree_orders_32_64_nmax(m, h):
    """Section III: a tree of order m and height h holds at most
    (m - 1) * m^(h-1) keys (leaves of m - 1 keys) in sum_{i<h} m^i nodes;
    the bulk load at fill 1 reaches both, and its export passes the
    checker with its content."""
    n = (m - 1) * m ** (h - 1)
    keys = np.arange(n, dtype=np.uint64) * 3 + 1
    pt = oracle.PointerTree(m, m - 1, 64)
    pt.bulk_load(keys, keys ^ np.uint64(5))
    st = pt.stats()
    assert st["height"] == h and st["n_inner"] + st["n_leaves"] == sum(m ** i for i in range(h))
    bits, ek, ev = oracle.check_export(pt.export())
    assert bits == 0, oracle.violations(bits)
    assert np.array_equal(ek, keys) and np.array_equal(ev, keys ^ np.uint64(5))
