"""GPU parity of the static tree of the paper's key and node variants --
32-byte keys compared byte by byte (Sections IV-C, IV-E) at orders 16, 32
and 64, and 8-byte keys at orders 32 and 64 (Section V-C) -- against the
oracle, bit for bit, through the C ABI: the built tree's export passes the
invariant checker and holds exactly the input; lookups (present, absent,
keys sharing long prefixes, the smallest and largest key values) and range
scans equal the oracle's; Section III's N_max node counts at fill 1; the
calls a static tree refuses."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

COMBOS = [(32, 16), (32, 32), (32, 64), (8, 32), (8, 64)]


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_21117_amd as g
    g.lib()


def keys32(n, seed, prefix_share=0.5):
    """n distinct 32-byte keys: a share of them agree on a random number of
    leading bytes with a common stem (deep comparisons), the rest uniform;
    the smallest and the largest key values are among them when n >= 2."""
    s = synth.Stream(seed, 77)
    m = n + n // 8 + 16
    k = s.draw(m * 4).view(np.uint8).reshape(m, 32).copy()
    stem = k[-1].copy()
    share = s.below(m, 32)
    deep = s.uniform01(m) < prefix_share
    take = deep[:, None] & (np.arange(32)[None, :] < share[:, None])
    k = np.where(take, stem[None, :], k)
    k[0], k[1] = 0, 0xFF
    k = np.unique(np.ascontiguousarray(k).view(np.dtype((np.void, 32))).ravel()).view(np.uint8).reshape(-1, 32)
    order = np.argsort(synth.Stream(seed, 76).draw(len(k)), kind="stable")
    k = k[order]
    edge = (k == 0).all(axis=1) | (k == 0xFF).all(axis=1)
    k = np.concatenate([k[edge], k[~edge]]) if n >= 2 else k[~edge]
    assert len(k) >= n
    return np.ascontiguousarray(k[:n])


def build(kb, m, n, seed, fill=1.0):
    import paper_2604_21117_amd as g
    if kb == 32:
        k = keys32(n, seed)
        assert len(k) == n
    else:
        k = synth.uniform_keys(n, seed, 64)
        if n >= 2:
            k[0], k[1] = 0, np.uint64((1 << 64) - 1)
    v = synth.values_for(k.view(np.uint64).reshape(len(k), -1)[:, 0] if kb == 32 else k, seed, 64) \
        if n else np.zeros(0, np.uint64)
    t = g.StaticTree(k, v, kb, m, fill=fill)
    ref = oracle.SortedBytes(k, v) if kb == 32 else oracle.SortedArray(k, v, 64)
    return t, ref, k


def queries(kb, keys, B, seed):
    """Half present keys, half absent; for 32-byte keys the absent half are
    present keys with one byte changed (they share all other bytes with a
    neighbour in key order), and both edge values appear."""
    s = synth.Stream(seed, 78)
    n = len(keys)
    if kb == 8:
        q = synth.mixed_queries(keys, B, seed, 64) if n else synth.absent_queries(keys, B, seed, 64)
        q[: min(B, 2)] = np.array([0, (1 << 64) - 1], dtype=np.uint64)[: min(B, 2)]
        return q
    if n == 0:
        return keys32(B, seed + 5)
    q = keys[s.below(B, n).astype(np.int64)].copy()
    half = s.uniform01(B) < 0.5
    pos = s.below(B, 32).astype(np.int64)
    delta = (s.below(B, 255) + 1).astype(np.uint8)
    rows = np.nonzero(half)[0]
    q[rows, pos[rows]] = q[rows, pos[rows]] + delta[rows]
    q[0] = 0
    if B > 1:
        q[1] = 0xFF
    return q


def check_lookup(t, ref, q):
    gv, gf = t.lookup(q)
    ov, of = ref.lookup(q)
    assert np.array_equal(gf, of), f"found flags differ at {np.nonzero(gf != of)[0][:8]}"
    assert np.array_equal(gv, ov), f"values differ at {np.nonzero(gv != ov)[0][:8]}"


def check_export(t, ref, kb):
    bits, ek, ev = oracle.check_export(t.export())
    assert bits == 0, oracle.violations(bits)
    assert np.array_equal(ek, ref.keys) and np.array_equal(ev, ref.vals)


def check_range(t, ref, kb, keys, seed, B=300):
    s = synth.Stream(seed, 79)
    lo = queries(kb, keys, B, seed + 3)
    hi = queries(kb, keys, B, seed + 4)
    mc = (s.below(B, 140)).astype(np.uint32)
    gc, goff, gk, gv = t.range(lo, hi, mc)
    oc, ooff, ok, ov = ref.range(lo, hi, mc)
    assert np.array_equal(gc, oc), f"range counts differ at {np.nonzero(gc != oc)[0][:8]}"
    for i in np.nonzero(oc)[0]:
        sl = slice(int(ooff[i]), int(ooff[i] + oc[i]))
        assert np.array_equal(gk[sl], ok[sl]) and np.array_equal(gv[sl], ov[sl]), f"range {i} differs"


@pytest.mark.parametrize("kb,m", COMBOS)
@pytest.mark.parametrize("n", [0, 1, 2, 14, 15, 16, 63, 64, 1000, 5000, 70000])
def test_static_build_lookup_range(kb, m, n):
    seed = 31 * n + m + kb
    t, ref, k = build(kb, m, n, seed)
    check_export(t, ref, kb)
    for B in (1, 7, 64, 1000, 4099, 9000):
        check_lookup(t, ref, queries(kb, k, B, seed + B))
    check_range(t, ref, kb, k, seed)
    st = t.stats()
    assert st["n_keys"] == n and st["key_bytes"] == kb
    t.close()


def _unique_rows(k):
    u = np.unique(np.ascontiguousarray(k).view(np.dtype((np.void, 32))).ravel())
    return u.view(np.uint8).reshape(-1, 32)


@pytest.mark.parametrize("m", [16, 32, 64])
def test_static_leading_word_ties(m):
    """Keys whose first 8 bytes come from a small pool, so that separators
    tie queries on their leading word both where the next key in order
    shares it and where it does not; queries are present keys, present keys
    with the last byte moved up or down (absent, same leading word), and
    every pool word with all-zero and all-one tails.  Lookups and range
    lower bounds against the oracle."""
    s = synth.Stream(901 + m, 1)
    n = 40000
    pool = s.draw(5000).view(np.uint8).reshape(5000, 8)
    k = s.draw(n * 4).view(np.uint8).reshape(n, 32).copy()
    k[:, :8] = pool[s.below(n, 5000).astype(np.int64)]
    k = _unique_rows(k)
    k = k[np.argsort(s.draw(len(k)), kind="stable")]
    v = synth.values_for(k.view(np.uint64).reshape(len(k), -1)[:, 0], 7, 64)
    import paper_2604_21117_amd as g
    t = g.StaticTree(k, v, 32, m)
    ref = oracle.SortedBytes(k, v)
    sk = ref.keys
    up, down = sk.copy(), sk.copy()
    up[:, 31] += 1
    down[:, 31] -= 1
    lo0, hi1 = np.zeros((5000, 32), np.uint8), np.full((5000, 32), 0xFF, np.uint8)
    lo0[:, :8] = pool
    hi1[:, :8] = pool
    q = np.concatenate([sk, up, down, lo0, hi1])
    q = q[np.argsort(s.draw(len(q)), kind="stable")]
    check_lookup(t, ref, q)
    B = 4000
    lo = q[:B]
    hi = q[B:2 * B]
    mc = s.below(B, 40).astype(np.uint32)
    gc, goff, gk, gv = t.range(lo, hi, mc)
    oc, ooff, ok, ov = ref.range(lo, hi, mc)
    assert np.array_equal(gc, oc), f"range counts differ at {np.nonzero(gc != oc)[0][:8]}"
    for i in np.nonzero(oc)[0]:
        sl = slice(int(ooff[i]), int(ooff[i] + oc[i]))
        assert np.array_equal(gk[sl], ok[sl]) and np.array_equal(gv[sl], ov[sl]), f"range {i} differs"
    t.close()


@pytest.mark.parametrize("kb,m", COMBOS)
@pytest.mark.parametrize("fill", [0.5, 0.75])
def test_static_partial_fill(kb, m, fill):
    seed = 5 + m
    t, ref, k = build(kb, m, 20000, seed, fill=fill)
    check_export(t, ref, kb)
    check_lookup(t, ref, queries(kb, k, 3000, seed))
    check_range(t, ref, kb, k, seed)


@pytest.mark.parametrize("kb,m,h", [(32, 16, 2), (32, 16, 3), (32, 16, 4), (32, 32, 3), (32, 64, 2), (32, 64, 3),
                                    (8, 32, 3), (8, 64, 3)])
def test_static_nmax_closed_form(kb, m, h):
    """Section III: at fill 1 a tree of (m - 1) m^(h-1) keys has height h
    and sum_{i<h} m^i nodes (every node full)."""
    n = (m - 1) * m ** (h - 1)
    t, ref, k = build(kb, m, n, 1000 + h)
    st = t.stats()
    assert st["height"] == h
    assert st["inner_used"] + st["leaf_used"] == sum(m ** i for i in range(h))
    assert st["leaf_used"] == m ** (h - 1)
    check_export(t, ref, kb)
    check_lookup(t, ref, queries(kb, k, 2000, 9))


@pytest.mark.parametrize("m", [16, 32, 64])
def test_static_paper_scale(m):
    """One million 32-byte entries (the paper's tree sizes reach 1M and 10M),
    a batch of 1000 (the paper's largest) and one of 2^20, every result
    against the oracle."""
    seed = 4000 + m
    t, ref, k = build(32, m, 1 << 20, seed)
    check_lookup(t, ref, queries(32, k, 1000, seed))
    check_lookup(t, ref, queries(32, k, 1 << 20, seed + 1))
    check_range(t, ref, 32, k, seed, B=2000)


def test_static_duplicate_keys_refused():
    import torch
    import paper_2604_21117_amd as g
    k = keys32(300, 3)
    k[200] = k[17]
    with pytest.raises(g.GtError) as e:
        g.StaticTree(k, np.arange(300, dtype=np.uint64), 32, 16)
    assert e.value.status == g.GT_ERR_DUPLICATE
    k8 = synth.uniform_keys(5000, 4, 64)
    k8[4999] = k8[3]
    with pytest.raises(g.GtError) as e:
        g.StaticTree(k8, k8, 8, 32)
    assert e.value.status == g.GT_ERR_DUPLICATE
    torch.cuda.synchronize()


def test_static_refusals():
    """A static tree takes no inserts, deletes, level-wise lookups, learned
    index or server; unsupported parameter sets size to 0."""
    import torch
    import paper_2604_21117_amd as g
    t, ref, k = build(32, 32, 3000, 8)
    L = g.lib()
    d = torch.zeros(64 * 32, dtype=torch.uint8, device="cuda")
    assert L.tree_insert_batch(t.h, g._ptr(d), g._ptr(d), 4, g._ptr(d), None) == g.GT_ERR_INVALID
    assert L.tree_delete_batch(t.h, g._ptr(d), 4, g._ptr(d), None) == g.GT_ERR_INVALID
    assert L.tree_lookup_levelwise(t.h, g._ptr(d), 4, 0, g._ptr(d), g._ptr(d), g._ptr(d), d.numel(), None) \
        == g.GT_ERR_INVALID
    assert L.tree_lookup_levelwise_noalloc(t.h, g._ptr(d), 4, 0, g._ptr(d), g._ptr(d), None) == g.GT_ERR_INVALID
    assert L.tree_lookup_levelwise_workspace_bytes(t.h, 4, 0) == 0
    assert L.li_arena_bytes(t.h, None) == 0
    h = C.c_void_p()
    assert L.srv_create(t.h, None, None, C.byref(h)) == g.GT_ERR_INVALID
    for kb, m in ((32, 128), (32, 8), (4, 32), (8, 16 + 1), (16, 16)):
        assert g.tree_arena_bytes(g.make_static_params(kb, m), 1000) == 0, (kb, m)
    # the tree still answers after the refusals
    check_lookup(t, ref, queries(32, k, 500, 8))
