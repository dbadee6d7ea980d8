"""Pins for the CPU oracle: brute force on tiny inputs, closed forms from
Section III, planted mistakes for the invariant checker, and random
operation sequences.  CPU only."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
import synth
from oracle.brute import Brute

MAX64 = (1 << 64) - 1
MAX32 = (1 << 32) - 1


def _small_keys(rng, n, width, lo=0, hi=None):
    hi = (1 << width) - 1 if hi is None else hi
    ks = set()
    while len(ks) < n:
        ks.add(int(rng.integers(lo, hi, endpoint=True, dtype=np.uint64)))
    return list(ks)


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("seed", range(12))
def test_lookup_insert_range_vs_brute(width, seed):
    rng = np.random.default_rng(seed)
    top = (1 << width) - 1
    # narrow key space so that batches hit present keys and duplicates often;
    # always include the edge keys 0 and max in play
    n = int(rng.integers(0, 64))
    keys = _small_keys(rng, n, width, 0, 200)
    if seed % 3 == 0:
        keys = list(set(keys) | {0, top})
    vals = [int(x) for x in rng.integers(0, top, len(keys), endpoint=True, dtype=np.uint64)]
    br = Brute(keys, vals, width)
    sa = oracle.SortedArray(keys, vals, width)
    pt = oracle.PointerTree(16, 16, width)
    pt.bulk_load(keys, vals)
    for step in range(4):
        B = int(rng.integers(0, 64))
        q = [int(x) for x in rng.integers(0, 210, B)] + [0, top, top - 1]
        bv, bf = br.lookup(q)
        sv, sf = sa.lookup(q)
        pv, pf = pt.lookup(q)
        assert list(sf) == bf and list(pf) == bf
        assert [int(x) for x in sv] == bv and [int(x) for x in pv] == bv
        # insert batch with in-batch duplicates and updates of present keys
        kb = [int(x) for x in rng.integers(0, 210, B)]
        if step == 1:
            kb += [top, 0, top]
        vb = [int(x) for x in rng.integers(0, top, len(kb), endpoint=True, dtype=np.uint64)]
        stb = br.insert(kb, vb)
        sts = sa.insert(kb, vb)
        stp = pt.insert(kb, vb)
        assert list(sts) == stb and list(stp) == stb
        bk, bvv = br.items()
        sk, sv2 = sa.items()
        assert [int(x) for x in sk] == bk and [int(x) for x in sv2] == bvv
        bits, ek, ev = oracle.check_export(pt.export())
        assert bits == 0, oracle.violations(bits)
        assert [int(x) for x in ek] == bk and [int(x) for x in ev] == bvv
        # ranges, including empty intervals and max = 0
        R = 16
        lo = [int(x) for x in rng.integers(0, 220, R)] + [0, top, 50]
        hi = [min(top, a + int(d)) for a, d in zip(lo, rng.integers(0, 60, len(lo)))]
        hi[-1] = 10  # lo > hi
        mc = [int(x) for x in rng.integers(0, 12, len(lo))] + []
        mc[0] = 0
        want = br.range(lo, hi, mc)
        for impl in (sa, pt):
            cnt, off, ok, ov = impl.range(lo, hi, mc)
            for i, w in enumerate(want):
                got = [(int(ok[off[i] + j]), int(ov[off[i] + j])) for j in range(int(cnt[i]))]
                assert got == w


def test_empty_and_single():
    for width in (32, 64):
        top = (1 << width) - 1
        sa = oracle.SortedArray([], [], width)
        pt = oracle.PointerTree(16, 16, width)
        pt.bulk_load([], [])
        v, f = sa.lookup([0, 5, top])
        assert list(f) == [0, 0, 0] and all(int(x) == top for x in v)
        v, f = pt.lookup([0, 5, top])
        assert list(f) == [0, 0, 0] and all(int(x) == top for x in v)
        bits, ek, _ = oracle.check_export(pt.export())
        assert bits == 0 and len(ek) == 0
        pt.insert([7], [9])
        sa.insert([7], [9])
        assert pt.stats()["height"] == 1
        v, f = pt.lookup([7, 8])
        assert list(f) == [1, 0] and int(v[0]) == 9


def test_lookup_closed_form_from_generator():
    """A key drawn as present returns hash(key ^ seed) with found = 1; a key
    drawn as absent returns all ones with found = 0 (Section IV-D)."""
    for width, seed in ((32, 1), (64, 2)):
        keys = synth.uniform_keys(5000, seed, width)
        vals = synth.values_for(keys, seed, width)
        sa = oracle.SortedArray(keys, vals, width)
        pt = oracle.PointerTree(16, 16, width)
        pt.bulk_load(keys, vals)
        pres = synth.present_queries(keys, 3000, seed)
        absn = synth.absent_queries(keys, 3000, seed, width)
        for impl in (sa, pt):
            v, f = impl.lookup(pres)
            assert f.all() and np.array_equal(v, synth.values_for(pres, seed, width))
            v, f = impl.lookup(absn)
            assert not f.any() and np.all(v == np.iinfo(v.dtype).max)


def _nmax(m, h):
    # Section III: a full tree of height h has sum_{i<h} m^i nodes
    return sum(m ** i for i in range(h))


@pytest.mark.parametrize("logn,h", [(4, 1), (8, 2), (12, 3), (16, 4), (20, 5)])
def test_bulk_load_node_counts_closed_form(logn, h):
    n = 1 << logn
    keys = np.arange(n, dtype=np.uint64) * 3 + 1
    pt = oracle.PointerTree(16, 16, 64)
    pt.bulk_load(keys, keys)
    s = pt.stats()
    assert s["height"] == h
    assert s["n_inner"] + s["n_leaves"] == _nmax(16, h)
    assert s["n_leaves"] == 16 ** (h - 1)


@pytest.mark.slow
def test_bulk_load_node_counts_2_24():
    n = 1 << 24
    keys = np.arange(n, dtype=np.uint64) * 2
    pt = oracle.PointerTree(16, 16, 64)
    pt.bulk_load(keys, keys)
    s = pt.stats()
    assert s["height"] == 6 and s["n_inner"] + s["n_leaves"] == 1118481


def test_bulk_load_fill_keeps_half_full():
    for n in [17, 31, 33, 100, 257, 1000, 4097]:
        for fill in (0.51, 0.7, 1.0):
            keys = np.arange(n, dtype=np.uint64)
            pt = oracle.PointerTree(16, 16, 64)
            pt.bulk_load(keys, keys, fill)
            bits, ek, _ = oracle.check_export(pt.export())
            assert bits == 0, (n, fill, oracle.violations(bits))
            assert len(ek) == n


def test_insert_status_formula():
    """First occurrence INSERTED iff absent before the batch, later ones
    UPDATED; the last occurrence's value wins."""
    sa = oracle.SortedArray([10, 20], [1, 2], 64)
    st_ = sa.insert([30, 10, 30, 40, 30], [5, 6, 7, 8, 9])
    assert list(st_) == [0, 1, 1, 0, 1]
    k, v = sa.items()
    assert list(k) == [10, 20, 30, 40] and list(v) == [6, 2, 9, 8]


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("seed", range(10))
def test_delete_vs_brute(width, seed):
    """Delete batches (present keys, absent keys, keys repeated in the batch,
    the edge keys) interleaved with inserts, against the one-at-a-time brute
    force: statuses, the remaining pairs and lookups after each batch."""
    rng = np.random.default_rng(500 + seed)
    top = (1 << width) - 1
    keys = _small_keys(rng, int(rng.integers(0, 80)), width, 0, 150)
    if seed % 2 == 0:
        keys = list(set(keys) | {0, top})
    vals = [int(x) for x in rng.integers(0, top, len(keys), endpoint=True, dtype=np.uint64)]
    br = Brute(keys, vals, width)
    sa = oracle.SortedArray(keys, vals, width)
    for step in range(6):
        B = int(rng.integers(0, 70))
        kb = [int(x) for x in rng.integers(0, 160, B)]
        if step % 3 == 1:
            kb += [top, 0, top, 0]
        stb = br.delete(kb)
        sts = sa.delete(kb)
        assert list(sts) == stb
        bk, bv = br.items()
        sk, sv = sa.items()
        assert [int(x) for x in sk] == bk and [int(x) for x in sv] == bv
        q = [int(x) for x in rng.integers(0, 170, 40)] + [0, top]
        gv, gf = sa.lookup(q)
        ev, ef = br.lookup(q)
        assert list(gf) == ef and [int(x) for x in gv] == ev
        ki = [int(x) for x in rng.integers(0, 160, int(rng.integers(0, 30)))]
        vi = [int(x) for x in rng.integers(0, top, len(ki), endpoint=True, dtype=np.uint64)]
        assert list(sa.insert(ki, vi)) == br.insert(ki, vi)


def test_delete_closed_forms():
    """Deleting every key empties the set with all statuses 1; deleting
    absent keys changes nothing; a repeated key reports 1 only at its first
    occurrence; deleting then re-inserting restores the set."""
    keys = np.arange(5, 5005, 5, dtype=np.uint64)
    vals = keys * 7
    sa = oracle.SortedArray(keys, vals, 64)
    st_ = sa.delete(keys + 1)
    assert not st_.any() and len(sa) == 1000
    st_ = sa.delete(np.array([10, 11, 10, 10, 4995, 5000, 5000], dtype=np.uint64))
    assert list(st_) == [1, 0, 0, 0, 1, 1, 0]
    k, v = sa.items()
    assert len(k) == 997 and 10 not in set(k.tolist()) and np.array_equal(v, k * 7)
    st_ = sa.insert(np.array([10, 4995, 5000], dtype=np.uint64), np.array([70, 4995 * 7, 35000], dtype=np.uint64))
    assert list(st_) == [0, 0, 0]
    k, v = sa.items()
    assert np.array_equal(k, keys) and np.array_equal(v, vals)
    st_ = sa.delete(synth.shuffle(keys, 3))
    assert st_.all() and len(sa) == 0
    assert not sa.delete(keys[:10]).any()


def test_range_closed_form():
    keys = np.arange(0, 3000, 3, dtype=np.uint64)
    sa = oracle.SortedArray(keys, keys + 1, 64)
    lo = np.array([0, 1, 2998, 100, 5000], dtype=np.uint64)
    hi = np.array([30, 1, 3005, 2000, 6000], dtype=np.uint64)
    mc = np.array([100, 5, 5, 7, 3], dtype=np.uint32)
    cnt, off, ok, ov = sa.range(lo, hi, mc)
    # multiples of 3 in [lo, min(hi, 2997)], capped by max
    want = [min(m, len(range(((a + 2) // 3) * 3, min(b, 2997) + 1, 3))) for a, b, m in zip(lo.tolist(), hi.tolist(), mc.tolist())]
    assert cnt.tolist() == want
    assert ok[off[3]: off[3] + cnt[3]].tolist() == list(range(102, 102 + 3 * 7, 3))
    for i in range(len(lo)):
        seg = slice(int(off[i]), int(off[i] + cnt[i]))
        assert np.array_equal(ov[seg], ok[seg] + 1)


def test_iqm_iqr():
    assert oracle.iqm(range(1, 9)) == 4.5           # mean(3, 4, 5, 6)
    assert oracle.iqm([9, 1, 1, 9, 5, 5, 5, 5]) == 5.0
    with pytest.raises(ValueError):
        oracle.iqm([1, 2, 3])
    assert oracle.iqr([1, 2, 3, 4, 5]) == 2.0


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_timed_batches_match_plain_lookup(threads):
    """The timed CPU-baseline path (threads created once, a barrier per
    batch) answers exactly as the plain definition, present and absent keys
    alike, and reports one positive time per batch."""
    keys = np.array(synth.uniform_keys(5000, 11, 64), dtype=np.uint64)
    vals = synth.values_for(keys, 11, 64)
    pt = oracle.PointerTree(16, 16, 64)
    pt.bulk_load(keys, vals)
    q = synth.mixed_queries(keys, 7 * 100, 12, 64)
    v, f, t = pt.lookup_batches_timed(q, 100, threads)
    sa = oracle.SortedArray(keys, vals, 64)
    ev, ef = sa.lookup(q)
    assert np.array_equal(f, ef) and np.array_equal(v, ev)
    assert len(t) == 7 and (t > 0).all()


# ---------------------------------------------------------- planted mistakes

def _tree_export(n=3000, width=64):
    keys = np.arange(n, dtype=np.uint64) * 7 + 3
    pt = oracle.PointerTree(16, 16, width)
    pt.bulk_load(keys, keys * 2)
    return pt, pt.export()


def _hdr(buf):
    return np.frombuffer(buf[:40].tobytes(), dtype=np.uint32).copy()


def _leaf_off(buf, leaf):
    h = _hdr(buf)
    kb, F, Cc, ni = int(h[1]), int(h[2]), int(h[3]), int(h[7])
    return 48 + ni * F * (kb + 4) + leaf * (Cc * 2 * kb + 8), kb, Cc


def _inner_off(buf, node):
    h = _hdr(buf)
    kb, F = int(h[1]), int(h[2])
    return 48 + node * F * (kb + 4), kb, F


def test_checker_accepts_valid():
    for width in (32, 64):
        _, b = _tree_export(5000, width)
        bits, ek, _ = oracle.check_export(b)
        assert bits == 0 and len(ek) == 5000


def test_checker_flags_unsorted_leaf():
    _, b = _tree_export()
    o, kb, _ = _leaf_off(b, 5)
    k0 = b[o:o + kb].copy()
    b[o:o + kb] = b[o + kb:o + 2 * kb]
    b[o + kb:o + 2 * kb] = k0
    assert oracle.check_export(b)[0] & oracle.V_SORTED


def test_checker_flags_bad_separator():
    _, b = _tree_export()
    o, kb, _ = _inner_off(b, 0)
    b[o:o + kb] = np.frombuffer(np.uint64(5).tobytes(), dtype=np.uint8)
    assert oracle.check_export(b)[0] & oracle.V_SEPARATOR


def test_checker_flags_broken_chain():
    _, b = _tree_export()
    o, kb, Cc = _leaf_off(b, 3)
    nx = o + 2 * Cc * kb + 4
    b[nx:nx + 4] = np.frombuffer(np.uint32(9).tobytes(), dtype=np.uint8)
    assert oracle.check_export(b)[0] & oracle.V_CHAIN


def test_checker_flags_shared_child():
    _, b = _tree_export()
    o, kb, F = _inner_off(b, 0)
    c0 = o + F * kb
    b[c0 + 4:c0 + 8] = b[c0:c0 + 4]
    assert oracle.check_export(b)[0] & oracle.V_REACH


def test_checker_flags_underfull_leaf_and_count():
    _, b = _tree_export()
    o, kb, Cc = _leaf_off(b, 2)
    b[o + 2 * Cc * kb:o + 2 * Cc * kb + 4] = np.frombuffer(np.uint32(3).tobytes(), dtype=np.uint8)
    bits = oracle.check_export(b)[0]
    assert bits & oracle.V_FILL and bits & oracle.V_COUNT


def test_checker_flags_bad_padding():
    pt = oracle.PointerTree(16, 16, 64)
    keys = np.arange(20, dtype=np.uint64)
    pt.bulk_load(keys, keys)            # two leaves of 10
    b = pt.export()
    o, kb, Cc = _leaf_off(b, 0)
    b[o + 12 * kb:o + 13 * kb] = np.frombuffer(np.uint64(0).tobytes(), dtype=np.uint8)
    assert oracle.check_export(b)[0] & oracle.V_PADDING


def test_checker_flags_unequal_depth():
    _, b = _tree_export()
    h = _hdr(b)
    h[4] += 1
    b[:40] = np.frombuffer(h.tobytes(), dtype=np.uint8)
    assert oracle.check_export(b)[0] & oracle.V_DEPTH


def _hand_export(shape, width):
    """A flat export written by hand from a nested shape: an inner node is a
    list of children, a leaf is an int (its key count).  Keys are 10, 20, 30,
    ... in leaf order; values are the keys plus one.  The layout follows the
    export format the library documents (entry i of an inner node is the
    largest key below child i, unused entries hold the largest key, unused
    child slots hold 0xFFFFFFFF; leaf slots past the count repeat the last
    key; the chain links plain leaf indices)."""
    kb, F, Cc = width // 8, 16, 16
    maxk = (1 << width) - 1
    inner, leaves = [], []
    nxt = [10]

    def depth(s):
        return 1 if isinstance(s, int) else 1 + depth(s[0])

    def make(s):
        if isinstance(s, int):
            ks = [nxt[0] + 10 * i for i in range(s)]
            nxt[0] += 10 * s
            leaves.append(ks)
            return (len(leaves) - 1) | 0x80000000, ks[-1]
        me = len(inner)
        inner.append(None)
        refs, tops = zip(*[make(c) for c in s])
        inner[me] = (list(refs), list(tops))
        return me, tops[-1]

    root, _ = make(shape)
    dt = np.uint32 if width == 32 else np.uint64
    out = bytearray()
    nkeys = sum(len(k) for k in leaves)
    out += np.array([0x58455447, kb, F, Cc, depth(shape), root, 0 if leaves else 0xFFFFFFFF,
                     len(inner), len(leaves), 0], dtype=np.uint32).tobytes()
    out += np.array([nkeys], dtype=np.uint64).tobytes()
    for refs, tops in inner:
        seps = tops[:-1] + [maxk] * (F - len(tops) + 1)
        out += np.array(seps, dtype=dt).tobytes()
        out += np.array(refs + [0xFFFFFFFF] * (F - len(refs)), dtype=np.uint32).tobytes()
    for j, ks in enumerate(leaves):
        out += np.array(ks + [ks[-1]] * (Cc - len(ks)), dtype=dt).tobytes()
        out += np.array([k + 1 for k in ks] + [0] * (Cc - len(ks)), dtype=dt).tobytes()
        out += np.array([len(ks), j + 1 if j + 1 < len(leaves) else 0xFFFFFFFF],
                        dtype=np.uint32).tobytes()
    return np.frombuffer(bytes(out), dtype=np.uint8).copy()


@pytest.mark.parametrize("width", [32, 64])
def test_checker_flags_underfull_inner_node(width):
    """Section III: every inner node but the root has at least m/2 = 8
    children.  A parent with 7 leaves under a valid root is flagged (fill
    only); the same tree with 8 is accepted."""
    ok = _hand_export([[8] * 8, [8] * 8], width)
    bits, ek, _ = oracle.check_export(ok)
    assert bits == 0, oracle.violations(bits)
    assert len(ek) == 128
    bad = _hand_export([[8] * 8, [8] * 7], width)
    assert oracle.check_export(bad)[0] == oracle.V_FILL
    # a full leaf count does not hide it: 7 children of 16 keys each
    bad = _hand_export([[16] * 8, [16] * 7], width)
    assert oracle.check_export(bad)[0] == oracle.V_FILL


@pytest.mark.parametrize("width", [32, 64])
def test_checker_flags_inner_root_with_one_child(width):
    """The root is exempt from the half-full rule but, when inner, has at
    least two children: a root over one parent is flagged (fill only); a
    root over two parents, and a root with exactly 2 leaves, are accepted."""
    bad = _hand_export([[8] * 8], width)
    assert oracle.check_export(bad)[0] == oracle.V_FILL
    assert oracle.check_export(_hand_export([[8] * 8, [8] * 8], width))[0] == 0
    assert oracle.check_export(_hand_export([8, 8], width))[0] == 0
    assert oracle.check_export(_hand_export([16], width))[0] == oracle.V_FILL


@pytest.mark.parametrize("width", [32, 64])
def test_checker_flags_overfull_inner_node(width):
    """No inner node exceeds the order: 16 children is the most an export
    can even describe; a 16-child parent is valid."""
    assert oracle.check_export(_hand_export([[8] * 16, [8] * 8], width))[0] == 0


# ------------------------------------------------------- random sequences

ops = st.lists(
    st.tuples(st.sampled_from(["ins", "look", "range"]),
              st.lists(st.integers(0, 300), min_size=0, max_size=40)),
    min_size=1, max_size=12)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(init=st.lists(st.integers(0, 300), unique=True, max_size=80), seq=ops,
       width=st.sampled_from([32, 64]))
def test_random_sequences(init, seq, width):
    vals = [(k * 2654435761) & ((1 << width) - 1) for k in init]
    br = Brute(init, vals, width)
    sa = oracle.SortedArray(init, vals, width)
    pt = oracle.PointerTree(16, 16, width)
    pt.bulk_load(init, vals)
    for t, (op, ks) in enumerate(seq):
        if op == "ins":
            vs = [(k * 40503 + t) & ((1 << width) - 1) for k in ks]
            s1 = br.insert(ks, vs)
            assert list(sa.insert(ks, vs)) == s1
            assert list(pt.insert(ks, vs)) == s1
            bits, ek, ev = oracle.check_export(pt.export())
            assert bits == 0, oracle.violations(bits)
            bk, bv = br.items()
            assert [int(x) for x in ek] == bk and [int(x) for x in ev] == bv
        elif op == "look":
            bv, bf = br.lookup(ks)
            for impl in (sa, pt):
                v, f = impl.lookup(ks)
                assert list(f) == bf and [int(x) for x in v] == bv
        else:
            lo = ks
            hi = [k + 25 for k in ks]
            mc = [(k % 7) + 1 for k in ks]
            want = br.range(lo, hi, mc)
            for impl in (sa, pt):
                cnt, off, ok, ov = impl.range(lo, hi, mc)
                for i, w in enumerate(want):
                    assert [(int(ok[off[i] + j]), int(ov[off[i] + j])) for j in range(int(cnt[i]))] == w
