"""Helpers shared by the GPU parity tests (inputs come from synth, expected
values from the oracle)."""
import numpy as np

import oracle
import synth


def mk_tree(keys, vals, kb, **kw):
    import paper_2604_21117_amd as g
    return g.Tree(keys, vals, kb, **kw)


def assert_lookup_parity(tree, sa: oracle.SortedArray, q):
    gv, gf = tree.lookup(q)
    ov, of = sa.lookup(q)
    assert np.array_equal(gf, of), f"found flags differ at {np.nonzero(gf != of)[0][:8]}"
    assert np.array_equal(gv, ov), f"values differ at {np.nonzero(gv != ov)[0][:8]}"


def assert_export_parity(tree, sa: oracle.SortedArray):
    buf = tree.export()
    bits, ek, ev = oracle.check_export(buf, len(sa))
    assert bits == 0, oracle.violations(bits)
    assert np.array_equal(ek, sa.keys) and np.array_equal(ev, sa.vals)


def assert_range_parity(tree, sa: oracle.SortedArray, lo, hi, mc):
    gc, goff, gk, gv = tree.range(lo, hi, mc)
    oc, ooff, ok, ov = sa.range(lo, hi, mc)
    assert np.array_equal(gc, oc), f"range counts differ at {np.nonzero(gc != oc)[0][:8]}"
    for i in np.nonzero(oc)[0]:
        s = slice(int(ooff[i]), int(ooff[i] + oc[i]))
        assert np.array_equal(gk[s], ok[s]) and np.array_equal(gv[s], ov[s]), f"range {i} differs"


def key_set(n, width, seed, edges=False):
    k = synth.uniform_keys(n, seed, width)
    if edges and n >= 2:
        top = np.iinfo(k.dtype).max
        k = np.unique(np.concatenate([k[:n - 2], np.array([0, top], dtype=k.dtype)]))
        k = synth.shuffle(k, seed)
    return k


def chain_positions(buf):
    """From a tree export: every key in key order with the position (in the
    leaf chain) of the leaf that holds it."""
    buf = np.asarray(buf, dtype=np.uint8)
    h = np.frombuffer(buf[:40].tobytes(), dtype=np.uint32)
    kb, F, Cc, first, ni, nl = int(h[1]), int(h[2]), int(h[3]), int(h[6]), int(h[7]), int(h[8])
    kd = np.uint64 if kb == 8 else np.uint32
    rin, rlf = F * (kb + 4), Cc * 2 * kb + 8
    base = 48 + ni * rin
    leaves = buf[base: base + nl * rlf].reshape(nl, rlf)
    lkeys = leaves[:, :Cc * kb].copy().view(kd).reshape(nl, Cc)
    meta = leaves[:, 2 * Cc * kb:].copy().view(np.uint32).reshape(nl, 2)
    order = []
    x = first
    while x != 0xFFFFFFFF:
        order.append(x)
        x = int(meta[x, 1])
    keys, pos = [], []
    for p, leaf in enumerate(order):
        c = int(meta[leaf, 0])
        keys.append(lkeys[leaf, :c])
        pos.append(np.full(c, p, dtype=np.int64))
    return np.concatenate(keys), np.concatenate(pos), len(order)
