"""Pins for the oracle's level-wise search (paper Sections IV-A and IV-F):
its results against the plain definition and brute force, and its FIFO
entries against an independent per-key walk of the exported tree.  CPU
only."""
import numpy as np
import pytest

import oracle
import synth
from oracle.brute import Brute


def _export_paths(buf, keys):
    """Per key, the node reference taken at each level, by walking the flat
    export (header, inner records, leaf records) one key at a time."""
    h = np.frombuffer(buf[:40].tobytes(), dtype=np.uint32)
    kb, F, height, root, n_inner = int(h[1]), int(h[2]), int(h[4]), int(h[5]), int(h[7])
    kdt = np.uint64 if kb == 8 else np.uint32
    rec = F * (kb + 4)
    inner = buf[48:48 + n_inner * rec]
    ikeys = [np.frombuffer(inner[i * rec:i * rec + F * kb].tobytes(), dtype=kdt) for i in range(n_inner)]
    ichild = [np.frombuffer(inner[i * rec + F * kb:(i + 1) * rec].tobytes(), dtype=np.uint32)
              for i in range(n_inner)]
    paths = []
    for k in keys:
        k = int(k)
        ref, p = root, [root]
        for _ in range(height - 1):
            sep = ikeys[ref]
            # first child whose entry is >= the key: count the entries below it
            c = sum(1 for i in range(F - 1) if int(sep[i]) < k)
            ref = int(ichild[ref][c])
            p.append(ref)
        paths.append(p)
    return paths, height


def _runs_by_level(runs, level):
    m = runs["level"] == level
    return runs["first"][m], runs["count"][m], runs["node"][m]


def _trees(width):
    """(name, pointer tree, sorted array) cases: empty, one key, one full
    leaf, two leaves, bulk loads at fill 1 and 0.5, and a tree grown by
    inserts (rewritten inner nodes, a taller root)."""
    rng = np.random.default_rng(11 + width)
    top = (1 << width) - 1
    out = []
    for n, fill in ((0, 1.0), (1, 1.0), (16, 1.0), (17, 1.0), (300, 1.0), (5000, 1.0), (5000, 0.5)):
        ks = np.unique(rng.integers(0, top, size=n, endpoint=True, dtype=np.uint64))
        if width == 32:
            ks = ks.astype(np.uint32)
        vs = synth.values_for(ks, 5, width)
        pt = oracle.PointerTree(16, 16, width)
        pt.bulk_load(ks, vs, fill)
        out.append((f"n{n}_f{fill}", pt, oracle.SortedArray(ks, vs, width), ks))
    ks = np.unique(rng.integers(0, top, size=400, endpoint=True, dtype=np.uint64))
    if width == 32:
        ks = ks.astype(np.uint32)
    vs = synth.values_for(ks, 6, width)
    pt = oracle.PointerTree(16, 16, width)
    pt.bulk_load(ks, vs)
    sa = oracle.SortedArray(ks, vs, width)
    for b in range(6):
        nk = rng.integers(0, top, size=900, endpoint=True, dtype=np.uint64)
        if width == 32:
            nk = nk.astype(np.uint32)
        nv = synth.values_for(nk, 7 + b, width)
        pt.insert(nk, nv)
        sa.insert(nk, nv)
    k_all, _ = sa.items()
    out.append(("grown", pt, sa, k_all))
    return out


def _sorted_batch(rng, present, width, B):
    top = (1 << width) - 1
    parts = [rng.integers(0, top, size=B // 2, endpoint=True, dtype=np.uint64)]
    if len(present):
        parts.append(np.asarray(present, dtype=np.uint64)[rng.integers(0, len(present), size=B - B // 2)])
    parts.append(np.array([0, top, top, 0], dtype=np.uint64))
    q = np.sort(np.concatenate(parts))
    return q.astype(np.uint32) if width == 32 else q


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_results_equal_the_plain_definition(width):
    rng = np.random.default_rng(3)
    for name, pt, sa, present in _trees(width):
        for B in (1, 7, 64, 1000):
            q = _sorted_batch(rng, present, width, B)
            v, f, _ = pt.lookup_levelwise(q)
            ev, ef = sa.lookup(q)
            assert np.array_equal(f, ef), name
            assert np.array_equal(v, ev), name


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_runs_follow_the_fifo_rules(width):
    """Per level the entries cut the sorted batch into consecutive runs that
    cover it exactly (the running key index of Section IV-A), each node
    appears once per level, level 0 is the root with the whole batch, and
    no run grows from one level to the next."""
    rng = np.random.default_rng(4)
    for name, pt, sa, present in _trees(width):
        q = _sorted_batch(rng, present, width, 999)
        _, _, runs = pt.lookup_levelwise(q)
        height = pt.stats()["height"]
        assert set(np.unique(runs["level"]).tolist()) == set(range(height)), name
        first0, count0, _ = _runs_by_level(runs, 0)
        assert list(count0) == [len(q)] and list(first0) == [0]
        prev_max = len(q)
        for lvl in range(height):
            first, count, node = _runs_by_level(runs, lvl)
            assert int(first[0]) == 0 and int(count.sum()) == len(q), name
            assert np.array_equal(first[1:], (first + count)[:-1]), name
            assert len(np.unique(node)) == len(node), name
            assert int(count.max()) <= prev_max
            prev_max = int(count.max())


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_runs_equal_an_independent_walk(width):
    """The runs at each level are exactly the maximal groups of consecutive
    sorted keys that an independent one-key-at-a-time walk of the exported
    tree sends through the same node."""
    rng = np.random.default_rng(5)
    for name, pt, sa, present in _trees(width):
        q = _sorted_batch(rng, present, width, 500)
        _, _, runs = pt.lookup_levelwise(q)
        paths, height = _export_paths(pt.export(), q)
        for lvl in range(height):
            nodes = [p[lvl] for p in paths]
            heads = [i for i in range(len(nodes)) if i == 0 or nodes[i] != nodes[i - 1]]
            counts = [b - a for a, b in zip(heads, heads[1:] + [len(nodes)])]
            first, count, _ = _runs_by_level(runs, lvl)
            assert [int(x) for x in first] == heads, (name, lvl)
            assert [int(x) for x in count] == counts, (name, lvl)


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_vs_brute_tiny(width):
    rng = np.random.default_rng(6)
    top = (1 << width) - 1
    for trial in range(20):
        n = int(rng.integers(0, 60))
        ks = sorted({int(x) for x in rng.integers(0, 200, size=n)} | ({0, top} if trial % 3 == 0 else set()))
        vs = [(k * 2654435761 + trial) & top for k in ks]
        br = Brute(ks, vs, width)
        pt = oracle.PointerTree(16, 16, width)
        pt.bulk_load(ks, vs)
        q = sorted(int(x) for x in rng.integers(0, 210, size=int(rng.integers(1, 64))))
        q += [top] if trial % 2 else [0]
        q.sort()
        bv, bf = br.lookup(q)
        v, f, _ = pt.lookup_levelwise(q)
        assert list(f) == bf and [int(x) for x in v] == bv


def test_levelwise_needs_an_ascending_batch():
    pt = oracle.PointerTree(16, 16, 64)
    pt.bulk_load(np.arange(100, dtype=np.uint64), np.arange(100, dtype=np.uint64))
    with pytest.raises(ValueError):
        pt.lookup_levelwise(np.array([5, 3], dtype=np.uint64))
    v, f, runs = pt.lookup_levelwise(np.array([], dtype=np.uint64))
    assert len(v) == 0 and len(runs["level"]) == 0
