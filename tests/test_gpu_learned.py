"""Learned index: results identical to the oracle (hence to the tree) on
every key set, error bounds exact over every trained key (predictions taken
from the GPU inference kernel itself), and a wrong window or a stale
directory costing fallbacks only."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree, assert_lookup_parity, chain_positions, key_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()


def _learned(tree, **kw):
    import paper_2604_21117_amd as g
    li = g.Learned(tree, **kw)
    li.train()
    return li


def _li_parity(li, sa, q):
    gv, gf = li.lookup(q)
    ov, of = sa.lookup(q)
    assert np.array_equal(gf, of), f"found differs at {np.nonzero(gf != of)[0][:8]}"
    assert np.array_equal(gv, ov), f"values differ at {np.nonzero(gv != ov)[0][:8]}"


def _check_bounds(tree, li):
    keys, pos, L = chain_positions(tree.export())
    m, p, lo, hi, kind = li.predict(keys)
    used = kind != 2
    err = pos - p.astype(np.int64)
    assert np.all(err[used] >= lo[used]) and np.all(err[used] <= hi[used])
    # the bounds are the exact extremes over the keys routed to each model
    for j in np.unique(m[used])[:200]:
        sel = used & (m == j)
        assert err[sel].min() == lo[sel][0] and err[sel].max() == hi[sel][0]
    return used.mean()


@pytest.mark.parametrize("search", [0, 1, 2])
@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("dist", ["uniform", "lognormal", "clustered"])
def test_learned_parity_and_bounds(width, dist, search):
    seed = 41
    n = 1 << 18
    if dist == "uniform":
        keys = synth.uniform_keys(n, seed, width)
    elif width == 32:
        pytest.skip("lognormal / clustered keys are u64 workloads")
    elif dist == "lognormal":
        keys = synth.lognormal_keys(n, seed)
    else:
        keys = synth.clustered_keys(n, seed)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=1 << 14, max_batch=1 << 14)
    # gate=1: the model path runs even where the quality gate would decline
    li = _learned(t, models=256, search=search, gate=1)
    assert li.stats()["declined"] == 0
    frac_used = _check_bounds(t, li)
    # keys in pieces with bounds (the rest walk the tree): uniform keys are
    # the model's workload; on clustered keys the uniform knot grid cannot
    # follow the cluster edges and more pieces exceed the window limit
    assert frac_used > {"uniform": 0.95, "lognormal": 0.5, "clustered": 0.3}[dist]
    q = synth.mixed_queries(keys, 60000, seed, width)
    _li_parity(li, sa, q)
    st = li.stats()
    assert st["lookups"] == 60000
    _li_parity(li, sa, q[:1024])  # a small batch (the default reads windows directly)
    # present keys inside their model's window never need the tree
    pres = synth.present_queries(keys, 20000, seed + 1)
    before = li.stats()["fallbacks"]
    _li_parity(li, sa, pres)
    assert li.stats()["fallbacks"] - before <= 20000 * (1 - frac_used) + 200


@pytest.mark.parametrize("kind", [1, 2])
def test_kinds(kind):
    seed, width = 43, 64
    keys = synth.lognormal_keys(100000, seed)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    li = _learned(t, models=128, kind=kind, max_window=256, gate=1)
    st = li.stats()
    if kind == 1:
        assert st["mlp_models"] == 0
    else:
        assert st["linear_models"] == 0 or st["mlp_models"] > 0
    _check_bounds(t, li)
    _li_parity(li, sa, synth.mixed_queries(keys, 30000, seed, width))


@pytest.mark.parametrize("dist", ["uniform", "lognormal", "clustered"])
def test_quality_gate(dist):
    """With the default gate an index whose models send many keys down the
    tree, or have wide windows, declines: lookups run the tree kernel (the
    model's counters do not move) and stay exact; uniform keys keep the
    model path.  gate=1 keeps the model path everywhere."""
    seed, width, n = 49, 64, 1 << 18
    keys = {"uniform": lambda: synth.uniform_keys(n, seed, width),
            "lognormal": lambda: synth.lognormal_keys(n, seed),
            "clustered": lambda: synth.clustered_keys(n, seed)}[dist]()
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    q = synth.mixed_queries(keys, 5000, seed, width)
    for gate in (0, 1):
        li = _learned(t, models=1024, gate=gate)
        st = li.stats()
        keys_tree_share = 1.0 - _check_bounds(t, li)
        expect = gate == 0 and (keys_tree_share > 0.25 or st["mean_window"] > 16.0)
        assert st["declined"] == (1 if expect else 0), (dist, gate, keys_tree_share, st["mean_window"])
        l0 = st["lookups"]
        _li_parity(li, sa, q)
        assert li.stats()["lookups"] - l0 == (0 if expect else len(q))
        if dist == "uniform":
            assert st["declined"] == 0
        li.close()


def test_forced_fallback_stays_exact():
    """Windows of one leaf: most predictions miss the key's leaf, so a miss
    resumes along the leaf chain from the window or descends from the root;
    windows past the last leaf are empty, so every query descends from the
    root.  Every answer stays exact."""
    seed, width = 44, 64
    keys = synth.uniform_keys(200000, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    li = _learned(t, gate=1)
    q = synth.mixed_queries(keys, 50000, seed, width)
    li.set_bounds(0, 0)
    _li_parity(li, sa, q)
    f0 = li.stats()["fallbacks"]
    li.set_bounds(20000, 20000)
    _li_parity(li, sa, q)
    assert li.stats()["fallbacks"] - f0 == len(q)


@pytest.mark.parametrize("search", [1, 2])
def test_stale_after_inserts_then_retrain(search):
    """Inserts split leaves after training: keys move to leaves the model
    never saw, and two leaves adjacent at training are no longer adjacent,
    so gaps between them prove nothing; every answer must still be exact."""
    seed, width = 45, 64
    keys = synth.uniform_keys(300000, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 16, max_batch=1 << 14)
    li = _learned(t, search=search)
    rng = np.random.default_rng(seed)
    for b in range(5):
        ins = synth.uniform_keys(10000, seed + 100 + b, width, exclude=sa.keys)
        k = np.concatenate([ins, keys[rng.integers(0, len(keys), 500)]])
        v = synth.values_for(k, seed + b, width)
        assert np.array_equal(t.insert(k, v), sa.insert(k, v))
        q = np.concatenate([k[:3000], synth.mixed_queries(sa.keys, 6000, seed + b, width)])
        _li_parity(li, sa, q)
    # a miss on the changed tree resumes along the leaf chain from its
    # window; only keys below every window leaf descend from the root
    st = li.stats()
    assert st["fallbacks"] <= st["lookups"] // 10, st
    li.train()
    _check_bounds(t, li)
    _li_parity(li, sa, synth.mixed_queries(sa.keys, 40000, seed, width))


def _edge_queries(keys):
    """Keys next to every leaf boundary: each leaf's first key, one below it
    (between two leaves), its last key and one above it, plus 0 and the
    largest key."""
    sk = np.sort(keys)
    top = np.iinfo(sk.dtype).max
    first, last = sk[0::16], sk[15::16]
    one = sk.dtype.type(1)
    below = first[first > 0] - one
    above = last[last < top] + one
    return np.concatenate([first, below, last, above, np.array([0, top], dtype=sk.dtype)])


@pytest.mark.parametrize("search", [1, 2])
@pytest.mark.parametrize("width", [32, 64])
def test_fresh_tree_misses_are_answered_by_the_model(width, search):
    """On an unchanged bulk-loaded tree, absent keys between two leaves,
    below the first or above the last leaf are proved absent from the window
    alone (no tree walk), and every answer matches the oracle."""
    seed = 47
    keys = synth.uniform_keys(1 << 17, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=1 << 16)
    li = _learned(t, models=128, search=search)
    q = _edge_queries(keys)
    f0 = li.stats()["fallbacks"]
    _li_parity(li, sa, q)
    assert li.stats()["fallbacks"] - f0 <= len(q) // 100
    absent = synth.absent_queries(keys, 20000, seed, width)
    f0 = li.stats()["fallbacks"]
    _li_parity(li, sa, absent)
    assert li.stats()["fallbacks"] - f0 <= 200


def test_gap_proof_needs_an_unchanged_tree():
    """After one insert batch (the tree's epoch moves), a key that moved to a
    new leaf between two trained leaves is found, not reported absent."""
    seed, width = 48, 64
    keys = synth.uniform_keys(1 << 16, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 14, max_batch=1 << 14)
    li = _learned(t, models=64, search=2)
    sk = np.sort(keys)
    # one new key inside every 4th full leaf: each of those leaves splits
    # and its upper half moves to a new leaf
    lo, hi = sk[0::16][::4], sk[1::16][::4]
    ins = (lo + (hi - lo) // np.uint64(2)).astype(np.uint64)
    ins = ins[(ins > lo) & (ins < hi)]
    v = synth.values_for(ins, seed + 1, width)
    assert np.array_equal(t.insert(ins, v), sa.insert(ins, v))
    _li_parity(li, sa, np.concatenate([keys, ins, _edge_queries(sa.keys)]))


@pytest.mark.parametrize("n", [0, 1, 7, 100, 5000])
def test_small_trees(n):
    seed, width = 46, 64
    keys = key_set(n, width, seed, edges=n > 2)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    li = _learned(t, models=64)
    q = np.concatenate([keys, synth.absent_queries(keys, 300, seed, width),
                        np.array([0, np.iinfo(np.uint64).max], dtype=np.uint64)])
    _li_parity(li, sa, q)
