"""GPU parity of the delete batch (Section III: nodes stay at least half
full) against the oracle: per-key statuses, the remaining pairs and every
structural invariant of the exported tree (sorted leaves, equal depth,
fill, separators, chain, reachability, padding), then lookups of every kind
on the shrunken tree.  Batches mix present, absent and repeated keys; both
sort paths (up to 2048 keys and above); merges inside a leaf parent, the
root shrinking to one leaf, and the rebuild when a parent would underflow."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree, key_set, assert_export_parity, assert_lookup_parity, assert_range_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_21117_amd as g
    g.lib()


def _del_batch(present, B, seed, width, frac_present=0.7):
    """B keys: present ones (some repeated), absent ones and the edge keys."""
    rng = np.random.default_rng(seed)
    dt = np.uint64 if width == 64 else np.uint32
    parts = []
    npres = int(B * frac_present) if len(present) else 0
    if npres:
        parts.append(np.asarray(present, dtype=dt)[rng.integers(0, len(present), npres)])
    parts.append(synth.uniform_keys(B - npres, seed + 1, width))
    k = np.concatenate(parts)[:B]
    if B >= 4:
        k[:2] = [0, np.iinfo(dt).max]
    return synth.shuffle(k, seed).astype(dt)


def _check_all(t, sa, width, seed, tag):
    assert_export_parity(t, sa)
    allk, _ = sa.items()
    q = synth.mixed_queries(allk, 2000, seed, width) if len(allk) else synth.uniform_keys(2000, seed, width)
    assert_lookup_parity(t, sa, q)
    gv, gf = t.lookup_levelwise(q)
    ov, of = sa.lookup(q)
    assert np.array_equal(gf, of) and np.array_equal(gv, ov), f"{tag}: level-wise"
    st = t.stats()
    assert st["n_keys"] == len(sa), f"{tag}: n_keys"


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n", [0, 1, 16, 17, 300, 5000, 70000])
def test_delete_sizes(width, n):
    seed = 1200 + n
    keys = key_set(n, width, seed, edges=(n % 2 == 1))
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=1 << 15)
    # above 16384 keys the merge list comes from a scan (key order)
    for i, B in enumerate((1, 7, 64, 1000, 2049, 5000, 20000)):
        allk, _ = sa.items()
        k = _del_batch(allk, B, seed + 10 * i, width)
        st = t.delete(k)
        assert np.array_equal(st, sa.delete(k)), f"n={n} B={B}: statuses"
        _check_all(t, sa, width, seed + i, f"n={n} B={B}")
    t.close()


@pytest.mark.parametrize("width", [32, 64])
def test_delete_until_empty_then_reinsert(width):
    """Deleting every key in batches shrinks the tree to one empty leaf; the
    tree then takes inserts again."""
    seed = 1300 + width
    keys = key_set(6000, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=1 << 12, max_batch=8192)
    order = synth.shuffle(keys, seed)
    for part in np.array_split(order, 5):
        st = t.delete(part)
        assert st.all() and np.array_equal(st, sa.delete(part))
        _check_all(t, sa, width, seed, "emptying")
    s = t.stats()
    assert s["n_keys"] == 0 and s["height"] == 1
    assert not t.delete(keys[:100]).any()
    nv = synth.values_for(keys, seed + 1, width)
    assert not t.insert(keys, nv).any()
    sa.insert(keys, nv)
    _check_all(t, sa, width, seed + 2, "re-inserted")
    t.close()


@pytest.mark.parametrize("width", [32, 64])
def test_delete_contiguous_slices(width):
    """Deleting runs of consecutive keys empties whole leaves and leaf
    parents: merges, and the rebuild when a parent would underflow."""
    seed = 1400 + width
    keys = np.sort(key_set(40000, width, seed))
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=8192)
    h0 = t.stats()["height"]
    for i, (a, b) in enumerate(((100, 130), (1000, 1200), (5000, 9000), (20000, 28000), (0, 3))):
        k = keys[a:b]
        st = t.delete(synth.shuffle(k, seed + i))
        assert np.array_equal(st, sa.delete(k)), f"slice {a}:{b}"
        _check_all(t, sa, width, seed + i, f"slice {a}:{b}")
    # nearly everything: the height goes down
    allk, _ = sa.items()
    k = allk[: len(allk) - 200]
    for part in np.array_split(k, 4):
        st = t.delete(part)
        assert np.array_equal(st, sa.delete(part))
        _check_all(t, sa, width, seed + 9, "nearly all")
    assert t.stats()["height"] < h0
    t.close()


@pytest.mark.parametrize("width", [32, 64])
def test_delete_interleaved_with_inserts(width):
    """Inserts leave leaves about half full, so single deletes merge; ranges
    and the learned index follow the tree (the index answers through the
    tree after a delete, and from its models again after training)."""
    import paper_2604_21117_amd as g
    seed = 1500 + width
    keys = key_set(3000, width, seed)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=1 << 13, max_batch=8192)
    li = g.Learned(t, models=64)
    li.train()
    rng = np.random.default_rng(seed)
    for step in range(8):
        nk = synth.uniform_keys(int(rng.integers(100, 4000)), seed + 100 + step, width)
        nv = synth.values_for(nk, seed + 200 + step, width)
        assert np.array_equal(t.insert(nk, nv), sa.insert(nk, nv))
        allk, _ = sa.items()
        k = _del_batch(allk, int(rng.integers(1, 3000)), seed + 300 + step, width, 0.8)
        assert np.array_equal(t.delete(k), sa.delete(k)), f"step {step}"
        _check_all(t, sa, width, seed + step, f"step {step}")
        allk, _ = sa.items()
        q = synth.mixed_queries(allk, 3000, seed + 400 + step, width)
        ov, of = sa.lookup(q)
        lv, lf = li.lookup(q)
        assert np.array_equal(lf, of) and np.array_equal(lv, ov), f"learned, step {step}"
        lo = q[:200]
        hi = lo + (np.iinfo(lo.dtype).max // 1000)
        hi = np.maximum(hi, lo)
        assert_range_parity(t, sa, lo, hi, np.full(200, 40, dtype=np.uint32))
        if step % 3 == 2:
            li.train()
            lv, lf = li.lookup(q)
            assert np.array_equal(lf, of) and np.array_equal(lv, ov), f"retrained, step {step}"
    li.close()
    t.close()


@pytest.mark.parametrize("width", [32, 64])
def test_delete_from_half_full_tree(width):
    """A bulk load at fill 0.5 leaves every leaf with 8 keys and every inner
    node with about 8 children, so a single delete leaves a leaf below half
    full whose parent cannot merge without falling below half full itself:
    every batch takes the in-place rebuild (at the tree's fill)."""
    seed = 1700 + width
    keys = key_set(50000, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, fill=0.5, max_batch=8192)
    for i, B in enumerate((1, 2, 16, 300, 3000, 8192)):
        allk, _ = sa.items()
        k = _del_batch(allk, B, seed + 10 * i, width, 0.9)
        assert np.array_equal(t.delete(k), sa.delete(k)), f"B={B}"
        _check_all(t, sa, width, seed + i, f"half full, B={B}")
    t.close()


@pytest.mark.parametrize("width", [32, 64])
def test_delete_grandparent_merges_and_root_shrink(width):
    """A height-3 tree at fill 0.5: a delete leaves a leaf parent below 64
    keys, so the root (the grandparent) merges its parents.  Deleting down
    to 200 keys leaves one parent as the root (height 2), down to 10 keys
    one leaf (height 1)."""
    seed = 1800 + width
    keys = key_set(800, width, seed, edges=True)  # 100 leaves of 8, 12 parents, a root
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, fill=0.5, max_batch=4096)
    assert t.stats()["height"] == 3
    for i, B in enumerate((1, 5, 40)):
        allk, _ = sa.items()
        k = _del_batch(allk, B, seed + 10 * i, width, 1.0)
        assert np.array_equal(t.delete(k), sa.delete(k)), f"B={B}"
        _check_all(t, sa, width, seed + i, f"grandparent, B={B}")
    assert t.stats()["height"] == 3
    for left, height in ((200, 2), (10, 1)):
        allk, _ = sa.items()
        k = synth.shuffle(allk, seed + left)[: len(allk) - left]
        assert t.delete(k).all() and sa.delete(k).all()
        _check_all(t, sa, width, seed + left, f"down to {left}")
        assert t.stats()["height"] == height, f"down to {left}"
    t.close()


@pytest.mark.parametrize("seed", range(12))
def test_delete_random_sequences(seed):
    """Random interleavings of insert and delete batches of random sizes on
    small trees (fill 0.5 or 1.0, a few hundred to a few thousand keys, u32
    and u64), so that leaf-parent merges, grandparent merges, root shrinks,
    rebuilds and regrowth follow each other; statuses, invariants and
    lookups against the oracle after every step."""
    rng = np.random.default_rng(2000 + seed)
    width = 32 if seed % 2 else 64
    n = int(rng.integers(100, 4000))
    keys = key_set(n, width, 2100 + seed, edges=(seed % 3 == 0))
    vals = synth.values_for(keys, 2100 + seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, fill=0.5 if seed % 4 < 2 else 1.0, leaf_slack=1 << 14, max_batch=4096)
    for step in range(10):
        allk, _ = sa.items()
        if rng.random() < 0.6 and len(allk):
            frac = float(rng.choice([0.05, 0.3, 0.9]))
            B = max(1, min(4096, int(len(allk) * frac) + int(rng.integers(0, 20))))
            k = _del_batch(allk, B, 2200 + 17 * seed + step, width, float(rng.choice([0.5, 0.95])))
            assert np.array_equal(t.delete(k), sa.delete(k)), f"seed {seed} step {step}: delete statuses"
        else:
            B = int(rng.integers(1, 3000))
            nk = synth.uniform_keys(B, 2300 + 17 * seed + step, width)
            nv = synth.values_for(nk, 2400 + step, width)
            assert np.array_equal(t.insert(nk, nv), sa.insert(nk, nv)), f"seed {seed} step {step}: insert"
        _check_all(t, sa, width, 2500 + step, f"seed {seed} step {step}")
    t.close()


def test_delete_argument_errors():
    import torch
    import paper_2604_21117_amd as g
    keys = key_set(100, 64, 1600)
    t = mk_tree(keys, synth.values_for(keys, 1600, 64), 8, max_batch=256)
    L = g.lib()
    k = t.dev(keys[:10])
    st = torch.empty(300, dtype=torch.uint8, device="cuda")
    big = t.dev(synth.uniform_keys(300, 1601, 64))
    assert L.tree_delete_batch(t.h, g._ptr(big), 300, g._ptr(st), None) == g.GT_ERR_CAPACITY
    assert L.tree_delete_batch(t.h, None, 10, g._ptr(st), None) == g.GT_ERR_INVALID
    assert L.tree_delete_batch(t.h, g._ptr(k), 10, None, None) == g.GT_ERR_INVALID
    assert L.tree_delete_batch(None, g._ptr(k), 10, g._ptr(st), None) == g.GT_ERR_INVALID
    assert L.tree_delete_batch(t.h, None, 0, None, None) == g.GT_OK
    assert t.stats()["n_keys"] == 100
    t.close()
