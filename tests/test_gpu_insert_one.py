"""The one-key insert kernel (a batch of B = 1) against the batch path and
the oracle.  Two trees built from the same keys take the same sequence of
one-key batches, one through the one-key kernel and one through the batch
path (testing switch off); statuses must equal the oracle's, and the two
trees' exports must be equal byte for byte (same node ids, separators,
padding and chain), with the oracle's checker and content comparison on
top.  Trees at fill 1.0 make every early insert split its whole path and
grow the root; the empty tree and a one-leaf root cover the degenerate
heights."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree, assert_lookup_parity, assert_export_parity, key_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()


def _insert(g, t, k, v, one):
    prev = g.set_single_key_insert(one)
    try:
        return t.insert(k, v)
    finally:
        g.set_single_key_insert(prev)


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n,steps,every", [(0, 120, 1), (1, 60, 1), (16, 120, 1), (256, 200, 1),
                                           (4096, 300, 3), (65536, 300, 25)])
def test_one_key_inserts_match_batch_path(width, n, steps, every):
    import paper_2604_21117_amd as g
    seed = 400 + n + width
    rng = np.random.default_rng(seed)
    keys = key_set(n, width, seed, edges=n > 2)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=2048, max_batch=64)
    b = mk_tree(keys, vals, width // 8, leaf_slack=2048, max_batch=64)
    top = np.iinfo(keys.dtype).max
    fresh = synth.uniform_keys(steps, seed + 7, width, purpose=synth.P_INSERT, exclude=keys)
    pool = np.concatenate([fresh, keys[:64], np.array([0, top, 1, top - 1], dtype=keys.dtype)])
    # mostly fresh keys in random order, with present keys, repeats and edges
    seq = np.where(rng.random(steps) < 0.8, fresh[rng.permutation(steps)], pool[rng.integers(0, len(pool), steps)])
    seq = seq.astype(keys.dtype)
    vmax = np.iinfo(np.uint32).max if width == 32 else np.iinfo(np.int64).max
    for i, k in enumerate(seq):
        kk = np.array([k], dtype=keys.dtype)
        vv = rng.integers(0, vmax, 1, dtype=np.uint64).astype(keys.dtype)
        want = sa.insert(kk, vv)
        sta = _insert(g, a, kk, vv, True)
        stb = _insert(g, b, kk, vv, False)
        assert np.array_equal(sta, want) and np.array_equal(stb, want), f"status differs at step {i}"
        if i % every == every - 1 or i + 1 == len(seq):
            ea, eb = a.export(), b.export()
            assert len(ea) == len(eb) and np.array_equal(ea, eb), f"trees differ after step {i}"
    assert g.tree_device_error(a.h) == g.GT_OK and g.tree_device_error(b.h) == g.GT_OK
    assert a.stats() == b.stats()
    assert_export_parity(a, sa)
    q = np.concatenate([seq, pool[rng.integers(0, len(pool), 300)]])
    assert_lookup_parity(a, sa, q)


@pytest.mark.parametrize("width", [32, 64])
def test_one_key_insert_grows_root_each_level(width):
    """A tree of 16^3 keys at fill 1.0 (height 3, every node full): the
    first new key splits its leaf, its parent and the root, and the height
    becomes 4; keys above the largest and below the smallest do the same on
    the chain's ends."""
    import paper_2604_21117_amd as g
    seed = 91
    keys = (np.arange(1, 4097, dtype=np.uint64) * 4).astype(np.uint32 if width == 32 else np.uint64)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=64, max_batch=16)
    b = mk_tree(keys, vals, width // 8, leaf_slack=64, max_batch=16)
    assert a.stats()["height"] == 3
    for k in (4 * 2000 + 1, 4 * 4096 + 7, 0, 4 * 1000 + 2, 4 * 4096 + 9):
        kk = np.array([k], dtype=keys.dtype)
        vv = synth.values_for(kk, seed + 1, width)
        want = sa.insert(kk, vv)
        assert np.array_equal(_insert(g, a, kk, vv, True), want)
        assert np.array_equal(_insert(g, b, kk, vv, False), want)
        assert np.array_equal(a.export(), b.export())
    assert a.stats()["height"] == 4
    assert_export_parity(a, sa)
    assert_lookup_parity(a, sa, np.concatenate([keys, np.array([0, 4 * 2000 + 1, 4 * 4096 + 9], dtype=keys.dtype)]))


def test_one_key_insert_capacity_refusal_matches_batch_path():
    """No room for a new leaf: the one-key kernel refuses like the batch
    path (capacity error, tree unchanged), and both then take an update of
    a present key."""
    import paper_2604_21117_amd as g
    width, seed = 64, 13
    keys = synth.uniform_keys(4096, seed, width)
    vals = synth.values_for(keys, seed, width)
    p = g.make_params(8, max_batch=16)
    arena = g.tree_arena_bytes(p, len(keys), 0)  # full leaves, no room for new ones
    a = mk_tree(keys, vals, 8, arena_bytes=arena, max_batch=16)
    b = mk_tree(keys, vals, 8, arena_bytes=arena, max_batch=16)
    before = a.export()
    kk = synth.uniform_keys(1, seed + 1, width, purpose=synth.P_INSERT, exclude=keys)
    vv = synth.values_for(kk, seed, width)
    for t, one in ((a, True), (b, False)):
        with pytest.raises(g.GtError) as e:
            _insert(g, t, kk, vv, one)
        assert e.value.status == g.GT_ERR_CAPACITY
        assert np.array_equal(t.export(), before)
    sa = oracle.SortedArray(keys, vals, width)
    kp = keys[5:6].copy()
    vp = synth.values_for(kp, seed + 9, width)
    want = sa.insert(kp, vp)
    assert np.array_equal(_insert(g, a, kp, vp, True), want)
    assert np.array_equal(_insert(g, b, kp, vp, False), want)
    assert np.array_equal(a.export(), b.export())
    assert_export_parity(a, sa)
