"""The one-launch insert (batches of 2 to 64 keys) against the four-kernel
small-batch path and the oracle.  Two trees built from the same keys take
the same sequence of batches, one in one launch and one through the four
kernels (testing switch off); statuses must equal the oracle's, and the two
trees' exports must be equal byte for byte (same node ids, separators,
padding and chain), with the oracle's checker and content comparison on
top.  Batches mix new keys, present keys (updates), repeats within a batch
(the last value wins) and the edge keys; trees at fill 1.0 make the first
batches split every level and grow the root; a batch that does not fit is
refused by both in the same way."""
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
    prev = g.set_one_launch_insert(one)
    try:
        return t.insert(k, v)
    finally:
        g.set_one_launch_insert(prev)


def _run_batches(g, a, b, sa, batches, width, seed, every, tag):
    rng = np.random.default_rng(seed)
    vmax = np.iinfo(np.uint32).max if width == 32 else np.iinfo(np.int64).max
    for i, kk in enumerate(batches):
        vv = rng.integers(0, vmax, len(kk), dtype=np.uint64).astype(kk.dtype)
        want = sa.insert(kk, vv)
        sta = _insert(g, a, kk, vv, True)
        stb = _insert(g, b, kk, vv, False)
        assert np.array_equal(sta, want) and np.array_equal(stb, want), f"{tag}: status differs at batch {i}"
        if i % every == every - 1 or i + 1 == len(batches):
            ea, eb = a.export(), b.export()
            assert len(ea) == len(eb) and np.array_equal(ea, eb), f"{tag}: trees differ after batch {i}"
            assert_lookup_parity(a, sa, kk)
    assert g.tree_device_error(a.h) == g.GT_OK and g.tree_device_error(b.h) == g.GT_OK
    assert a.stats() == b.stats()
    assert_export_parity(a, sa)


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n", [0, 1, 17, 300, 4096, 65536])
def test_small_insert_batches_match_four_kernels(width, n):
    """Batches of 2..64 keys: mostly new keys, with present keys, repeats
    inside a batch and the edge keys."""
    import paper_2604_21117_amd as g
    seed = 900 + n + width
    rng = np.random.default_rng(seed)
    keys = key_set(n, width, seed, edges=n > 2)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    top = np.iinfo(keys.dtype).max
    fresh = synth.uniform_keys(64 * 80, seed + 7, width, purpose=synth.P_INSERT, exclude=keys)
    pool = np.concatenate([keys[:64], np.array([0, top, 1, top - 1], dtype=keys.dtype)])
    batches, at = [], 0
    for i in range(40 if n <= 300 else 80):
        B = int(rng.integers(2, 65))
        take = fresh[at:at + B]
        at += B
        kk = np.concatenate([take, pool[rng.integers(0, len(pool), B // 4 + 1)]])
        kk = np.concatenate([kk, kk[rng.integers(0, len(kk), B // 8 + 1)]])[:64]
        batches.append(kk[rng.permutation(len(kk))].astype(keys.dtype))
    _run_batches(g, a, b, sa, batches, width, seed, 4, f"n={n}")
    assert_lookup_parity(a, sa, np.concatenate([np.concatenate(batches), keys[:300]]))


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("B", [2, 8, 64])
def test_small_insert_batches_grow_full_tree(width, B):
    """A tree of 16^3 keys at fill 1.0 (height 3, every node full): the
    first batches split leaves, parents and the root, and the tree grows;
    later ones land in half-full pieces."""
    import paper_2604_21117_amd as g
    seed = 31 + B
    keys = (np.arange(1, 4097, dtype=np.uint64) * 64).astype(np.uint32 if width == 32 else np.uint64)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    assert a.stats()["height"] == 3
    fresh = synth.uniform_keys(B * 40, seed + 1, width, purpose=synth.P_INSERT, exclude=keys)
    fresh = (fresh % np.array(64 * 4097, dtype=keys.dtype)).astype(keys.dtype)  # inside the key range
    batches = [fresh[c:c + B] for c in range(0, len(fresh), B)]
    _run_batches(g, a, b, sa, batches, width, seed, 1, f"B={B}")
    assert a.stats()["height"] >= 4


def test_small_insert_capacity_refusal_matches_four_kernels():
    """No room for new leaves: the one-launch insert refuses like the four
    kernels (capacity error, tree unchanged), and both then take a batch of
    updates of present keys."""
    import paper_2604_21117_amd as g
    width, seed = 64, 17
    keys = synth.uniform_keys(4096, seed, width)
    vals = synth.values_for(keys, seed, width)
    p = g.make_params(8, max_batch=64)
    arena = g.tree_arena_bytes(p, len(keys), 0)  # full leaves, no room for new ones
    a = mk_tree(keys, vals, 8, arena_bytes=arena, max_batch=64)
    b = mk_tree(keys, vals, 8, arena_bytes=arena, max_batch=64)
    before = a.export()
    kk = synth.uniform_keys(40, seed + 1, width, purpose=synth.P_INSERT, exclude=keys)
    vv = synth.values_for(kk, seed, width)
    for t, one in ((a, True), (b, False)):
        with pytest.raises(g.GtError) as e:
            _insert(g, t, kk, vv, one)
        assert e.value.status == g.GT_ERR_CAPACITY
        assert np.array_equal(t.export(), before)
    sa = oracle.SortedArray(keys, vals, width)
    kp = keys[100:140].copy()
    vp = synth.values_for(kp, seed + 9, width)
    want = sa.insert(kp, vp)
    assert np.array_equal(_insert(g, a, kp, vp, True), want)
    assert np.array_equal(_insert(g, b, kp, vp, False), want)
    assert np.array_equal(a.export(), b.export())
    assert_export_parity(a, sa)


@pytest.mark.parametrize("width", [32, 64])
def test_small_insert_batches_of_one_repeated_key(width):
    """Degenerate batches: one key repeated 2..64 times (new, then present,
    the edge keys 0 and the largest), all keys already present (updates
    only), and a batch of 64 distinct keys inside one leaf's range."""
    import paper_2604_21117_amd as g
    seed = 71
    keys = key_set(4096, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    top = np.iinfo(keys.dtype).max
    fresh = synth.uniform_keys(8, seed + 3, width, purpose=synth.P_INSERT, exclude=keys)
    batches = []
    for k, n in ((fresh[0], 2), (fresh[1], 64), (fresh[1], 17), (keys[5], 33), (0, 64), (top, 64), (fresh[2], 3)):
        batches.append(np.full(n, k, dtype=keys.dtype))
    batches.append(keys[100:164].copy())
    srt = np.sort(keys)
    lo = int(srt[2000])
    run = np.arange(lo + 1, lo + 65, dtype=np.uint64).astype(keys.dtype)
    batches.append(run[~np.isin(run, keys)][:64])
    _run_batches(g, a, b, sa, [x for x in batches if len(x) >= 2], width, seed, 1, "degenerate")
