"""The one-launch delete (batches of at most 64 keys) against the batch path
and the oracle.  Two trees built from the same keys take the same sequence
of batches, one through the one-launch path and one through the batch
path's kernels (testing switch off); statuses must equal the oracle's, and
the two trees' exports must be equal byte for byte (same node ids,
separators, padding and chain), with the oracle's checker and content
comparison on top.  Deleting runs of consecutive keys empties leaves, leaf
parents and grandparents in turn, so the sequences pass through the parent
merges (several in one batch, one wave each), the grandparent merge, the
root shrinking level by level and the host's rebuild; random sequences mix
present, absent and repeated keys, within a batch too."""
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


def _delete(g, t, k, one):
    prev = g.set_one_launch_delete(one)
    try:
        return t.delete(k)
    finally:
        g.set_one_launch_delete(prev)


def _run(g, a, b, sa, seq, every, tag, heights=None):
    for i, k in enumerate(seq):
        kk = np.array([k], dtype=seq.dtype)
        want = sa.delete(kk)
        sta = _delete(g, a, kk, True)
        stb = _delete(g, b, kk, False)
        assert np.array_equal(sta, want) and np.array_equal(stb, want), f"{tag}: status differs at step {i}"
        if heights is not None:
            heights.add(a.stats()["height"])
        if i % every == every - 1 or i + 1 == len(seq):
            ea, eb = a.export(), b.export()
            assert len(ea) == len(eb) and np.array_equal(ea, eb), f"{tag}: trees differ after step {i}"
            # lookups go through the top-levels mirror, which the commit
            # refreshes only when a mirrored node changed
            assert_lookup_parity(a, sa, seq[max(0, i - 2 * every):i + 1])
    assert g.tree_device_error(a.h) == g.GT_OK and g.tree_device_error(b.h) == g.GT_OK
    assert a.stats() == b.stats()
    assert_export_parity(a, sa)


def _reinsert(a, b, sa, keys, width, seed):
    """Put deleted keys back (inserts also descend through the mirror)."""
    if len(keys) == 0:
        return
    vals = synth.values_for(keys, seed + 3, width)
    for c in range(0, len(keys), 16):
        kk, vv = keys[c:c + 16], vals[c:c + 16]
        want = sa.insert(kk, vv)
        assert np.array_equal(a.insert(kk, vv), want) and np.array_equal(b.insert(kk, vv), want)
    assert np.array_equal(a.export(), b.export())
    assert_export_parity(a, sa)


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n,steps,every", [(0, 40, 1), (1, 20, 1), (16, 60, 1), (17, 60, 1), (300, 400, 4),
                                           (4096, 600, 20), (65536, 400, 50)])
def test_one_key_deletes_match_batch_path(width, n, steps, every):
    """Mostly present keys in random order, with absent keys, keys deleted
    before and the edge keys."""
    import paper_2604_21117_amd as g
    seed = 500 + n + width
    rng = np.random.default_rng(seed)
    keys = key_set(n, width, seed, edges=n > 2)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    top = np.iinfo(keys.dtype).max
    absent = synth.uniform_keys(steps, seed + 7, width, purpose=synth.P_INSERT, exclude=keys)
    present = keys[rng.permutation(len(keys))] if len(keys) else absent
    pool = np.concatenate([absent, np.array([0, top, 1, top - 1], dtype=keys.dtype)])
    seq = np.where(rng.random(steps) < 0.75, present[np.arange(steps) % len(present)],
                   pool[rng.integers(0, len(pool), steps)]).astype(keys.dtype)
    _run(g, a, b, sa, seq, every, f"n={n}")
    q = np.concatenate([seq, keys[:300]]) if len(keys) else seq
    assert_lookup_parity(a, sa, q)
    _reinsert(a, b, sa, np.unique(seq[np.isin(seq, keys)])[:160], width, seed)
    assert_lookup_parity(a, sa, q)


@pytest.mark.parametrize("width", [32, 64])
def test_one_key_deletes_drain_a_tree(width):
    """Every key of a 16^3-key tree at fill 1.0 (height 3), in ascending
    order: leaves and leaf parents underflow and merge, the root's parents
    merge under it, and the tree shrinks to height 2, then 1, then empty."""
    import paper_2604_21117_amd as g
    seed = 77
    keys = (np.arange(1, 4097, dtype=np.uint64) * 5).astype(np.uint32 if width == 32 else np.uint64)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=16)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=16)
    assert a.stats()["height"] == 3
    heights = set()
    seq = keys.copy()
    for c in range(0, len(seq), 256):
        _run(g, a, b, sa, seq[c:c + 256], 32, f"keys {c}..", heights)
    assert a.stats()["n_keys"] == 0
    assert {3, 2, 1} <= heights
    _reinsert(a, b, sa, keys[::7], width, seed)
    assert_lookup_parity(a, sa, keys)


@pytest.mark.parametrize("width", [32, 64])
def test_one_key_deletes_of_a_key_run_at_height_4(width):
    """A run of 6000 consecutive keys out of 2^16 at fill 1.0 (height 4):
    parents and grandparents below the root underflow; the grandparent merge
    runs below the root, and once a grandparent would fall below half full
    the host rebuilds the tree (both paths report the same flag)."""
    import paper_2604_21117_amd as g
    seed = 5
    keys = (np.arange(1, 65537, dtype=np.uint64) * 3).astype(np.uint32 if width == 32 else np.uint64)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=16)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=16)
    assert a.stats()["height"] == 4 and a.stats()["leaf_used"] == 4096
    seq = keys[20000:26000]
    _run(g, a, b, sa, seq, 500, "run")
    assert_lookup_parity(a, sa, np.concatenate([keys[19990:26010], keys[::97]]))
    # merges never give leaves back; only the rebuild's bulk load does
    assert a.stats()["leaf_used"] < 4096
    _reinsert(a, b, sa, seq[::5], width, seed)
    assert_lookup_parity(a, sa, np.concatenate([keys[19990:26010], keys[::97]]))


def _run_batches(g, a, b, sa, batches, every, tag):
    for i, kk in enumerate(batches):
        want = sa.delete(kk)
        sta = _delete(g, a, kk, True)
        stb = _delete(g, b, kk, False)
        assert np.array_equal(sta, want) and np.array_equal(stb, want), f"{tag}: status differs at batch {i}"
        if i % every == every - 1 or i + 1 == len(batches):
            ea, eb = a.export(), b.export()
            assert len(ea) == len(eb) and np.array_equal(ea, eb), f"{tag}: trees differ after batch {i}"
            assert_lookup_parity(a, sa, kk)
    assert g.tree_device_error(a.h) == g.GT_OK and g.tree_device_error(b.h) == g.GT_OK
    assert a.stats() == b.stats()
    assert_export_parity(a, sa)


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n", [0, 17, 300, 4096, 65536])
def test_small_delete_batches_match_batch_path(width, n):
    """Batches of 2..64 keys: present keys in random order with repeats
    inside a batch, absent keys and the edge keys."""
    import paper_2604_21117_amd as g
    seed = 700 + n + width
    rng = np.random.default_rng(seed)
    keys = key_set(n, width, seed, edges=n > 2)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    top = np.iinfo(keys.dtype).max
    absent = synth.uniform_keys(256, seed + 7, width, purpose=synth.P_INSERT, exclude=keys)
    present = keys[rng.permutation(len(keys))] if len(keys) else absent
    pool = np.concatenate([absent, np.array([0, top, 1, top - 1], dtype=keys.dtype)])
    batches, at = [], 0
    for i in range(60 if n <= 300 else 120):
        B = int(rng.integers(2, 65))
        take = present[at:at + B]
        at = (at + B) % max(len(present), 1)
        kk = np.concatenate([take, pool[rng.integers(0, len(pool), B // 4 + 1)]])
        kk = np.concatenate([kk, kk[rng.integers(0, len(kk), B // 8 + 1)]])[:64]
        batches.append(kk[rng.permutation(len(kk))].astype(keys.dtype))
    _run_batches(g, a, b, sa, batches, 5, f"n={n}")
    _reinsert(a, b, sa, np.unique(np.concatenate(batches)[np.isin(np.concatenate(batches), keys)])[:160], width,
              seed)


@pytest.mark.parametrize("width", [32, 64])
def test_small_delete_batches_of_key_runs(width):
    """Runs of 64 consecutive keys out of 2^16 at fill 1.0 (height 4): each
    batch empties four leaves of one parent, so merges, grandparent merges
    and the host's rebuild come in quick succession; then the whole tree
    goes, 64 keys a batch, down to empty."""
    import paper_2604_21117_amd as g
    seed = 9
    keys = (np.arange(1, 65537, dtype=np.uint64) * 7).astype(np.uint32 if width == 32 else np.uint64)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    a = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    b = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=64)
    runs = [keys[c:c + 64] for c in range(8192, 8192 + 64 * 80, 64)]
    _run_batches(g, a, b, sa, runs, 10, "runs")
    assert a.stats()["leaf_used"] < 4096  # the host rebuilt the tree at least once
    rest = sa.items()[0]
    order = np.random.default_rng(seed).permutation(len(rest))
    _run_batches(g, a, b, sa, [rest[order[c:c + 64]] for c in range(0, len(rest), 64)], 100, "all")
    assert a.stats()["n_keys"] == 0
