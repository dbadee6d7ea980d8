"""GPU parity of insert batches against the oracle: statuses, resulting
content (in-order export == oracle's sorted array), tree invariants after
every batch, lookups afterwards, all bit-exact.  Also the all-or-nothing
capacity error and run-to-run repeatability of the tree layout."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree, assert_lookup_parity, assert_export_parity, assert_range_parity, key_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()


def test_c1_config():
    """2^16 u32 keys, 1024 lookups (half present), 1024 fresh inserts, then
    every key looked up and all invariants checked."""
    seed, width = 1, 32
    keys = synth.uniform_keys(1 << 16, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 4, leaf_slack=4096, max_batch=4096)
    assert_lookup_parity(t, sa, synth.mixed_queries(keys, 1024, seed, width))
    ins = synth.uniform_keys(1024, seed + 1, width, purpose=synth.P_INSERT, exclude=keys)
    iv = synth.values_for(ins, seed + 1, width)
    st = t.insert(ins, iv)
    assert np.array_equal(st, sa.insert(ins, iv))
    assert (st == 0).all()
    assert t.stats()["n_keys"] == (1 << 16) + 1024
    assert_export_parity(t, sa)
    allk = np.concatenate([keys, ins])
    assert_lookup_parity(t, sa, allk)


def _random_batch(rng, pool, B, width):
    """Keys from a pool that mixes present keys, repeats and fresh keys."""
    k = pool[rng.integers(0, len(pool), B)]
    v = rng.integers(0, np.iinfo(np.uint32).max if width == 32 else np.iinfo(np.int64).max, B,
                     dtype=np.uint64).astype(k.dtype)
    return k, v


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n,batches", [(0, [1, 5, 16, 17, 300]), (1, [15, 1, 2]), (17, [40, 1000]),
                                       (5000, [1, 2, 3000, 5000, 700]), (70000, [4096, 1, 2049]),
                                       (3000, [64, 65, 100, 128, 129, 512, 513, 2048])])
def test_insert_sequences(width, n, batches):
    seed = 31 + n
    rng = np.random.default_rng(seed)
    keys = key_set(n, width, seed, edges=n > 2)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=8192, max_batch=8192)
    fresh = synth.uniform_keys(20000, seed + 7, width, exclude=keys)
    top = np.iinfo(keys.dtype).max
    pool = np.concatenate([keys, fresh, np.array([0, top], dtype=keys.dtype)])
    for bi, B in enumerate(batches):
        k, v = _random_batch(rng, pool, B, width)
        st = t.insert(k, v)
        assert np.array_equal(st, sa.insert(k, v)), f"status differs in batch {bi}"
        assert_export_parity(t, sa)
        q = np.concatenate([k[:500], pool[rng.integers(0, len(pool), 500)]])
        assert_lookup_parity(t, sa, q)
    sk = np.sort(sa.keys).astype(keys.dtype)
    if len(sk):
        lo = sk[rng.integers(0, len(sk), 200)]
        span = (rng.integers(0, 1 << 20, 200).astype(np.uint64) << np.uint64(width - 24)).astype(keys.dtype)
        hi = np.where(lo > top - span, top, lo + span).astype(keys.dtype)
        mc = rng.integers(1, 80, 200).astype(np.uint32)
        assert_range_parity(t, sa, lo, hi, mc)


@pytest.mark.parametrize("width", [32, 64])
def test_clustered_overload_grows_root(width):
    """Thousands of new keys inside one leaf's key range: the leaf splits
    into hundreds of pieces and the root grows by several levels."""
    seed = 77
    keys = np.arange(0, 64 * 1000, 1000, dtype=np.uint64).astype(np.uint32 if width == 32 else np.uint64)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=4096, max_batch=8192)
    h0 = t.stats()["height"]
    ins = (np.arange(1, 6001, dtype=np.uint64) + 5000).astype(keys.dtype)  # inside one leaf's range
    iv = synth.values_for(ins, seed, width)
    st = t.insert(ins, iv)
    assert np.array_equal(st, sa.insert(ins, iv))
    assert t.stats()["height"] > h0 + 1
    assert_export_parity(t, sa)
    assert_lookup_parity(t, sa, np.concatenate([ins, keys]))


def test_capacity_error_leaves_tree_unchanged():
    import paper_2604_21117_amd as g
    width, seed = 64, 5
    keys = synth.uniform_keys(20000, seed, width)
    vals = synth.values_for(keys, seed, width)
    p = g.make_params(8, max_batch=2048)
    arena = g.tree_arena_bytes(p, len(keys), 0)  # no room for new leaves
    t = mk_tree(keys, vals, 8, arena_bytes=arena, max_batch=2048)
    before = t.export()
    ins = synth.uniform_keys(2000, seed + 1, width, exclude=keys)
    with pytest.raises(g.GtError) as e:
        t.insert(ins, ins)
    assert e.value.status == g.GT_ERR_CAPACITY
    assert np.array_equal(t.export(), before)
    sa = oracle.SortedArray(keys, vals, width)
    assert_lookup_parity(t, sa, np.concatenate([keys[:1000], ins[:1000]]))
    # updates need no new node and still go through
    st = t.insert(keys[:100], keys[:100])
    assert (st == 1).all()


@pytest.mark.parametrize("B", [1, 40, 100])
def test_capacity_error_small_batches(B):
    """Small batches are planned and applied by their own kernels (one
    workgroup applies up to 64 keys).  A refused batch changes nothing, not
    even the values of the present keys it carries; an update-only batch of
    the same size then goes through."""
    import paper_2604_21117_amd as g
    width, seed = 64, 6
    keys = synth.uniform_keys(20000, seed, width)
    vals = synth.values_for(keys, seed, width)
    p = g.make_params(8, max_batch=2048)
    arena = g.tree_arena_bytes(p, len(keys), 0)  # full leaves, no room for new ones
    t = mk_tree(keys, vals, 8, arena_bytes=arena, max_batch=2048)
    before = t.export()
    fresh = synth.uniform_keys(B, seed + 1, width, exclude=keys)
    ins = np.concatenate([fresh[:B - B // 2], keys[:B // 2]])
    with pytest.raises(g.GtError) as e:
        t.insert(ins, ins)
    assert e.value.status == g.GT_ERR_CAPACITY
    assert np.array_equal(t.export(), before)
    sa = oracle.SortedArray(keys, vals, width)
    upd = keys[1000:1000 + B]
    nv = synth.values_for(upd, seed + 2, width)
    assert np.array_equal(t.insert(upd, nv), sa.insert(upd, nv))
    assert_export_parity(t, sa)


def test_repeatable_layout():
    """The same build and insert batches give byte-identical trees (node
    allocation follows a scan in key order, not atomics)."""
    width, seed = 64, 13
    keys = synth.uniform_keys(100000, seed, width)
    vals = synth.values_for(keys, seed, width)
    batches = [synth.uniform_keys(B, seed + 10 + B, width, exclude=keys) for B in (1000, 5000, 1)]
    exports = []
    for lanes, lds in ((16, 3), (4, 1)):
        t = mk_tree(keys, vals, 8, leaf_slack=20000, max_batch=8192, lanes_per_query=lanes, lds_levels=lds)
        for b in batches:
            t.insert(b, b)
        exports.append(t.export())
    assert np.array_equal(exports[0], exports[1])


def test_large_batch_radix_path():
    """B = 2^17 into 2^20 keys (device-wide radix sort, thousands of
    touched leaves per level)."""
    width, seed = 64, 21
    keys = synth.uniform_keys(1 << 20, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 16, max_batch=1 << 17)
    rng = np.random.default_rng(seed)
    fresh = synth.uniform_keys(1 << 17, seed + 1, width, exclude=keys)
    k = np.concatenate([fresh[: (1 << 17) - 5000], keys[rng.integers(0, len(keys), 5000)]])
    k = synth.shuffle(k, seed)
    v = synth.values_for(k, seed + 3, width)
    st = t.insert(k, v)
    assert np.array_equal(st, sa.insert(k, v))
    assert_export_parity(t, sa)
    assert_lookup_parity(t, sa, k[:200000])


@pytest.mark.parametrize("width", [32, 64])
def test_radix_path_repeats_last_writer_wins(width):
    """Batches above the rank-sort limit go through the device radix sort,
    whose tiles find their output offsets by look-back over earlier tiles.
    Heavy in-batch repeats in shuffled order (a few hundred keys, each dozens
    of times, half of them already present) make the last occurrence's value
    win only if the sort keeps equal keys in batch order; small-range keys
    leave every upper digit zero, so one digit's run spans every tile."""
    seed = 23
    keys = synth.uniform_keys(1 << 14, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=1 << 13, max_batch=1 << 16)
    rng = np.random.default_rng(seed)
    dt = keys.dtype
    for B in (2049, 6151, 40000):
        fresh = synth.uniform_keys(300, seed + B, width, exclude=keys)
        k = np.concatenate([fresh[rng.integers(0, 300, B // 2)], keys[rng.integers(0, 300, B - B // 2)]])
        k = k.astype(dt)
        v = rng.integers(0, np.iinfo(dt).max, B, dtype=dt, endpoint=True)
        assert np.array_equal(t.insert(k, v), sa.insert(k, v)), f"statuses, B={B}"
        assert_export_parity(t, sa)
    small = np.arange(1, 9000, 3, dtype=dt)
    k = small[rng.integers(0, len(small), 30000)]
    v = rng.integers(0, np.iinfo(dt).max, len(k), dtype=dt, endpoint=True)
    assert np.array_equal(t.insert(k, v), sa.insert(k, v)), "statuses, small-range keys"
    assert_export_parity(t, sa)
    assert_lookup_parity(t, sa, np.concatenate([small, keys[:5000]]))


@pytest.mark.parametrize("xcd", [0, 1])
def test_mirror_follows_top_levels(xcd):
    """Height-5 tree (2^20 u64 keys), three mirrored inner levels staged in
    LDS.  Sparse batches split leaves only, so the mirrored levels stay as
    they are; clustered batches split level-3 nodes and rewrite mirrored
    level-2 nodes.  Lookups through the mirror (and the XCD splitters taken
    from it) match the oracle after every batch."""
    width, seed = 64, 41
    keys = synth.uniform_keys(1 << 20, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 15, max_batch=4096, lds_levels=3, xcd_split=xcd)
    assert t.stats()["height"] == 5
    rng = np.random.default_rng(seed)
    sk = np.sort(keys)
    fresh = synth.uniform_keys(1 << 15, seed + 3, width, exclude=keys)
    for bi in range(8):
        if bi % 2 == 0:
            k = fresh[bi * 1024:(bi + 1) * 1024]
        else:
            j = int(rng.integers(0, len(sk) - 5000))
            lo, hi = int(sk[j]), int(sk[j + 4000])
            k = np.unique(rng.integers(lo, hi, 3000, dtype=np.uint64))
            k = synth.shuffle(k, seed + bi)
        v = synth.values_for(k, seed + 100 + bi, width)
        st = t.insert(k, v)
        assert np.array_equal(st, sa.insert(k, v)), f"status differs in batch {bi}"
        q = np.concatenate([k, keys[rng.integers(0, len(keys), (1 << 15) - len(k) - 4096)],
                            fresh[-4096:]])
        assert_lookup_parity(t, sa, q)
    assert_export_parity(t, sa)
