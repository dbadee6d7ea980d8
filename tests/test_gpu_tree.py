"""GPU parity of build, lookup and range against the oracle (bit-exact),
through the C ABI.  Tree shapes span one leaf, ragged leaf/inner tails,
several tiles of queries, both key widths and every launch configuration."""
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
    import paper_2604_21117_amd as g
    g.lib()


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n", [0, 1, 2, 15, 16, 17, 255, 256, 257, 4109, 65536])
def test_build_lookup_sizes(width, n):
    seed = 100 + n
    keys = key_set(n, width, seed, edges=(n % 2 == 1))
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    st = t.stats()
    assert st["n_keys"] == n
    assert_export_parity(t, sa)
    B = 1000
    q = np.concatenate([synth.present_queries(keys, B // 2, seed) if n else np.zeros(0, keys.dtype),
                        synth.absent_queries(keys, B // 2, seed, width),
                        np.array([0, np.iinfo(keys.dtype).max, 1], dtype=keys.dtype)])
    q = synth.shuffle(q, seed)
    assert_lookup_parity(t, sa, q)


def test_c1_closed_form_node_count():
    """2^16 keys at fill 1.0: 4096 leaves, 273 inner nodes, height 4
    (Section III: sum_{i<h} 16^i = 4369 nodes)."""
    keys = synth.uniform_keys(1 << 16, 1, 32)
    vals = synth.values_for(keys, 1, 32)
    t = mk_tree(keys, vals, 4, max_batch=4096)
    st = t.stats()
    assert st["height"] == 4 and st["leaf_used"] == 4096 and st["inner_used"] == 273


@pytest.mark.parametrize("lanes", [4, 8, 16])
@pytest.mark.parametrize("qpg", [1, 2, 4])
@pytest.mark.parametrize("lds", [1, 2, 3, 4])
@pytest.mark.parametrize("vc", [1, 2])
def test_launch_configs_agree(lanes, qpg, lds, vc):
    width, seed = 64, 7
    keys = key_set(70000, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=4096, lanes_per_query=lanes, queries_per_group=qpg, lds_levels=lds,
                value_coload=vc)
    q = synth.mixed_queries(keys, 5003, seed, width)
    q[:2] = [0, np.iinfo(np.uint64).max]
    assert_lookup_parity(t, sa, q)
    lo, hi, mc = synth.range_starts_and_lengths(keys, 777, seed, 60)
    hi = np.minimum(lo.astype(np.uint64) + np.uint64(1 << 52), np.iinfo(np.uint64).max).astype(np.uint64)
    assert_range_parity(t, sa, lo, hi, mc)


@pytest.mark.parametrize("width", [32, 64])
def test_range_edge_cases(width):
    seed = 9
    keys = key_set(3000, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    top = np.iinfo(keys.dtype).max
    sk = np.sort(keys)
    lo = np.array([0, 0, top, sk[5], sk[100], sk[100], 7, sk[-1], sk[50] + 1], dtype=keys.dtype)
    hi = np.array([top, 0, top, sk[5], sk[99], sk[400], 6, top, sk[60]], dtype=keys.dtype)
    mc = np.array([100, 3, 3, 1, 10, 500, 4, 2, 0], dtype=np.uint32)
    assert_range_parity(t, sa, lo, hi, mc)
    lo2, hi2, mc2 = synth.range_starts_and_lengths(keys, 4000, seed, 100)
    assert_range_parity(t, sa, lo2, hi2, mc2)


def test_duplicate_build_keys_rejected():
    import paper_2604_21117_amd as g
    keys = np.array([5, 9, 5, 11], dtype=np.uint64)
    with pytest.raises(g.GtError) as e:
        mk_tree(keys, keys, 8, max_batch=1024)
    assert e.value.status == g.GT_ERR_DUPLICATE


def test_duplicate_queries_and_all_present():
    width, seed = 64, 11
    keys = key_set(50000, width, seed)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    q = np.repeat(keys[:100], 7)
    assert_lookup_parity(t, sa, q)
    assert_lookup_parity(t, sa, keys)          # every key once
    gv, gf = t.lookup(keys)
    assert gf.all() and np.array_equal(gv, synth.values_for(keys, seed, width))


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n", [5, 300, 3000, 200000])
@pytest.mark.parametrize("xcd,stream", [(1, 2), (1, 1), (1, 0), (2, 2), (2, 0), (2, 1)])
def test_large_batch_paths(width, n, xcd, stream):
    """Batches above the XCD-split threshold (2^15): the split and the plain
    kernel, with streaming loads of both leaf lines, of the value line only
    (the default) or of neither, agree bit for bit with the oracle, for
    trees with and without splitter keys."""
    seed = 50 + n
    keys = key_set(n, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096, xcd_split=xcd, leaf_stream=stream)
    q = synth.mixed_queries(keys, 70001, seed, width)
    q[:3] = [0, np.iinfo(keys.dtype).max, keys[0]]
    assert_lookup_parity(t, sa, q)


@pytest.mark.parametrize("width", [32, 64])
def test_default_shapes_across_batch_sizes(width):
    """With the shape left to the library, lookups switch lanes per query,
    queries per group and LDS staging at 2^13 and 2^15 queries; batches on
    both sides of each switch (and ragged tails) match the oracle, present
    and absent keys, learned index included."""
    import paper_2604_21117_amd as g
    seed = 71
    keys = key_set(1 << 18, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    li = g.Learned(t, models=256)
    li.train()
    for B in (1, 63, (1 << 13) - 1, 1 << 13, (1 << 13) + 1, (1 << 15) - 1, 1 << 15, (1 << 15) + 17):
        q = synth.mixed_queries(keys, B, seed + B, width)
        assert_lookup_parity(t, sa, q)
        gv, gf = li.lookup(q)
        ov, of = sa.lookup(q)
        assert np.array_equal(gf, of) and np.array_equal(gv, ov), f"learned, B={B}"


@pytest.mark.parametrize("width", [32, 64])
def test_dense_runs_and_huge_gaps(width):
    """Lookups on a key set of dense runs of consecutive keys and a few huge
    gaps (nodes whose separators are a few units apart beside nodes that span
    half the key space), both edge values, and absent keys on both sides of
    every present one; batches on both sides of the large-batch shape
    switch."""
    top = (1 << width) - 1
    rng = np.random.default_rng(7 + width)
    dense = np.arange(1, 30000, dtype=np.uint64)
    far = np.array([top // 3, top // 3 + 1, top // 2, top - 1, top], dtype=np.uint64)
    mid = (np.uint64(1) << np.uint64(width - 8)) + rng.integers(0, 1 << 20, 20000).astype(np.uint64)
    keys = np.unique(np.concatenate([dense, far, mid])).astype(np.uint32 if width == 32 else np.uint64)
    keys = synth.shuffle(keys, 3)
    vals = synth.values_for(keys, 9, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    sk = np.sort(keys)
    q = np.concatenate([sk, sk - 1, sk + 1, np.array([0], dtype=sk.dtype)]).astype(sk.dtype)
    q = q[rng.permutation(len(q))]
    assert_lookup_parity(t, sa, q)
    assert_lookup_parity(t, sa, q[:1000])
