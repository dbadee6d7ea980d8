"""The failure path of the device radix sort (inputs above 2048 keys),
forced from the host through the testing hook that sets its look-back
limit: at 0 every workgroup of a pass but the first gives up at once, so
every kernel still ends normally.  A failed sort must surface as an error,
never as a wrong answer reported as good: the bulk load returns
GT_ERR_DEVICE, an insert or delete batch is refused with the tree
unchanged, a level-wise lookup sets the internal bit of the error word.  Sorts that need
no look-back (batches up to 4096 keys, one tile) are unaffected, and with
the limit restored every path is exact again."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree, key_set

pytestmark = pytest.mark.gpu


@pytest.fixture()
def g():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_21117_amd as g
    g.lib()
    old = g.set_sort_spin_limit(1 << 20)
    assert old == 1 << 20, "the default limit"
    yield g
    g.set_sort_spin_limit(old)


def _batch(keys, B, seed, width):
    """B keys: half fresh, half present (updates), shuffled."""
    fresh = synth.uniform_keys(B - B // 2, seed, width, exclude=keys)
    rng = np.random.default_rng(seed)
    present = keys[rng.choice(len(keys), B // 2, replace=False)]
    k = synth.shuffle(np.concatenate([fresh, present]), seed)
    return k, synth.values_for(k, seed + 1, width)


@pytest.mark.parametrize("width", [32, 64])
def test_forced_sort_failure_is_reported_and_harmless(g, width):
    seed = 4100 + width
    keys = key_set(30000, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=1 << 12, max_batch=1 << 14)
    before = t.export().copy()

    g.set_sort_spin_limit(0)
    try:
        # bulk load above one tile: the sort fails, the build reports it
        with pytest.raises(g.GtError) as e:
            mk_tree(keys, vals, width // 8)
        assert e.value.status == g.GT_ERR_DEVICE
        # insert above one tile: refused, tree byte for byte unchanged
        k, v = _batch(keys, 9000, seed + 1, width)
        with pytest.raises(g.GtError) as e:
            t.insert(k, v)
        assert e.value.status == g.GT_ERR_DEVICE
        assert np.array_equal(t.export(), before), "a refused batch changed the tree"
        assert g.tree_device_error(t.h) == g.GT_OK, "reading the word clears it"
        # delete above one tile: refused too
        with pytest.raises(g.GtError) as e:
            t.delete(synth.shuffle(keys[:9000], seed))
        assert e.value.status == g.GT_ERR_DEVICE
        assert np.array_equal(t.export(), before), "a refused delete changed the tree"
        # level-wise lookup above one tile: the internal bit is set
        q = synth.mixed_queries(keys, 9000, seed + 2, width)
        t.lookup_levelwise(q)
        assert g.tree_device_error(t.h) == g.GT_ERR_DEVICE
        assert g.tree_device_error(t.h) == g.GT_OK
        # one tile (no look-back) and the small paths are unaffected
        for B in (100, 2048, 3000, 4096):
            q = synth.mixed_queries(keys, B, seed + B, width)
            gv, gf = t.lookup_levelwise(q)
            ov, of = sa.lookup(q)
            assert np.array_equal(gf, of) and np.array_equal(gv, ov), f"level-wise B={B}"
            assert g.tree_device_error(t.h) == g.GT_OK
        k, v = _batch(keys, 3000, seed + 3, width)
        st = t.insert(k, v)
        ost = sa.insert(k, v)
        assert np.array_equal(st, ost)
    finally:
        g.set_sort_spin_limit(1 << 20)

    # restored: the large paths are exact again
    t2 = mk_tree(keys, vals, width // 8, leaf_slack=1 << 12, max_batch=1 << 14)
    for tree in (t, t2):
        if tree is t2:
            sa2 = oracle.SortedArray(keys, vals, width)
        else:
            sa2 = sa
        k, v = _batch(sa2.items()[0], 9000, seed + 4, width)
        st = tree.insert(k, v)
        assert np.array_equal(st, sa2.insert(k, v))
        q = synth.mixed_queries(sa2.items()[0], 9000, seed + 5, width)
        gv, gf = tree.lookup_levelwise(q)
        ov, of = sa2.lookup(q)
        assert np.array_equal(gf, of) and np.array_equal(gv, ov)
        bits, ek, ev = oracle.check_export(tree.export(), len(sa2))
        assert bits == 0 and np.array_equal(ek, sa2.keys) and np.array_equal(ev, sa2.vals)
        assert g.tree_device_error(tree.h) == g.GT_OK
    t2.close()
    t.close()
