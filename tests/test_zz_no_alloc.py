"""The level-wise lookup that allocates nothing (its workspace is a fixed
device array inside the library) against the workspace entry point and the
oracle, through the C ABI: two calls in a row, the second with a smaller
batch, on both sort paths, presorted batches and both key widths; a batch
whose workspace would not fit the array is refused with nothing written."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree, key_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_21117_amd as g
    g.lib()


def _both(t, q, presorted):
    """Results of the allocation-free call and of the workspace call on the
    same device batch."""
    import torch
    import paper_2604_21117_amd as g
    qd = t.dev(q)
    flags = g.GT_LW_PRESORTED if presorted else 0
    va = torch.empty(len(q), dtype=t.tdtype, device=t.device)
    fa = torch.empty(len(q), dtype=torch.uint8, device=t.device)
    g.tree_lookup_levelwise_noalloc(t.h, qd, flags, va, fa)
    vb, fb = t.lookup_levelwise_dev(qd, presorted)
    torch.cuda.synchronize()
    return (g.to_numpy(va, t.udtype), g.to_numpy(fa)), (g.to_numpy(vb, t.udtype), g.to_numpy(fb))


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("sizes", [(5000, 300), (2048, 2047), (70000, 3000), (1000, 1)])
def test_noalloc_matches_workspace_call(width, sizes):
    seed = 4242 + sizes[0]
    keys = key_set(60000, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    for presorted in (False, True):
        for B in sizes:   # second call smaller than the first
            q = synth.mixed_queries(keys, B, seed + B, width)
            if presorted:
                q = np.sort(q)
            (va, fa), (vb, fb) = _both(t, q, presorted)
            ov, of = sa.lookup(q)
            tag = f"width={width} B={B} presorted={presorted}"
            assert np.array_equal(fa, fb) and np.array_equal(va, vb), tag + ": differs from the workspace call"
            assert np.array_equal(fa, of) and np.array_equal(va, ov), tag + ": differs from the oracle"


def test_noalloc_largest_batches_and_refusal():
    """The largest documented batches fit (8-byte keys: 2^18 sorted by the
    library, 2^20 presorted); one that needs more scratch is refused with
    GT_ERR_CAPACITY and leaves the outputs untouched; a smaller call after
    both still answers right."""
    import torch
    import paper_2604_21117_amd as g
    seed = 99
    keys = key_set(1 << 17, 64, seed)
    vals = synth.values_for(keys, seed, 64)
    sa = oracle.SortedArray(keys, vals, 64)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    cap = g.GT_LW_NOALLOC_SCRATCH_BYTES
    for B, presorted in (((1 << 18), False), ((1 << 20), True)):
        flags = g.GT_LW_PRESORTED if presorted else 0
        assert g.tree_lookup_levelwise_workspace_bytes(t.h, B, flags) <= cap
        q = synth.mixed_queries(keys, B, seed + B, 64)
        if presorted:
            q = np.sort(q)
        (va, fa), (vb, fb) = _both(t, q, presorted)
        ov, of = sa.lookup(q)
        assert np.array_equal(fa, of) and np.array_equal(va, ov), f"B={B}"
        assert np.array_equal(fa, fb) and np.array_equal(va, vb), f"B={B}"
    B = 1 << 19
    assert g.tree_lookup_levelwise_workspace_bytes(t.h, B, 0) > cap
    qd = t.dev(synth.present_queries(keys, B, seed))
    vo = torch.full((B,), 7, dtype=torch.int64, device=t.device)
    fo = torch.full((B,), 9, dtype=torch.uint8, device=t.device)
    rc = g.lib().tree_lookup_levelwise_noalloc(t.h, g._ptr(qd), B, 0, g._ptr(vo), g._ptr(fo), None)
    assert rc == g.GT_ERR_CAPACITY
    torch.cuda.synchronize()
    assert (g.to_numpy(fo) == 9).all() and (g.to_numpy(vo) == 7).all()
    q = synth.mixed_queries(keys, 777, seed, 64)
    (va, fa), _ = _both(t, q, False)
    ov, of = sa.lookup(q)
    assert np.array_equal(fa, of) and np.array_equal(va, ov)


def test_noalloc_argument_errors():
    import torch
    import paper_2604_21117_amd as g
    keys = key_set(100, 64, 5)
    t = mk_tree(keys, synth.values_for(keys, 5, 64), 8)
    qd = t.dev(keys)
    vo = torch.empty(100, dtype=torch.int64, device=t.device)
    fo = torch.empty(100, dtype=torch.uint8, device=t.device)
    L = g.lib()
    assert L.tree_lookup_levelwise_noalloc(None, g._ptr(qd), 100, 0, g._ptr(vo), g._ptr(fo), None) == g.GT_ERR_INVALID
    assert L.tree_lookup_levelwise_noalloc(t.h, g._ptr(qd), 100, 2, g._ptr(vo), g._ptr(fo), None) == g.GT_ERR_INVALID
    assert L.tree_lookup_levelwise_noalloc(t.h, None, 100, 0, g._ptr(vo), g._ptr(fo), None) == g.GT_ERR_INVALID
    assert L.tree_lookup_levelwise_noalloc(t.h, g._ptr(qd), 0, 0, None, None, None) == g.GT_OK
