"""GPU parity of the level-wise lookup (paper Sections IV-A and IV-F)
against the oracle, bit for bit, through the C ABI: library-sorted and
caller-sorted batches, both key widths, trees from one leaf to several
levels, trees grown by inserts (rewritten nodes, a taller root), both sort
paths (rank sort up to 2048 queries, radix sort above), duplicates, edge
keys, and graph replays."""
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


def _check(t, sa, q, presorted=False, tag=""):
    gv, gf = t.lookup_levelwise(q, presorted=presorted)
    ov, of = sa.lookup(q)
    assert np.array_equal(gf, of), f"{tag}: found flags differ at {np.nonzero(gf != of)[0][:8]}"
    assert np.array_equal(gv, ov), f"{tag}: values differ at {np.nonzero(gv != ov)[0][:8]}"


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("n", [0, 1, 16, 17, 257, 4109, 70000])
def test_levelwise_sizes(width, n):
    seed = 900 + n
    keys = key_set(n, width, seed, edges=(n % 2 == 1))
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    top = np.iinfo(keys.dtype).max
    for B in (1, 5, 64, 65, 1000, 2048, 2049, 5000):
        q = synth.mixed_queries(keys, B, seed + B, width) if n else synth.absent_queries(keys, B, seed, width)
        q[: min(B, 3)] = np.array([0, top, 1], dtype=keys.dtype)[: min(B, 3)]
        _check(t, sa, q, False, f"n={n} B={B} sorted here")
        _check(t, sa, np.sort(q), True, f"n={n} B={B} presorted")


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_unsorted_input_flagged_presorted(width):
    """A batch passed as presorted that is not in order still gets correct
    results (the runs are only shorter)."""
    seed = 77
    keys = key_set(20000, width, seed)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    for B in (100, 3000, 40000):
        q = synth.mixed_queries(keys, B, seed + B, width)
        _check(t, sa, q, True, f"B={B} unsorted, flagged presorted")
        _check(t, sa, q[::-1].copy(), True, f"B={B} descending, flagged presorted")


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_duplicates_and_zipf(width):
    seed = 78
    keys = key_set(1 << 16, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    z = synth.Zipf(len(keys), 0.99, seed)
    for B in (1024, 1 << 16):
        q = keys[z.indices(B)]
        _check(t, sa, q, False, f"zipf B={B}")
        _check(t, sa, np.sort(q), True, f"zipf B={B} presorted")
    q = np.repeat(keys[:7], 300)
    _check(t, sa, synth.shuffle(q, seed), False, "seven keys repeated")
    _check(t, sa, q, True, "seven keys repeated, presorted")


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_after_inserts(width):
    """Inserts rewrite inner nodes (their child references come from the
    child line) and grow the root; the host's launch count follows a bound
    on the height, and lookups stay exact."""
    seed = 79
    keys = key_set(300, width, seed)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, leaf_slack=1 << 14, max_batch=4096)
    h0 = t.stats()["height"]
    for b in range(6):
        nk = synth.uniform_keys(4000, seed + 10 + b, width)
        nv = synth.values_for(nk, seed + 20 + b, width)
        t.insert(nk, nv)
        sa.insert(nk, nv)
        allk, _ = sa.items()
        q = synth.mixed_queries(allk, 3000, seed + b, width)
        _check(t, sa, q, False, f"after insert batch {b}")
        _check(t, sa, np.sort(q), True, f"after insert batch {b}, presorted")
    assert t.stats()["height"] > h0


@pytest.mark.parametrize("width", [32, 64])
def test_levelwise_library_sort_degenerate_digits(width):
    """Batches above 2048 keys are sorted by the device radix sort; here every
    key is equal (each pass puts every element in one digit, so every tile's
    look-back sums one digit over all earlier tiles), or keys differ only in
    the top byte, or only in the low byte."""
    seed = 82
    keys = key_set(20000, width, seed, edges=True)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, width // 8, max_batch=4096)
    dt = keys.dtype
    rng = np.random.default_rng(seed)
    B = 40000
    same = np.full(B, keys[123], dtype=dt)
    _check(t, sa, same, False, "all keys equal")
    hi = (rng.integers(0, 256, B).astype(np.uint64) << np.uint64(width - 8)).astype(dt)
    _check(t, sa, hi, False, "top byte only")
    lo = np.concatenate([keys[rng.integers(0, len(keys), B // 2)],
                         (rng.integers(0, 256, B - B // 2)).astype(dt)])
    _check(t, sa, synth.shuffle(lo, seed), False, "present keys and low-byte keys")


def test_levelwise_workspace_and_errors():
    import torch
    import paper_2604_21117_amd as g
    keys = key_set(5000, 64, 80)
    vals = synth.values_for(keys, 80, 64)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    q = t.dev(synth.mixed_queries(keys, 3000, 80, 64))
    need = g.tree_lookup_levelwise_workspace_bytes(t.h, 3000, 0)
    need_p = g.tree_lookup_levelwise_workspace_bytes(t.h, 3000, g.GT_LW_PRESORTED)
    assert need > need_p > 0
    assert g.tree_lookup_levelwise_workspace_bytes(t.h, 3000, 2) == 0
    vo = torch.empty(3000, dtype=torch.int64, device="cuda")
    fo = torch.empty(3000, dtype=torch.uint8, device="cuda")
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    st = g.lib().tree_lookup_levelwise(t.h, g._ptr(q), 3000, 0, g._ptr(vo), g._ptr(fo), g._ptr(small),
                                       need - 1, None)
    assert st == g.GT_ERR_CAPACITY
    st = g.lib().tree_lookup_levelwise(t.h, g._ptr(q), 3000, 4, g._ptr(vo), g._ptr(fo), g._ptr(small),
                                       need - 1, None)
    assert st == g.GT_ERR_INVALID
    assert g.lib().tree_lookup_levelwise(t.h, g._ptr(q), 0, 0, None, None, None, 0, None) == g.GT_OK
    # a workspace full of garbage gives the same results (contents ignored)
    ws = torch.full((need,), 0xA5, dtype=torch.uint8, device="cuda")
    g.tree_lookup_levelwise(t.h, q, 0, vo, fo, ws)
    sa = oracle.SortedArray(keys, vals, 64)
    ov, of = sa.lookup(g.to_numpy(q, np.uint64))
    assert np.array_equal(g.to_numpy(fo), of) and np.array_equal(g.to_numpy(vo, np.uint64), ov)


def test_levelwise_graph_replays():
    """Captured into a HIP graph (both sort paths and the presorted path),
    every replay, with eager work between replays, gives the eager results."""
    import torch
    import paper_2604_21117_amd as g
    seed, width = 81, 64
    keys = key_set(1 << 17, width, seed)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=4096)
    stream = torch.cuda.Stream()
    cases = []
    for B, pre in ((1000, False), (9000, False), (9000, True)):
        q = synth.mixed_queries(keys, B, seed + B, width)
        if pre:
            q = np.sort(q)
        cases.append((q, t.dev(q), pre, t.levelwise_workspace(B, pre),
                      torch.empty(B, dtype=torch.int64, device="cuda"),
                      torch.empty(B, dtype=torch.uint8, device="cuda")))

    def launch():
        for q, qd, pre, ws, vo, fo in cases:
            g.tree_lookup_levelwise(t.h, qd, g.GT_LW_PRESORTED if pre else 0, vo, fo, ws, stream)

    with torch.cuda.stream(stream):
        launch()
    stream.synchronize()
    for q, qd, pre, ws, vo, fo in cases:
        ov, of = sa.lookup(q)
        assert np.array_equal(g.to_numpy(fo), of) and np.array_equal(g.to_numpy(vo, np.uint64), ov)
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=stream):
        launch()
    extra = t.dev(synth.present_queries(keys, 4096, seed + 99))
    for r in range(4):
        with torch.cuda.stream(stream):
            for q, qd, pre, ws, vo, fo in cases:
                vo.fill_(-1)
                fo.fill_(7)
                ws.fill_(0x5A)
        t.lookup_levelwise_dev(extra)  # eager work between replays
        stream.synchronize()
        gr.replay()
        stream.synchronize()
        for i, (q, qd, pre, ws, vo, fo) in enumerate(cases):
            ov, of = sa.lookup(q)
            assert np.array_equal(g.to_numpy(fo), of) and np.array_equal(g.to_numpy(vo, np.uint64), ov), \
                f"replay {r}, case {i}"
