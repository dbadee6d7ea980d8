"""Lookups captured into a HIP graph (as the benchmark submits them):
every replay, with eager work and synchronisations between replays, gives
the eager results, which match the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    import torch
    import paper_2604_21117_amd as g
    assert torch.cuda.is_available()
    seed, width, n, B, nb = 61, 64, 1 << 18, 1024, 4
    keys = synth.uniform_keys(n, seed, width)
    vals = synth.values_for(keys, seed, width)
    sa = oracle.SortedArray(keys, vals, width)
    t = mk_tree(keys, vals, 8, max_batch=1 << 14)
    li = g.Learned(t, models=256)
    li.train()
    stream = torch.cuda.Stream()
    qs = [synth.mixed_queries(keys, B, seed + i, width) for i in range(nb)]
    qd = [t.dev(q) for q in qs]
    outs = [(torch.empty(B, dtype=torch.int64, device="cuda"), torch.empty(B, dtype=torch.uint8, device="cuda"))
            for _ in range(2 * nb)]

    def launch():
        for i in range(nb):
            g.tree_lookup_batch(t.h, qd[i], outs[i][0], outs[i][1], stream)
            g.li_lookup_batch(li.h, qd[i], outs[nb + i][0], outs[nb + i][1], stream)

    def read():
        return [(g.to_numpy(v, np.uint64).copy(), g.to_numpy(f).copy()) for v, f in outs]

    with torch.cuda.stream(stream):
        launch()
    stream.synchronize()
    eager = read()
    for i in range(nb):
        ov, of = sa.lookup(qs[i])
        for k in (i, nb + i):
            assert np.array_equal(eager[k][1], of) and np.array_equal(eager[k][0], ov)
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=stream):
        launch()
    extra = t.dev(synth.present_queries(keys, 4096, seed + 99))
    for r in range(4):
        with torch.cuda.stream(stream):
            for v, f in outs:
                v.fill_(-1)
                f.fill_(7)
        t.lookup_dev(extra)  # eager work between replays
        stream.synchronize()
        gr.replay()
        stream.synchronize()
        got = read()
        for k in range(2 * nb):
            assert np.array_equal(got[k][0], eager[k][0]) and np.array_equal(got[k][1], eager[k][1]), \
                f"replay {r}, output {k}"
