"""Serving runtime: a mix of lookup / insert / range / delete batches admitted while
others run gives, for every batch, exactly the result of applying the
batches one at a time in admission order (checked against the oracle and
against the same batches run alone); graphs and direct launches agree;
admission refuses what can never fit and never deadlocks."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import mk_tree

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()


def _batches(spec):
    import paper_2604_21117_amd as g
    return [g.Batch(op, k, v, m, a) for (op, k, v, m, a) in spec]


def _oracle_replay(sa, batches):
    """Sequential application in submission order; returns expected outputs."""
    exp = []
    for b in batches:
        if b.op == 0:
            exp.append(sa.lookup(b.keys))
        elif b.op == 1:
            exp.append((sa.insert(b.keys, b.values),))
        elif b.op == 3:
            exp.append((sa.delete(b.keys),))
        else:
            exp.append(sa.range(b.keys, b.values, b.max_out))
    return exp


def _compare(batches, exp):
    for i, (b, e) in enumerate(zip(batches, exp)):
        if b.op == 0:
            assert np.array_equal(b.out1, e[1]) and np.array_equal(b.out0, e[0]), f"lookup batch {i}"
        elif b.op in (1, 3):
            assert np.array_equal(b.out0, e[0]), f"{'insert' if b.op == 1 else 'delete'} batch {i}"
        else:
            cnt, off, ok, ov = e
            assert np.array_equal(b.count, cnt), f"range batch {i} counts"
            for q in range(len(cnt)):
                s = slice(int(off[q]), int(off[q] + cnt[q]))
                assert np.array_equal(b.out0[s], ok[s]) and np.array_equal(b.out1[s], ov[s]), f"range {i}/{q}"


def _setup(seed, n=1 << 16, width=64):
    keys = synth.uniform_keys(n, seed, width)
    vals = synth.values_for(keys, seed, width)
    fresh = synth.uniform_keys(200000, seed + 1, width, exclude=keys)
    return keys, vals, fresh


@pytest.mark.parametrize("graphs", [1, 2])
def test_mix_equals_sequential(graphs):
    import paper_2604_21117_amd as g
    seed = 60 + graphs
    keys, vals, fresh = _setup(seed)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 15, max_batch=1024)
    srv = g.Server(t, use_graphs=graphs, slots=8, read_streams=4, max_range=128)
    spec = synth.serving_mix(keys, 800, seed, bmax=300, rate=40000.0, zipf=synth.Zipf(len(keys), 0.99, seed),
                             fresh=fresh)
    # a few batches with duplicates and updates of present keys
    spec.append((1, np.concatenate([keys[:50], keys[:50]]), np.arange(100, dtype=np.uint64), None, spec[-1][4]))
    batches = _batches(spec)
    assert srv.replay(batches) == g.GT_OK
    sa = oracle.SortedArray(keys, vals, 64)
    _compare(batches, _oracle_replay(sa, batches))
    st = srv.stats()
    assert sum(st["done"]) == len(batches) and st["refused"] == 0
    assert st["p99_us"] >= st["p50_us"] > 0
    # device intervals from timing events: some work, and no more than the
    # wall time (the union of intervals, not their sum)
    assert 0.0 < st["busy_frac"] <= 1.05
    if graphs == 1:
        assert st["graph_launches"] >= len(batches)
    srv.close()
    bits, ek, ev = oracle.check_export(t.export(), len(sa))
    assert bits == 0 and np.array_equal(ek, sa.keys) and np.array_equal(ev, sa.vals)


@pytest.mark.parametrize("graphs,learned", [(1, False), (2, False), (1, True)])
def test_mix_with_deletes_equals_sequential(graphs, learned):
    """Every tenth batch of the mix becomes a delete of present (and some
    absent, some repeated) keys: reads and writes still see exactly the
    batches admitted before them; a learned index answers through the tree
    after a delete until the server retrains it."""
    import paper_2604_21117_amd as g
    seed = 70 + graphs + (10 if learned else 0)
    keys, vals, fresh = _setup(seed)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 15, max_batch=1024)
    li = None
    if learned:
        li = g.Learned(t, models=256)
        li.train()
    srv = g.Server(t, li, use_graphs=graphs, slots=8, read_streams=4, max_range=128,
                   retrain_log2=14 if learned else 0)
    spec = synth.serving_mix(keys, 600, seed, bmax=300, rate=40000.0, zipf=synth.Zipf(len(keys), 0.99, seed),
                             fresh=fresh)
    rng = np.random.default_rng(seed)
    pool = np.concatenate([keys, fresh[:20000]])
    for i in range(5, len(spec), 10):
        B = int(rng.integers(1, 300))
        dk = pool[rng.integers(0, len(pool), B)]
        if B > 4:
            dk[:2] = dk[2]  # repeated in the batch
        spec[i] = (3, dk, None, None, spec[i][4])
    batches = _batches(spec)
    assert srv.replay(batches) == g.GT_OK
    sa = oracle.SortedArray(keys, vals, 64)
    _compare(batches, _oracle_replay(sa, batches))
    st = srv.stats()
    assert sum(st["done"]) == len(batches) and st["refused"] == 0 and st["done"][3] == len(range(5, len(spec), 10))
    if graphs == 1:
        assert st["direct_launches"] >= st["done"][3]  # deletes are never captured
    srv.close()
    bits, ek, ev = oracle.check_export(t.export(), len(sa))
    assert bits == 0 and np.array_equal(ek, sa.keys) and np.array_equal(ev, sa.vals)
    if li is not None:
        q = synth.mixed_queries(sa.items()[0], 4000, seed, 64)
        ov, of = sa.lookup(q)
        lv, lf = li.lookup(q)
        assert np.array_equal(lf, of) and np.array_equal(lv, ov)
        li.close()
    t.close()


def test_alone_equals_in_mix():
    import paper_2604_21117_amd as g
    seed = 70
    keys, vals, fresh = _setup(seed)
    spec = synth.serving_mix(keys, 300, seed, bmax=200, rate=None, fresh=fresh)
    outs = []
    for mode in ("mix", "alone"):
        t = mk_tree(keys, vals, 8, leaf_slack=1 << 15, max_batch=1024)
        srv = g.Server(t, slots=8)
        batches = _batches(spec)
        if mode == "mix":
            assert srv.replay(batches) == g.GT_OK
        else:
            for b in batches:
                assert srv.wait(srv.submit(b)) == g.GT_OK
        outs.append(batches)
        srv.close()
    for i, (a, b) in enumerate(zip(*outs)):
        if a.op == 2:
            # a range query's slot is defined only up to its count
            assert np.array_equal(a.count, b.count), f"range batch {i} counts"
            off = np.concatenate([[0], np.cumsum(a.max_out.astype(np.int64))[:-1]])
            for q in range(len(a.count)):
                s = slice(int(off[q]), int(off[q] + a.count[q]))
                assert np.array_equal(a.out0[s], b.out0[s]) and np.array_equal(a.out1[s], b.out1[s]), \
                    f"range batch {i}, query {q}"
        else:
            assert np.array_equal(a.out0, b.out0), f"batch {i}"
            if a.out1 is not None:
                assert np.array_equal(a.out1, b.out1), f"batch {i}"


def test_learned_lookups_in_server():
    import paper_2604_21117_amd as g
    seed = 71
    keys, vals, fresh = _setup(seed, n=1 << 17)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 15, max_batch=1024)
    li = g.Learned(t, models=256)
    li.train()
    srv = g.Server(t, learned=li, slots=8)
    spec = synth.serving_mix(keys, 400, seed, bmax=512, rate=50000.0, fresh=fresh)
    batches = _batches(spec)
    assert srv.replay(batches) == g.GT_OK
    _compare(batches, _oracle_replay(oracle.SortedArray(keys, vals, 64), batches))
    srv.close()


def test_server_recaptures_after_learned_changes():
    """The server caches a graph per lookup bucket; overwriting the learned
    index's bounds (the tree unchanged) or retraining it changes what a
    lookup launch must be, so the same bucket afterwards still matches the
    oracle (a stale graph would take the narrowed windows as exact and report
    present keys absent)."""
    import paper_2604_21117_amd as g
    seed = 73
    keys, vals, fresh = _setup(seed, n=1 << 16)
    sa = oracle.SortedArray(keys, vals, 64)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 14, max_batch=1024)
    li = g.Learned(t, models=128)
    li.train()
    srv = g.Server(t, learned=li, slots=2)
    q = synth.present_queries(keys, 512, seed)

    def run():
        b = g.Batch(0, q)
        assert srv.wait(srv.submit(b)) == g.GT_OK
        v, f = sa.lookup(q)
        assert np.array_equal(b.out1, f) and np.array_equal(b.out0, v)

    run()
    li.set_bounds(0, 0)
    run()
    li.train()
    run()
    assert srv.stats()["graph_launches"] >= 3
    srv.close()


def test_server_retrains_learned_index():
    """With retrain_log2 set, the server retrains the learned index after
    every 2^retrain_log2 inserted keys (admission paused, in-flight batches
    drained) and recaptures its lookup graphs; every result still equals the
    sequential replay, and the index ends trained on the inserted keys."""
    import paper_2604_21117_amd as g
    seed = 74
    keys, vals, fresh = _setup(seed, n=1 << 16)
    sa = oracle.SortedArray(keys, vals, 64)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 15, max_batch=1024)
    li = g.Learned(t, models=128)
    li.train()
    n0 = li.stats()["trained_keys"]
    srv = g.Server(t, learned=li, slots=8, read_streams=4, retrain_log2=13)
    spec = synth.serving_mix(keys, 400, seed, bmax=512, rate=30000.0, fresh=fresh)
    batches = _batches(spec)
    assert srv.replay(batches) == g.GT_OK
    _compare(batches, _oracle_replay(sa, batches))
    inserted = sum(len(b.keys) for b in batches if b.op == 1)
    st = srv.stats()
    assert 1 <= st["retrains"] <= inserted >> 13, (st["retrains"], inserted)
    assert st["retrain_s"] > 0
    assert li.stats()["trained_keys"] > n0
    srv.close()
    bits, ek, ev = oracle.check_export(t.export(), len(sa))
    assert bits == 0 and np.array_equal(ek, sa.keys)


def test_admission_cap():
    import paper_2604_21117_amd as g
    seed = 72
    keys, vals, fresh = _setup(seed, n=1 << 14)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 12, max_batch=1024)
    # room for one 64-key lookup batch at a time; a 1024-key batch never fits
    srv = g.Server(t, slots=4, mem_cap=64 * 17)
    big = g.Batch(0, keys[:1024])
    small = [g.Batch(0, keys[i * 64:(i + 1) * 64]) for i in range(20)]
    tb = srv.submit(big)
    ts = [srv.submit(b) for b in small]
    assert srv.wait(tb) == g.GT_ERR_ADMISSION
    assert all(srv.wait(x) == g.GT_OK for x in ts)
    sa = oracle.SortedArray(keys, vals, 64)
    for b in small:
        v, f = sa.lookup(b.keys)
        assert np.array_equal(b.out0, v) and np.array_equal(b.out1, f)
    srv.close()


def test_padded_lookups_stay_on_the_learned_path():
    """Served lookup batches are padded to a power of two.  With a learned
    index made stale by inserts, a padding entry must not be a key that
    misses its window (such a key goes down the tree): present-key batches
    of uneven sizes cause no tree descent, and their results are exact."""
    import paper_2604_21117_amd as g
    seed = 75
    keys, vals, fresh = _setup(seed, n=1 << 16)
    t = mk_tree(keys, vals, 8, leaf_slack=1 << 14, max_batch=1024)
    li = g.Learned(t, models=128)
    li.train()
    for c in range(0, 3000, 1000):
        k = fresh[c:c + 1000]
        assert (t.insert(k, synth.values_for(k, seed, 64)) == 0).all()
    srv = g.Server(t, learned=li, slots=4)
    f0 = li.stats()["fallbacks"]
    sa = oracle.SortedArray(np.concatenate([keys, fresh[:3000]]),
                            np.concatenate([vals, synth.values_for(fresh[:3000], seed, 64)]), 64)
    for B in (3, 100, 513, 1000):
        q = synth.present_queries(keys, B, seed + B)
        b = g.Batch(0, q)
        assert srv.wait(srv.submit(b)) == g.GT_OK
        v, f = sa.lookup(q)
        assert np.array_equal(b.out1, f) and np.array_equal(b.out0, v)
    srv.close()
    # padding with an absent key made up to half of a bucket descend the
    # tree (513 keys pad to 1024); a present key may descend only after a
    # long chain of splits, which 3000 inserts into 4096 leaves hardly make
    assert li.stats()["fallbacks"] - f0 <= 0.01 * (3 + 100 + 513 + 1000)
    li.close()
    t.close()
