"""Parity at the benchmark's full size: 2^24 uniform u64 keys (seed 2) with
the benchmark's arena, 1024 learned models and the launch shapes the
benchmark times (B = 1024 and 2^20).  Present queries are checked against
the generator's closed form (value = hash(key ^ seed)), absent ones must
miss, and a mixed sample is compared with the oracle one by one."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

SEED, LOG2N = 2, 24


@pytest.fixture(scope="module")
def full():
    import torch
    import paper_2604_21117_amd as g
    assert torch.cuda.is_available()
    n = 1 << LOG2N
    keys = synth.uniform_keys(n, SEED, 64)
    vals = synth.values_for(keys, SEED, 64)
    tree = g.Tree(keys, vals, 8, leaf_slack=(1 << 20) + (1 << 18), max_batch=1 << 20)
    li = g.Learned(tree, models=1024)
    li.train()
    yield {"keys": keys, "vals": vals, "tree": tree, "li": li}
    li.close()
    tree.close()


def _closed_form(v, f, q):
    assert f.all(), f"misses at {np.nonzero(f == 0)[0][:8]}"
    assert np.array_equal(v, synth.values_for(q, SEED, 64)), "values differ from hash(key ^ seed)"


def test_shape_of_the_full_tree(full):
    st = full["tree"].stats()
    assert st["n_keys"] == 1 << 24 and st["height"] == 6
    assert st["leaf_used"] == 1 << 20 and st["inner_used"] == 69905


def test_b1024_batches_plain_and_learned(full):
    keys, tree, li = full["keys"], full["tree"], full["li"]
    allq = synth.present_queries(keys, 16 * 1024, SEED, purpose=1000)
    for i in range(16):
        q = allq[i * 1024:(i + 1) * 1024]
        _closed_form(*tree.lookup(q), q)
        _closed_form(*li.lookup(q), q)
        _closed_form(*tree.lookup_levelwise(q), q)
    absent = synth.absent_queries(keys, 1024, SEED, 64)
    for v, f in (tree.lookup(absent), li.lookup(absent), tree.lookup_levelwise(absent)):
        assert not f.any() and np.all(v == np.uint64(0xFFFFFFFFFFFFFFFF))


def test_2p20_batch_every_path(full):
    keys, tree, li = full["keys"], full["tree"], full["li"]
    q = synth.present_queries(keys, 1 << 20, SEED, purpose=5000)
    _closed_form(*tree.lookup(q), q)
    _closed_form(*li.lookup(q), q)
    _closed_form(*tree.lookup_levelwise(q), q)
    qs = np.sort(q)
    _closed_form(*tree.lookup_levelwise(qs, presorted=True), qs)


def test_mixed_sample_against_the_oracle(full):
    keys, vals, tree, li = full["keys"], full["vals"], full["tree"], full["li"]
    sa = oracle.SortedArray(keys, vals, 64)
    q = synth.mixed_queries(keys, 1 << 16, SEED + 5, 64)
    top = np.iinfo(np.uint64).max
    q[:4] = [0, top, keys.min(), keys.max()]
    ov, of = sa.lookup(q)
    for name, (v, f) in (("plain", tree.lookup(q)), ("learned", li.lookup(q)),
                         ("levelwise", tree.lookup_levelwise(q))):
        assert np.array_equal(f, of), f"{name}: found flags differ at {np.nonzero(f != of)[0][:8]}"
        assert np.array_equal(v, ov), f"{name}: values differ at {np.nonzero(v != ov)[0][:8]}"


def test_delete_2p20_on_the_full_tree():
    """A 2^20-key delete batch on its own 2^24-key tree (the benchmark's
    shape): every deleted key now misses, a sample of the others still hits
    with hash(key ^ seed), the count and the exported invariants hold, and
    the learned index answers through the tree, then from its models again
    after training."""
    import paper_2604_21117_amd as g
    n = 1 << LOG2N
    keys = synth.uniform_keys(n, SEED, 64)
    vals = synth.values_for(keys, SEED, 64)
    tree = g.Tree(keys, vals, 8, max_batch=1 << 20)
    li = g.Learned(tree, models=1024)
    li.train()
    gone = synth.shuffle(keys, SEED + 21)[:1 << 20]
    st = tree.delete(gone)
    assert st.all()
    assert tree.stats()["n_keys"] == n - (1 << 20)
    assert not tree.delete(gone[:4096]).any()
    v, f = tree.lookup(gone[:1 << 16])
    assert not f.any()
    keep = np.setdiff1d(keys, gone, assume_unique=True)
    q = synth.shuffle(keep, SEED + 22)[:1 << 16]
    _closed_form(*tree.lookup(q), q)
    _closed_form(*li.lookup(q), q)
    _closed_form(*tree.lookup_levelwise(q), q)
    bits, ek, _ = oracle.check_export(tree.export(), n - (1 << 20))
    assert bits == 0, oracle.violations(bits)
    assert np.array_equal(ek, np.sort(keep))
    li.train()
    _closed_form(*li.lookup(q), q)
    v, f = li.lookup(gone[:1 << 16])
    assert not f.any()
    li.close()
    tree.close()
