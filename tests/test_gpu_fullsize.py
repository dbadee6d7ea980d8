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


# --------------------------------------------- the configured runs at size

_KEYS = {}


def _keys(log2n, seed):
    """The generator's key set (cached: 2^26 keys take a while on the host)."""
    if (log2n, seed) not in _KEYS:
        k = synth.uniform_keys(1 << log2n, seed, 64)
        _KEYS[(log2n, seed)] = (k, synth.values_for(k, seed, 64))
    return _KEYS[(log2n, seed)]


def test_mix_90_10_on_the_full_tree():
    """The 90/10 protocol on its own 2^24-key tree: per batch size (1 ..
    1024, then 2^20) and query distribution, batches that are lookups with
    probability 0.9, else inserts of fresh keys.  Every lookup result is
    checked: keys of the bulk load and keys inserted earlier must hit with
    hash(key ^ seed), fresh keys not inserted yet must miss; every insert
    status must be INSERTED.  At the end the exported tree passes the
    checker and holds exactly the bulk load plus the inserted keys."""
    import paper_2604_21117_amd as g
    keys, vals = _keys(LOG2N, SEED)
    n = len(keys)
    tree = g.Tree(keys, vals, 8, leaf_slack=(1 << 22), max_batch=1 << 20)
    points = [(b, reps) for b, reps in ((1, 60), (8, 60), (64, 60), (256, 60), (1024, 60), (1 << 20, 6))]
    kinds = {}
    for dist in ("uniform", "zipf"):
        for b, reps in points:
            kind = synth.Stream(SEED, 9000 + b + (dist == "zipf")).uniform01(reps) >= 0.9
            if b == 1 << 20:
                kind[:] = False             # one 2^20 insert per distribution
            kind[reps // 2] = True          # at least one insert per point
            kinds[(dist, b)] = kind
    need = sum(int(k.sum()) * b for (d, b), k in kinds.items()) + 64
    fresh = synth.uniform_keys(need, SEED + 3, 64, purpose=synth.P_INSERT, exclude=keys)
    zipf = synth.Zipf(n, 0.99, SEED)
    fpos, inserted = 0, []
    for dist in ("uniform", "zipf"):
        for b, reps in points:
            kind = kinds[(dist, b)]
            for r in range(reps):
                if kind[r]:
                    k = fresh[fpos:fpos + b]
                    fpos += b
                    st = tree.insert(k, synth.values_for(k, SEED, 64))
                    assert (st == 0).all(), (dist, b, r)
                    inserted.append(k)
                    continue
                q = synth.present_queries(keys, b, SEED + r, purpose=9500 + b) if dist == "uniform" else \
                    keys[zipf.indices(b)]
                if inserted and b >= 8:
                    # a quarter from keys inserted so far, a few not yet inserted
                    ins = np.concatenate(inserted)
                    j = synth.Stream(SEED + r, 9700 + b).below(b // 4, len(ins))
                    q[:b // 4] = ins[j]
                    q[b // 4: b // 4 + 3] = fresh[fpos + 5: fpos + 8]
                v, f = tree.lookup(q)
                absent = np.isin(q, fresh[fpos:fpos + 16])
                assert not f[absent].any() and (v[absent] == np.uint64((1 << 64) - 1)).all(), (dist, b, r)
                _closed_form(v[~absent], f[~absent], q[~absent])
    assert g.tree_device_error(tree.h) == g.GT_OK
    allk = np.concatenate([keys] + inserted)
    bits, ek, ev = oracle.check_export(tree.export(), len(allk))
    assert bits == 0, oracle.violations(bits)
    assert np.array_equal(ek, np.sort(allk)) and np.array_equal(ev, synth.values_for(ek, SEED, 64))
    tree.close()


def test_insert_2p20_into_the_full_tree():
    """The benchmark's 2^20-key insert into the 2^24-key tree: statuses
    against the oracle's, then the exported tree against the oracle's state
    (checker and content), and every inserted key found."""
    import paper_2604_21117_amd as g
    keys, vals = _keys(LOG2N, SEED)
    tree = g.Tree(keys, vals, 8, leaf_slack=(1 << 21) + (1 << 19), max_batch=1 << 20)
    k = synth.uniform_keys(1 << 20, SEED + 1, 64, purpose=synth.P_INSERT, exclude=keys)
    # a few repeats and updates of present keys inside the batch
    k[-64:] = k[:64]
    k[-128:-64] = keys[:64]
    v = synth.values_for(k, SEED + 9, 64)
    sa = oracle.SortedArray(keys, vals, 64)
    st = tree.insert(k, v)
    assert np.array_equal(st, sa.insert(k, v))
    bits, ek, ev = oracle.check_export(tree.export(), len(sa))
    assert bits == 0, oracle.violations(bits)
    assert np.array_equal(ek, sa.keys) and np.array_equal(ev, sa.vals)
    gv, gf = tree.lookup(k)
    ov, of = sa.lookup(k)
    assert np.array_equal(gf, of) and np.array_equal(gv, ov)
    assert tree.stats()["height"] >= 6
    tree.close()


def test_learned_staleness_protocol_every_result():
    """The learned-index protocol on 2^24 keys: from a trained index, 1024
    rounds of a B = 1024 lookup batch (learned and plain) followed by an
    insert batch of 1024 fresh keys (2^20 inserts), every lookup result
    checked; every 64 rounds the learned path also answers keys inserted
    since training (hit) and fresh keys not inserted (miss); then the
    retrain, and old and new keys through the retrained index."""
    import paper_2604_21117_amd as g
    keys, vals = _keys(LOG2N, SEED)
    tree = g.Tree(keys, vals, 8, leaf_slack=(1 << 21) + (1 << 19), max_batch=1 << 20)
    li = g.Learned(tree, models=1024)
    li.train()
    B, rounds = 1024, 1024
    allq = synth.present_queries(keys, 64 * B, SEED, purpose=1000)
    fresh = synth.uniform_keys(rounds * B + 4096, SEED + 1, 64, purpose=synth.P_INSERT, exclude=keys)
    for r in range(rounds):
        q = allq[(r % 64) * B:(r % 64 + 1) * B]
        _closed_form(*li.lookup(q), q)
        _closed_form(*tree.lookup(q), q)
        k = fresh[r * B:(r + 1) * B]
        assert (tree.insert(k, synth.values_for(k, SEED, 64), check=False) == 0).all()
        if r % 64 == 63:
            ins = fresh[:(r + 1) * B]
            qi = ins[synth.Stream(SEED, r).below(B, len(ins))]
            _closed_form(*li.lookup(qi), qi)
            v, f = li.lookup(fresh[rounds * B:rounds * B + 4096])
            assert not f.any() and (v == np.uint64((1 << 64) - 1)).all()
    assert g.tree_device_error(tree.h) == g.GT_OK
    li.train()
    q = np.concatenate([allq[:B], fresh[:B], fresh[(rounds - 1) * B:rounds * B]])
    _closed_form(*li.lookup(q), q)
    li.close()
    tree.close()


def test_serving_2p26_mix():
    """Serving on 2^26 resident keys (seed 5), plain tree and learned index:
    batches B ~ U{1..1024}, 80 % lookups / 15 % inserts of fresh keys / 5 %
    ranges, Zipf(0.99) keys, Poisson arrivals at a rate that keeps batches in
    flight together.  Every lookup must hit with hash(key ^ 5) (they ask for
    keys of the bulk load), every insert must report INSERTED, and every
    range must equal the sorted slice of the bulk load merged with the keys
    inserted before it in admission order."""
    import paper_2604_21117_amd as g
    s5 = 5
    keys, vals = _keys(26, s5)
    sk = np.sort(keys)
    tree = g.Tree(keys, vals, 8, leaf_slack=1 << 21, max_batch=1024)
    li = g.Learned(tree, models=1024)
    fresh = synth.uniform_keys(1 << 20, s5 + 1, 64, purpose=synth.P_INSERT, exclude=keys)
    zipf = synth.Zipf(len(keys), 0.99, s5)
    prev = np.zeros(0, dtype=np.uint64)
    fpos = 0
    for run, learned in enumerate((False, True)):
        if learned:
            li.train()
        srv = g.Server(tree, learned=li if learned else None, slots=16, read_streams=4)
        spec = synth.serving_mix(keys, 1500, s5 + 60 + run, bmax=1024, rate=20000.0, zipf=zipf, fresh=fresh[fpos:])
        fpos += sum(len(kk) for (op, kk, vv, mm, aa) in spec if op == 1)
        batches = [g.Batch(op, kk, vv, mm, aa) for (op, kk, vv, mm, aa) in spec]
        assert srv.replay(batches) == g.GT_OK
        ins_k = [b.keys for b in batches if b.op == g.OP_INSERT]
        ins_j = [np.full(len(b.keys), j) for j, b in enumerate(batches) if b.op == g.OP_INSERT]
        ck = np.concatenate(ins_k)
        cj = np.concatenate(ins_j)
        o = np.argsort(ck, kind="stable")
        ck, cj = ck[o], cj[o]
        for j, b in enumerate(batches):
            if b.op == g.OP_LOOKUP:
                assert b.out1.all() and np.array_equal(b.out0, synth.values_for(b.keys, s5, 64)), ("lookup", j)
            elif b.op == g.OP_INSERT:
                assert (b.out0 == 0).all(), ("insert", j)
            else:
                off = np.concatenate([[0], np.cumsum(b.max_out.astype(np.int64))])
                cur_all = ck[cj < j]
                for i in range(len(b.keys)):
                    lo, mx, c = b.keys[i], int(b.max_out[i]), int(b.count[i])
                    want = np.sort(np.concatenate([sk[np.searchsorted(sk, lo):][:mx],
                                                   prev[np.searchsorted(prev, lo):][:mx],
                                                   cur_all[np.searchsorted(cur_all, lo):][:mx]]))[:mx]
                    assert np.array_equal(b.out0[off[i]:off[i] + c], want), ("range", j, i)
        prev = np.sort(np.concatenate([prev, ck]))
        srv.close()
    li.close()
    tree.close()
