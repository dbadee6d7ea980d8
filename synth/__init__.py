"""Seeded synthetic inputs for the batched B+-tree workloads.

This module only draws inputs: keys, values, query batches and insert
batches.  It holds none of the tree arithmetic (no search, merge or split)
and imports neither the oracle nor the GPU library, so both sides of every
parity test are fed from here.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): the state advances
by the golden-ratio increment and each output is the state passed through
the splitmix64 finaliser.  The finaliser applied to ``key ^ seed`` is also
the value hash of the workloads (``hash64``; ``hash32`` is its low 32 bits).

The paper evaluates search over random tree entries and random search keys
(Section V-A).  The distributions added here (Zipf, lognormal, clustered)
stand in for public learned-index benchmark key sets; no such dataset is
read, every key is synthetic.
"""
from __future__ import annotations

import numpy as np

U64 = np.uint64
GOLDEN = U64(0x9E3779B97F4A7C15)
M1 = U64(0xBF58476D1CE4E5B9)
M2 = U64(0x94D049BB133111EB)

# purpose tags for independent sub-streams of one master seed
P_KEYS, P_PRESENT, P_ABSENT, P_SHUFFLE, P_INSERT, P_ZIPF, P_PERM, \
    P_LOGN, P_CLUST, P_MIX, P_RANGE, P_SIZE = range(1, 13)


def _mix(z: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser on a uint64 array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> U64(30))) * M1
        z = (z ^ (z >> U64(27))) * M2
        return z ^ (z >> U64(31))


def hash64(x) -> np.ndarray:
    return _mix(np.asarray(x, dtype=U64).copy())


def hash32(x) -> np.ndarray:
    return (hash64(x) & U64(0xFFFFFFFF)).astype(np.uint32)


class Stream:
    """One splitmix64 stream; ``draw(n)`` returns the next n outputs."""

    def __init__(self, seed: int, purpose: int = 0):
        base = hash64(np.array([(int(seed) * 0x100000001B3 + purpose) & 0xFFFFFFFFFFFFFFFF],
                               dtype=U64))[0]
        self.state = U64(base)
        self.count = 0

    def draw(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            idx = np.arange(self.count + 1, self.count + 1 + n, dtype=U64)
            z = self.state + idx * GOLDEN
        self.count += n
        return _mix(z)

    def uniform01(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) from the top 53 bits."""
        return (self.draw(n) >> U64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def below(self, n: int, bound: int) -> np.ndarray:
        """Integers uniform in [0, bound) (multiply-shift on 53 bits)."""
        return np.minimum((self.uniform01(n) * bound).astype(np.int64), bound - 1)


def _mask(width: int) -> np.uint64:
    return U64(0xFFFFFFFF) if width == 32 else U64(0xFFFFFFFFFFFFFFFF)


def dtype_of(width: int):
    return np.uint32 if width == 32 else np.uint64


def distinct_from(stream_fn, n: int, width: int, exclude: np.ndarray | None = None) -> np.ndarray:
    """Draw until n distinct keys are held, dropping repeats (first draw wins)
    and anything in ``exclude``; returns keys in draw order."""
    out = np.empty(0, dtype=U64)
    excl = None if exclude is None or len(exclude) == 0 else np.unique(np.asarray(exclude, dtype=U64))
    while len(out) < n:
        need = n - len(out)
        cand = stream_fn(need + need // 8 + 16)
        allc = np.concatenate([out, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        allc = allc[first]
        if excl is not None:
            allc = allc[~np.isin(allc, excl, assume_unique=False)]
        out = allc[:n] if len(allc) >= n else allc
    return out.astype(dtype_of(width))


def uniform_keys(n: int, seed: int, width: int = 64, purpose: int = P_KEYS,
                 exclude: np.ndarray | None = None) -> np.ndarray:
    """n distinct keys uniform over [0, 2^width), in draw order."""
    s = Stream(seed, purpose)
    m = _mask(width)
    return distinct_from(lambda k: s.draw(k) & m, n, width, exclude)


def values_for(keys: np.ndarray, seed: int, width: int = 64) -> np.ndarray:
    """value = hash(key ^ seed) at the key width (hash32 uses the low 32 bits
    of the seed)."""
    k = np.asarray(keys).astype(U64)
    if width == 32:
        return hash32(k ^ U64(int(seed) & 0xFFFFFFFF))
    return hash64(k ^ U64(int(seed) & 0xFFFFFFFFFFFFFFFF))


def present_queries(keys: np.ndarray, B: int, seed: int, purpose: int = P_PRESENT) -> np.ndarray:
    """B keys drawn uniformly, with replacement, from the present keys."""
    s = Stream(seed, purpose)
    return np.asarray(keys)[s.below(B, len(keys))]


def absent_queries(keys: np.ndarray, B: int, seed: int, width: int = 64,
                   purpose: int = P_ABSENT) -> np.ndarray:
    """B uniform keys that are not present (drawn with replacement among
    absent values)."""
    s = Stream(seed, purpose)
    m = _mask(width)
    ks = np.unique(np.asarray(keys).astype(U64))
    out = np.empty(0, dtype=U64)
    while len(out) < B:
        c = s.draw(B - len(out) + 8) & m
        c = c[~np.isin(c, ks)]
        out = np.concatenate([out, c])[:B]
    return out.astype(dtype_of(width))


def shuffle(x: np.ndarray, seed: int, purpose: int = P_SHUFFLE) -> np.ndarray:
    """Seeded permutation (argsort of one splitmix64 draw per element)."""
    s = Stream(seed, purpose)
    return np.asarray(x)[np.argsort(s.draw(len(x)), kind="stable")]


def mixed_queries(keys: np.ndarray, B: int, seed: int, width: int = 64,
                  frac_present: float = 0.5) -> np.ndarray:
    """B queries: a share present (uniform over keys), the rest absent,
    shuffled together."""
    npres = int(round(B * frac_present))
    q = np.concatenate([present_queries(keys, npres, seed),
                        absent_queries(keys, B - npres, seed, width)])
    return shuffle(q, seed)


class Zipf:
    """Zipf(theta) over ranks 1..n by inverse transform on the exact CDF,
    with rank -> key index scrambled by a seeded permutation so that hot
    keys are not neighbours in key order."""

    def __init__(self, n: int, theta: float, seed: int):
        w = 1.0 / np.power(np.arange(1, n + 1, dtype=np.float64), theta)
        cdf = np.cumsum(w)
        self.cdf = cdf / cdf[-1]
        self.perm = np.argsort(Stream(seed, P_PERM).draw(n), kind="stable")
        self.stream = Stream(seed, P_ZIPF)

    def ranks(self, B: int) -> np.ndarray:
        u = self.stream.uniform01(B)
        return np.minimum(np.searchsorted(self.cdf, u, side="right"), len(self.cdf) - 1)

    def indices(self, B: int) -> np.ndarray:
        return self.perm[self.ranks(B)]


def lognormal_keys(n: int, seed: int, mu: float = 0.0, sigma: float = 2.0) -> np.ndarray:
    """n distinct u64 keys: z ~ N(0,1) by Box-Muller, clipped to [-6, 6];
    x = exp(mu + sigma z); key = floor(x / exp(mu + 6 sigma) * (2^64 - 1))."""
    s = Stream(seed, P_LOGN)
    top = np.exp(mu + 6.0 * sigma)

    def draw(k):
        u1 = s.uniform01(k)
        u2 = s.uniform01(k)
        z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
        z = np.clip(z, -6.0, 6.0)
        x = np.exp(mu + sigma * z) / top
        # floor(x * (2^64-1)) computed in two halves to stay exact-ish in fp64
        v = np.minimum(x * 18446744073709551615.0, 18446744073709549568.0)
        return v.astype(U64)

    return distinct_from(draw, n, 64)


def clustered_keys(n: int, seed: int, clusters: int = 64, span_bits: int = 40) -> np.ndarray:
    """n distinct u64 keys in ``clusters`` dense clusters: bases uniform in
    [0, 2^64 - 2^span), sorted, redrawn while two lie within 2^span; then n/c
    keys uniform in each [b, b + 2^span)."""
    s = Stream(seed, P_CLUST)
    span = 1 << span_bits
    lim = (1 << 64) - span
    while True:
        b = np.sort((s.uniform01(clusters) * lim).astype(U64))
        if clusters < 2 or np.all(np.diff(b.astype(object)) >= span):
            break
    per = [n // clusters + (1 if j < n % clusters else 0) for j in range(clusters)]
    parts = []
    for j in range(clusters):
        base = b[j]
        parts.append(distinct_from(lambda k: base + (s.draw(k) >> U64(64 - span_bits)), per[j], 64))
    return shuffle(np.concatenate(parts), seed, P_CLUST)


def range_starts_and_lengths(keys: np.ndarray, B: int, seed: int, max_len: int = 100,
                             zipf: Zipf | None = None):
    """Range batch: lo = present key (Zipf-chosen when ``zipf`` is given,
    else uniform), hi = all-ones, max = U{1..max_len}."""
    s = Stream(seed, P_RANGE)
    keys = np.asarray(keys)
    if zipf is not None:
        lo = keys[zipf.indices(B)]
    else:
        lo = keys[s.below(B, len(keys))]
    mx = (s.below(B, max_len) + 1).astype(np.uint32)
    hi = np.full(B, np.iinfo(keys.dtype).max, dtype=keys.dtype)
    return lo, hi, mx


def serving_mix(keys: np.ndarray, n_batches: int, seed: int, width: int = 64, bmax: int = 1024,
                mix=(0.8, 0.15, 0.05), rate: float | None = None, zipf: Zipf | None = None,
                max_len: int = 100, fresh: np.ndarray | None = None):
    """A serving workload: per batch (op, keys, values, max, arrival_s).

    op 0 lookup / 1 insert / 2 range drawn with probabilities `mix`; size
    B ~ U{1..bmax}; lookup keys and range starts from the present keys
    (Zipf when given, else uniform); insert keys taken in order from `fresh`
    (absent keys) with values hash(key ^ seed) -- an insert batch beyond the
    end of `fresh` becomes a lookup batch; range hi = all ones and
    max ~ U{1..max_len}; Poisson arrivals at `rate` batches per second (all
    at 0 when rate is None).  All draws are made at once and cut into
    batches."""
    s = Stream(seed, P_MIX)
    u = s.uniform01(n_batches)
    cum = np.cumsum(mix)
    ops = np.searchsorted(cum / cum[-1], u, side="right").astype(np.int64)
    sizes = (s.below(n_batches, bmax) + 1).astype(np.int64)
    if rate:
        gaps = -np.log1p(-s.uniform01(n_batches)) / rate
        arrivals = np.cumsum(gaps) - gaps[0]
    else:
        arrivals = np.zeros(n_batches)
    keys = np.asarray(keys)
    top = np.iinfo(keys.dtype).max
    ins = ops == 1
    if fresh is None:
        ops[ins] = 0
    else:
        need = np.cumsum(np.where(ins, sizes, 0))
        ops[ins & (need > len(fresh))] = 0
    ins = ops == 1
    n_ins = int(sizes[ins].sum())
    ik = fresh[:n_ins] if n_ins else np.zeros(0, dtype=keys.dtype)
    iv = values_for(ik, seed, width) if n_ins else ik
    n_read = int(sizes[~ins].sum())
    ridx = zipf.indices(n_read) if zipf is not None else s.below(n_read, len(keys))
    rk = keys[ridx]
    n_rng = int(sizes[ops == 2].sum())
    rmx = (s.below(n_rng, max_len) + 1).astype(np.uint32)
    out = []
    pi = pr = pm = 0
    for i in range(n_batches):
        B = int(sizes[i])
        op = int(ops[i])
        at = float(arrivals[i])
        if op == 1:
            out.append((1, ik[pi:pi + B], iv[pi:pi + B], None, at))
            pi += B
            continue
        k = rk[pr:pr + B]
        pr += B
        if op == 0:
            out.append((0, k, None, None, at))
        else:
            out.append((2, k, np.full(B, top, dtype=keys.dtype), rmx[pm:pm + B], at))
            pm += B
    return out
