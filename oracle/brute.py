"""Brute force for tiny inputs: an unsorted list of (key, value) pairs,
searched by linear scan.  TEST INFRASTRUCTURE ONLY.

Each function is the plain definition written out with pure-Python loops,
for n and B up to a few hundred: lookup returns the value or the paper's -1
(all ones at the key width) with found = 0 (Section IV-D); an insert batch
applies its pairs one at a time in batch order, a delete batch removes its
keys one at a time (1 for a key found, else 0); a range lists the pairs with
lo <= key <= hi in ascending key order, cut to the first max of them.
"""
from __future__ import annotations


def _ones(width: int) -> int:
    return (1 << width) - 1


class Brute:
    def __init__(self, keys=(), vals=(), width: int = 64):
        self.width = width
        self.pairs = []  # unsorted (key, value)
        for k, v in zip(keys, vals):
            for p in self.pairs:
                if p[0] == int(k):
                    raise ValueError("duplicate key")
            self.pairs.append([int(k), int(v)])

    def lookup(self, q):
        vals, found = [], []
        for k in q:
            hit = None
            for p in self.pairs:
                if p[0] == int(k):
                    hit = p[1]
            vals.append(_ones(self.width) if hit is None else hit)
            found.append(0 if hit is None else 1)
        return vals, found

    def insert(self, ks, vs):
        status = []
        for k, v in zip(ks, vs):
            for p in self.pairs:
                if p[0] == int(k):
                    p[1] = int(v)
                    status.append(1)
                    break
            else:
                self.pairs.append([int(k), int(v)])
                status.append(0)
        return status

    def delete(self, ks):
        status = []
        for k in ks:
            for i, p in enumerate(self.pairs):
                if p[0] == int(k):
                    self.pairs.pop(i)
                    status.append(1)
                    break
            else:
                status.append(0)
        return status

    def range(self, lo, hi, maxc):
        out = []
        for a, b, m in zip(lo, hi, maxc):
            sel = [p for p in self.pairs if int(a) <= p[0] <= int(b)]
            # selection sort, to stay independent of library sorting
            res = []
            while sel and len(res) < int(m):
                j = 0
                for t in range(1, len(sel)):
                    if sel[t][0] < sel[j][0]:
                        j = t
                res.append((sel[j][0], sel[j][1]))
                sel.pop(j)
            out.append(res)
        return out

    def items(self):
        s = sorted(self.pairs)
        return [p[0] for p in s], [p[1] for p in s]


class BruteBytes:
    """Brute force over byte-string keys (the paper's 32-byte keys) with
    8-byte values: keys are Python bytes, whose built-in order is the
    byte-by-byte order with byte 0 first, each byte unsigned."""

    def __init__(self, keys=(), vals=()):
        self.pairs = []
        for k, v in zip(keys, vals):
            k = bytes(k)
            for p in self.pairs:
                if p[0] == k:
                    raise ValueError("duplicate key")
            self.pairs.append((k, int(v)))

    def lookup(self, q):
        vals, found = [], []
        for k in q:
            k = bytes(k)
            hit = None
            for p in self.pairs:
                if p[0] == k:
                    hit = p[1]
            vals.append((1 << 64) - 1 if hit is None else hit)
            found.append(0 if hit is None else 1)
        return vals, found

    def range(self, lo, hi, maxc):
        out = []
        for a, b, m in zip(lo, hi, maxc):
            a, b = bytes(a), bytes(b)
            sel = [p for p in self.pairs if a <= p[0] <= b]
            # selection sort, so the order owes nothing to a library sort
            res = []
            while sel and len(res) < int(m):
                j = 0
                for t in range(1, len(sel)):
                    if sel[t][0] < sel[j][0]:
                        j = t
                res.append(sel.pop(j))
            out.append(res)
        return out

    def items(self):
        return sorted(self.pairs)

