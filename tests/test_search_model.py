"""Host models of two index computations in the peel kernel, checked
exhaustively on small cases for the two properties the kernel relies on:
every array read stays inside its range, and the result equals the plain
definition.

* Lockstep search of one key in two sorted, non-empty ranges: both binary
  searches advance together; a range already narrowed down re-reads its
  last slot. Result: the key's position in each range, or the range's end.
* Segment lookup of a probe unit p in the exclusive prefix offsets
  off[0..nb] (off[0] = 0 <= p < off[nb]): the last segment lo with
  off[lo] <= p, by binary search in a lane's first pass and by a gallop from
  the lane's previous segment afterwards (units only grow from pass to pass).
"""
from __future__ import annotations

import bisect
import itertools
import random


def find2(a, lo1, hi1, lo2, hi2, x, reads):
    l1, h1, l2, h2 = lo1, hi1, lo2, hi2
    while l1 < h1 or l2 < h2:
        m1 = l1 + ((h1 - l1) >> 1) if l1 < h1 else hi1 - 1
        m2 = l2 + ((h2 - l2) >> 1) if l2 < h2 else hi2 - 1
        reads.append((1, m1))
        reads.append((2, m2))
        v1, v2 = a[m1], a[m2]
        if l1 < h1:
            if v1 < x:
                l1 = m1 + 1
            else:
                h1 = m1
        if l2 < h2:
            if v2 < x:
                l2 = m2 + 1
            else:
                h2 = m2
    i1 = l1 if l1 < hi1 else hi1 - 1
    i2 = l2 if l2 < hi2 else hi2 - 1
    reads.append((1, i1))
    reads.append((2, i2))
    p1 = l1 if (l1 < hi1 and a[i1] == x) else hi1
    p2 = l2 if (l2 < hi2 and a[i2] == x) else hi2
    return p1, p2


def plain_find(a, lo, hi, x):
    p = bisect.bisect_left(a, x, lo, hi)
    return p if p < hi and a[p] == x else hi


def test_lockstep_search_reads_in_range_and_finds_keys():
    rng = random.Random(5)
    for _ in range(3000):
        n1, n2 = rng.randint(1, 12), rng.randint(1, 12)
        r1 = sorted(rng.sample(range(40), n1))
        r2 = sorted(rng.sample(range(40), n2))
        pad = rng.randint(0, 3)
        a = [rng.randint(0, 50) for _ in range(pad)] + r1 + r2 + [rng.randint(0, 50) for _ in range(pad)]
        lo1, hi1 = pad, pad + n1
        lo2, hi2 = hi1, hi1 + n2
        for x in range(-1, 42):
            reads = []
            p1, p2 = find2(a, lo1, hi1, lo2, hi2, x, reads)
            assert all(lo1 <= i < hi1 for r, i in reads if r == 1)
            assert all(lo2 <= i < hi2 for r, i in reads if r == 2)
            assert p1 == plain_find(a, lo1, hi1, x)
            assert p2 == plain_find(a, lo2, hi2, x)


def segment_binary(off, nb, p, reads):
    lo, hi = 0, nb
    while hi - lo > 1:
        mid = (lo + hi) >> 1
        reads.append(mid)
        if off[mid] <= p:
            lo = mid
        else:
            hi = mid
    return lo


def segment_gallop(off, nb, p, hint, reads):
    lo, hi = hint, nb
    if lo != 0:
        step = 1
        while lo + step < nb:
            reads.append(lo + step)
            if off[lo + step] > p:
                break
            lo += step
            step <<= 1
        hi = lo + step if lo + step < nb else nb
    while hi - lo > 1:
        mid = (lo + hi) >> 1
        reads.append(mid)
        if off[mid] <= p:
            lo = mid
        else:
            hi = mid
    return lo


def test_segment_gallop_matches_binary_search():
    rng = random.Random(9)
    for _ in range(400):
        nb = rng.randint(1, 40)
        # segment sizes, some empty
        sizes = [rng.choice([0, 0, 1, 2, 5, 17]) for _ in range(nb)]
        if sum(sizes) == 0:
            sizes[rng.randrange(nb)] = 3
        off = [0] + list(itertools.accumulate(sizes))   # off[nb] = P
        P = off[nb]
        nthreads = rng.randint(1, 12)
        for lane in range(min(nthreads, P)):
            hint = 0
            for p in range(lane, P, nthreads):   # one lane's passes
                reads = []
                lo = segment_gallop(off, nb, p, hint, reads)
                assert all(0 < i < nb for i in reads)
                assert lo == segment_binary(off, nb, p, [])
                assert off[lo] <= p < off[lo + 1]   # a non-empty segment holds p
                hint = lo
