"""Pins of the ILUT ordering (Section 3, "Smoother": a fill-reducing
permutation precedes the factorisation; the reading taken is nested
dissection over grid lines).  The order of a small case is derived by hand
from the definition (tests/golden/nd_order.json); the defining property,
uncoupled halves ordered before their separator, is checked on 2-D and 3-D
line grids; the permutation is a bijection that keeps grid lines whole."""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nd_order.json")


def test_hand_derived_line_order():
    g = json.load(open(GOLD))
    # a 2-D problem whose interior has 20 lines: n_el + p - 2 = 20 with p = 2
    o = O.Oracle(2, g["p"], g["nint"], opts=O.Options(nd_leaf=g["leaf"]), ilut=False)
    perm = o.perm()
    nint = g["nint"]
    lines = [perm[q * nint] // nint for q in range(nint)]
    assert lines == g["lines"]


@pytest.mark.parametrize("dim,p,nel", [(2, 3, 40), (2, 5, 64), (3, 2, 12), (3, 3, 14)])
def test_ordering_is_line_preserving_bijection(dim, p, nel):
    o = O.Oracle(dim, p, nel, ilut=False)
    perm = o.perm()
    nint = nel + p - 2
    assert np.array_equal(np.sort(perm), np.arange(o.n))
    for q in range(o.n // nint):
        blk = perm[q * nint:(q + 1) * nint]
        assert np.array_equal(blk, blk[0] + np.arange(nint)) and blk[0] % nint == 0


def _line_order(o, nint):
    perm = o.perm()
    return [perm[q * nint] // nint for q in range(o.n // nint)]


@pytest.mark.parametrize("p,nel", [(2, 60), (5, 80), (3, 120)])
def test_separator_splits_uncoupled_halves(p, nel):
    """The last p lines of the order form the top separator; every other line
    lies on one side of it, the lines of the two sides are never coupled by the
    stiffness matrix, and one side is ordered entirely before the other."""
    o = O.Oracle(2, p, nel, ilut=False)
    nint = nel + p - 2
    order = _line_order(o, nint)
    sep = sorted(order[-p:])
    assert sep == list(range(sep[0], sep[0] + p))
    left = [l for l in order[:-p] if l < sep[0]]
    right = [l for l in order[:-p] if l > sep[-1]]
    assert len(left) + len(right) == nint - p
    A = o.A().tocsr()
    coupled = np.zeros((nint, nint), dtype=bool)
    for i in range(A.shape[0]):
        for j in A.indices[A.indptr[i]:A.indptr[i + 1]]:
            coupled[i // nint, j // nint] = True
    assert not coupled[np.ix_(left, right)].any()
    pos = {l: q for q, l in enumerate(order)}
    assert max(pos[l] for l in left) < min(pos[l] for l in right)
