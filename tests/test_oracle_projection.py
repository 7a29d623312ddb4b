"""Pins of the indirect projection p -> p-1 -> ... -> 1 (Appendix A): each
degree-q level transfers to degree q-1 on the same mesh (lumped L2
projection with int phi_q phi_{q-1}, pinned by the Kronecker identity in
test_oracle_assembly) and its coarse correction is one V-cycle of the
degree-(q-1) level; degree 2 keeps the degree-1 h-multigrid of the direct
method.

Fixed independently: at p = 2 the indirect and direct methods are the same
method, so their V-cycles agree bit for bit; the chain has the level sizes
the definition gives; and the paper's counts with an indirect projection
(Appendix A) and their closeness to the direct ones."""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_vcycles.json")


@pytest.mark.parametrize("geom", [0, 1])
def test_indirect_is_direct_at_degree_2(geom):
    od = O.Oracle(2, 2, 32, geom=geom, rhs=geom)
    oi = O.Oracle(2, 2, 32, geom=geom, rhs=geom, opts=O.Options(projection=1))
    x0 = np.random.default_rng(1).uniform(-1, 1, od.n)
    xd, sd, itd, hd = od.solve(od.f(), x0=x0, tol=1e-10)
    xi, si, iti, hi = oi.solve(oi.f(), x0=x0, tol=1e-10)
    assert sd == si == 0 and itd == iti
    assert np.array_equal(hd, hi) and np.array_equal(xd, xi)


@pytest.mark.parametrize("p", [3, 4, 5])
def test_chain_levels(p):
    nel = 16
    o = O.Oracle(2, p, nel, opts=O.Options(projection=1), ilut=False)
    assert o.n == (nel + p - 2) ** 2
    assert o.n1 == (nel + p - 3) ** 2          # coarse space of degree p - 1
    od = O.Oracle(2, p, nel, ilut=False)
    assert od.n1 == (nel - 1) ** 2             # direct: degree 1
    # the transfer is the degree p x degree p-1 one, lumped by degree p-1 masses
    P = o.P()
    assert P.shape == (o.n, o.n1)
    assert np.all(o.ml1() > 0)


def test_paper_iteration_counts_indirect():
    gold = json.load(open(GOLD))["projection_annulus"]
    for p in (3, 4, 5):
        counts = {}
        for proj in (0, 1):
            o = O.Oracle(2, p, 64, geom=1, rhs=1, opts=O.Options(projection=proj))
            x0 = np.random.default_rng(0).uniform(-1, 1, o.n)
            _, st, it, _ = o.solve(o.f(), x0=x0, tol=1e-8)
            assert st == 0
            counts[proj] = it
        paper = gold["indirect"][0][gold["p"].index(p)]    # h = 2^-6
        assert abs(counts[1] - paper) <= 1, (p, counts, paper)
        assert abs(counts[1] - counts[0]) <= 1, (p, counts)
