"""Pins of the consistent-mass transfers (Appendix B): restriction
r1 = M_1^{-1} P_p^1 r and prolongation u += M_p^{-1} P_1^p e1 with the
consistent interior mass matrices instead of their row-sum lumped diagonals.

Fixed independently of the oracle's formulas:
  * at degree p = 1 the transfer matrix P_1^1 is the degree-1 mass matrix
    itself, so both consistent transfers are the identity (the lumped ones
    are not) - this fails for a wrong mass matrix, a transposed transfer or
    an inaccurate inner solve;
  * the paper's V-cycle counts with consistent masses (Appendix B), and its
    observation that with ILUT they hardly differ from the lumped ones."""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_vcycles.json")


@pytest.mark.parametrize("geom", [0, 1])
def test_consistent_transfers_are_identity_at_degree_1(geom):
    rng = np.random.default_rng(2)
    oc = O.Oracle(2, 1, 16, geom=geom, rhs=geom, opts=O.Options(mass_transfer=1), ilut=False)
    ol = O.Oracle(2, 1, 16, geom=geom, rhs=geom, ilut=False)
    assert oc.n == oc.n1
    v = rng.uniform(-1, 1, oc.n)
    for f in ("restrict", "prolong_delta"):
        y = getattr(oc, f)(v)
        assert np.linalg.norm(y - v) <= 1e-12 * np.linalg.norm(v), f
        yl = getattr(ol, f)(v)
        assert np.linalg.norm(yl - v) >= 1e-3 * np.linalg.norm(v), f   # lumping is not exact


def test_paper_iteration_counts_consistent_vs_lumped():
    gold = json.load(open(GOLD))["mass_transfer_annulus"]
    for p in (2, 3, 4, 5):
        counts = {}
        for mt in (0, 1):
            o = O.Oracle(2, p, 64, geom=1, rhs=1, opts=O.Options(mass_transfer=mt))
            x0 = np.random.default_rng(0).uniform(-1, 1, o.n)
            _, st, it, _ = o.solve(o.f(), x0=x0, tol=1e-8)
            assert st == 0
            counts[mt] = it
        paper = gold["consistent"][0][gold["p"].index(p)]   # h = 2^-6
        assert abs(counts[1] - paper) <= 1, (p, counts, paper)
        assert abs(counts[1] - counts[0]) <= 1, (p, counts)
