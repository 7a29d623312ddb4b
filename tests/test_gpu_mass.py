"""Consistent-mass transfers (Appendix B) on the GPU against the oracle's,
through the C ABI.  The GPU solves with M_1 and M_p by conjugate gradients
preconditioned with the lumped masses (to 1e-13), the oracle by plain CG
(to 1e-14); at p = 5 the mass matrix has condition number about 5e4, so
transferred vectors agree to 5e-11 relative; whole
solves by the residual-history metric (1e-9) and iteration counts within
one.  At degree 1 both transfers are the identity (P_1^1 = M_1)."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


CASES = [(2, 2, 16, 0), (2, 3, 32, 1), (2, 5, 64, 1), (3, 2, 8, 0)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "d%dp%dn%dg%d" % c)
def test_consistent_transfers_and_solve_match_oracle(case):
    import paper_1901_01685_amd as pmg
    dev = _dev()
    dim, p, nel, g = case
    print("mass case", case, flush=True)
    s = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, device=0, mass_transfer=pmg.MASS_CONSISTENT)
    o = O.Oracle(dim, p, nel, geom=g, rhs=g, opts=O.Options(mass_transfer=1))
    rng = np.random.default_rng(3)
    r = rng.uniform(-1, 1, s.n)
    r1 = torch.empty(s.n1, dtype=torch.float64, device=dev)
    s.restrict(torch.tensor(r, device=dev), r1)
    assert _rel(r1.cpu().numpy(), o.restrict(r)) < 5e-11
    e1 = rng.uniform(-1, 1, s.n1)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    s.prolong(torch.tensor(e1, device=dev), x)
    assert _rel(x.cpu().numpy(), o.prolong_delta(e1)) < 5e-11
    # whole solve
    b = torch.empty(s.n, dtype=torch.float64, device=dev)
    s.rhs(b)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    st, it, rel, r0, _, hist = s.solve(b, x, tol=1e-8)
    xo, sto, ito, histo = o.solve(o.f(), tol=1e-8)
    print(case, "gpu", it, "oracle", ito, flush=True)
    assert st == pmg.OK and sto == 0 and abs(it - ito) <= 1
    k = min(len(hist), len(histo))
    assert np.abs(hist[:k] - histo[:k]).max() <= 1e-9, (hist, histo)


def test_consistent_transfers_are_identity_at_degree_1():
    import paper_1901_01685_amd as pmg
    dev = _dev()
    s = pmg.Solver(2, 1, 32, geometry=1, rhs_kind=1, device=0, mass_transfer=pmg.MASS_CONSISTENT)
    assert s.n == s.n1
    v = np.random.default_rng(5).uniform(-1, 1, s.n)
    out = torch.empty(s.n1, dtype=torch.float64, device=dev)
    s.restrict(torch.tensor(v, device=dev), out)
    assert _rel(out.cpu().numpy(), v) < 1e-12
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    s.prolong(torch.tensor(v, device=dev), x)
    assert _rel(x.cpu().numpy(), v) < 1e-12


def test_consistent_bicgstab_and_counts_like_lumped():
    import paper_1901_01685_amd as pmg
    dev = _dev()
    its = {}
    for mt in (pmg.MASS_LUMPED, pmg.MASS_CONSISTENT):
        s = pmg.Solver(2, 4, 64, geometry=1, rhs_kind=1, device=0, mass_transfer=mt)
        b = torch.empty(s.n, dtype=torch.float64, device=dev)
        s.rhs(b)
        x = torch.zeros(s.n, dtype=torch.float64, device=dev)
        st, it, *_ = s.solve(b, x, tol=1e-8)
        assert st == pmg.OK
        x = torch.zeros(s.n, dtype=torch.float64, device=dev)
        st2, it2, rel2, *_ = s.bicgstab(b, x, tol=1e-8)
        assert st2 == pmg.OK and rel2 <= 1e-8 and it2 <= 4
        its[mt] = it
    assert abs(its[0] - its[1]) <= 1, its
