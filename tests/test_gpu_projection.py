"""Indirect projection p -> p-1 -> ... -> 1 (Appendix A) on the GPU against
the oracle's chain of levels, through the C ABI: whole solves by the
residual-history metric (1e-10) and iteration counts within one; at p = 2
the indirect method is the direct one, bit for bit; graph replays equal
kernel-by-kernel launches (the graph also holds the inner levels' kernels);
BiCGSTAB with the indirect V-cycle as preconditioner."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = [(2, 3, 32, 0, 0), (2, 4, 32, 1, 0), (2, 5, 64, 1, 0), (3, 3, 8, 0, 0), (2, 4, 32, 0, 1)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "d%dp%dn%dg%d" % c[:4] + ("cdr" if c[4] else ""))
def test_indirect_solve_matches_oracle(case):
    import paper_1901_01685_amd as pmg
    dev = _dev()
    dim, p, nel, g, pde = case
    print("indirect case", case, flush=True)
    s = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, pde=pde, device=0, projection=pmg.PROJ_INDIRECT)
    o = O.Oracle(dim, p, nel, geom=g, rhs=g, pde=pde, opts=O.Options(projection=1))
    assert s.n1 == o.n1
    x0 = np.random.default_rng(0).uniform(-1, 1, s.n)
    b = torch.empty(s.n, dtype=torch.float64, device=dev)
    s.rhs(b)
    x = torch.tensor(x0, device=dev)
    st, it, rel, r0, _, hist = s.solve(b, x, tol=1e-8)
    xo, sto, ito, histo = o.solve(o.f(), x0=x0, tol=1e-8)
    print(case, "gpu", it, "oracle", ito, flush=True)
    assert st == pmg.OK and sto == 0 and abs(it - ito) <= 1
    k = min(len(hist), len(histo))
    assert np.abs(hist[:k] - histo[:k]).max() <= 1e-10, (hist, histo)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-7 * np.linalg.norm(xo)


def test_indirect_is_direct_at_degree_2_and_graph_equals_eager():
    import paper_1901_01685_amd as pmg
    dev = _dev()
    sd = pmg.Solver(2, 2, 64, geometry=1, rhs_kind=1, device=0)
    si = pmg.Solver(2, 2, 64, geometry=1, rhs_kind=1, device=0, projection=pmg.PROJ_INDIRECT)
    b = torch.empty(sd.n, dtype=torch.float64, device=dev)
    sd.rhs(b)
    xd, xi = torch.zeros_like(b), torch.zeros_like(b)
    outd, outi = sd.solve(b, xd, tol=1e-10), si.solve(b, xi, tol=1e-10)
    assert outd[1] == outi[1] and torch.equal(xd, xi)
    # graph replays against eager launches with a three-level chain (p = 4)
    sg = pmg.Solver(2, 4, 32, device=0, projection=pmg.PROJ_INDIRECT, graphs=1)
    se = pmg.Solver(2, 4, 32, device=0, projection=pmg.PROJ_INDIRECT, graphs=0)
    b = torch.empty(sg.n, dtype=torch.float64, device=dev)
    sg.rhs(b)
    x0 = torch.tensor(np.random.default_rng(4).uniform(-1, 1, sg.n), device=dev)
    xg, xe = x0.clone(), x0.clone()
    rg, re = torch.empty_like(b), torch.empty_like(b)
    sg.residual(b, xg, rg)
    se.residual(b, xe, re)
    for k in range(4):
        ng = sg.vcycle(b, xg, rg, norm=True)
        ne = se.vcycle(b, xe, re, norm=True)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and ng == ne, k


def test_indirect_bicgstab_matches_oracle():
    import paper_1901_01685_amd as pmg
    dev = _dev()
    s = pmg.Solver(2, 4, 64, geometry=1, rhs_kind=1, device=0, projection=pmg.PROJ_INDIRECT)
    o = O.Oracle(2, 4, 64, geom=1, rhs=1, opts=O.Options(projection=1))
    f = o.f()
    xo, so, io, ho = o.bicgstab(f, tol=1e-10)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    st, it, rel, *_ = s.bicgstab(torch.tensor(f, device=dev), x, tol=1e-10)
    assert st == pmg.OK and so == 0 and abs(it - io) <= 1 and it <= 5
    assert np.linalg.norm(o.residual(f, x.cpu().numpy())) <= 1.01e-10 * np.linalg.norm(f)
