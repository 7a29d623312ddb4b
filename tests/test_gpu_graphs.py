"""Outer steps replayed from cached HIP graphs give exactly what the same
kernels give launched one by one (stated tolerance: bitwise, same kernels and
launch shapes).  Every replay is checked, with eager work and
synchronisations between replays, after a change of vectors (re-capture),
and for whole FP64 and mixed-precision solves."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("case", [(2, 3, 64, 0), (2, 4, 32, 1), (3, 2, 12, 0)], ids=lambda c: "d%dp%dn%dg%d" % c)
def test_vcycle_replays_match_eager(case):
    import paper_1901_01685_amd as pmg
    _need_gpu()
    dim, p, nel, g = case
    sg = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, device=0, graphs=1)
    se = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, device=0, graphs=0)
    dev = torch.device("cuda:0")
    n = sg.n
    b = torch.empty(n, dtype=torch.float64, device=dev)
    sg.rhs(b)
    rng = np.random.default_rng(3)
    x0 = torch.tensor(rng.uniform(-1, 1, n), device=dev)
    for vecs in range(2):  # second round: other vectors, so the graph is captured again
        xg, xe = x0.clone(), x0.clone()
        rg, re = torch.empty_like(b), torch.empty_like(b)
        sg.residual(b, xg, rg)
        se.residual(b, xe, re)
        for it in range(5):
            ng = sg.vcycle(b, xg, rg, norm=True)
            ne = se.vcycle(b, xe, re, norm=True)
            torch.cuda.synchronize()
            assert torch.equal(xg, xe) and torch.equal(rg, re), (vecs, it)
            assert ng == ne
            # eager work of the program between replays
            tmp = torch.empty_like(b)
            sg.residual(b, x0, tmp)
            (tmp * 2.0).sum().item()
        x0 = x0 * 0.5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solves_match_eager(precision):
    import paper_1901_01685_amd as pmg
    _need_gpu()
    kw = {"precision": pmg.FP32_IN_FP64} if precision == "mixed" else {}
    sg = pmg.Solver(2, 4, 64, device=0, graphs=1, **kw)
    se = pmg.Solver(2, 4, 64, device=0, graphs=0, **kw)
    dev = torch.device("cuda:0")
    b = torch.empty(sg.n, dtype=torch.float64, device=dev)
    sg.rhs(b)
    for rep in range(2):
        xg = torch.zeros_like(b)
        xe = torch.zeros_like(b)
        rg = sg.solve(b, xg, tol=1e-10)
        re = se.solve(b, xe, tol=1e-10)
        torch.cuda.synchronize()
        assert rg[0] == pmg.OK and re[0] == pmg.OK
        assert rg[1] == re[1] and np.array_equal(rg[5], re[5]), (rg[1], re[1])
        assert torch.equal(xg, xe)
