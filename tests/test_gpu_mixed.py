"""Mixed precision (FP32 V-cycle inside FP64 defect correction): the returned
x must reach the FP64 relative residual 1e-10, recomputed independently
(oracle residual on small cases, scipy FP64 SpMV with the exported operator
at the full quarter-annulus size), and it is compared with the FP64 oracle
solution.  The inner V-cycle runs in FP32 (FP32 accumulation); the outer
residual, the update and the p = 1 coarse solve stay FP64."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("case", [(2, 3, 32, 0), (2, 5, 32, 1), (2, 5, 64, 1), (3, 2, 12, 0), (2, 4, 64, 0, 1)],
                         ids=lambda c: "d%dp%dn%dg%d" % c[:4] + ("cdr" if len(c) > 4 else ""))
def test_mixed_reaches_fp64_tolerance(case):
    import paper_1901_01685_amd as pmg
    dev = _dev()
    dim, p, nel, g = case[:4]
    pde = case[4] if len(case) > 4 else 0
    print("mixed case", case, flush=True)
    sm = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, pde=pde, device=0, precision=pmg.FP32_IN_FP64)
    sd = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, pde=pde, device=0)
    o = O.Oracle(dim, p, nel, geom=g, rhs=g, pde=pde)
    n = sm.n
    b = torch.empty(n, dtype=torch.float64, device=dev)
    sm.rhs(b)
    xm = torch.zeros(n, dtype=torch.float64, device=dev)
    st, it_m, rel_m, r0, _, hist_m = sm.solve(b, xm, tol=1e-10)
    xd = torch.zeros(n, dtype=torch.float64, device=dev)
    st_d, it_d, rel_d, *_ = sd.solve(b, xd, tol=1e-10)
    assert st == pmg.OK and st_d == pmg.OK
    assert rel_m <= 1e-10
    # independent FP64 residual of the returned x
    f = o.f()
    xmh = xm.cpu().numpy()
    rel_or = np.linalg.norm(o.residual(f, xmh)) / np.linalg.norm(f)
    assert rel_or <= 1.01e-10, rel_or
    # error against the FP64 oracle solution
    xo, sto, ito, _ = o.solve(f, tol=1e-12)
    err = np.linalg.norm(xmh - xo) / np.linalg.norm(xo)
    print(f"mixed {case}: outer {it_m} (fp64 {it_d}), relres {rel_m:.2e}, oracle relres {rel_or:.2e}, "
          f"error vs oracle {err:.2e}", flush=True)
    assert err <= 1e-8
    # the FP32 inner cycle contracts almost like the FP64 one
    assert it_m <= it_d + 3


def test_mixed_full_size_quarter_annulus():
    """The mixed-precision workload: quarter annulus, p = 5, h = 1/512
    (265,225 unknowns), FP64 relative residual 1e-10."""
    import scipy.sparse as sp
    import paper_1901_01685_amd as pmg
    dev = _dev()
    sm = pmg.Solver(2, 5, 512, geometry=1, rhs_kind=1, device=0, precision=pmg.FP32_IN_FP64)
    n = sm.n
    print("annulus p5 h1/512 n", n, flush=True)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    sm.rhs(b)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    st, it, rel, r0, secs, hist = sm.solve(b, x, tol=1e-10)
    assert st == pmg.OK and rel <= 1e-10
    A = sm.export(pmg.OP_A)
    bh, xh = b.cpu().numpy(), x.cpu().numpy()
    rel_cpu = np.linalg.norm(bh - A @ xh) / np.linalg.norm(bh)
    print(f"mixed full: {it} outer steps, {secs*1e3:.1f} ms, relres {rel:.2e} (scipy {rel_cpu:.2e})",
          flush=True)
    assert rel_cpu <= 1.01e-10
    # FP64 solve of the same problem for the error report
    sd = pmg.Solver(2, 5, 512, geometry=1, rhs_kind=1, device=0)
    xd = torch.zeros(n, dtype=torch.float64, device=dev)
    std, itd, reld, *_ = sd.solve(b, xd, tol=1e-12)
    err = float(torch.linalg.norm(x - xd) / torch.linalg.norm(xd))
    print(f"fp64: {itd} V-cycles to {reld:.2e}; mixed vs fp64 error {err:.2e}", flush=True)
    assert err <= 1e-8
