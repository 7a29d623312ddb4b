"""The timed configuration itself (2-D unit square, p = 5, h = 1/1024,
1,054,729 unknowns, the launch shapes bench.py times), where the oracle is too
slow to set up: properties that hold at any size, checked on the host with the
library's exported operators (whose equality with the oracle's is pinned at
smaller sizes by the host tests).  Stated tolerances: the residual kernel and
the triangular solves normwise 1e-12 relative (summation order only); the
whole solve's residual recomputed on the host within 1 % of the tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_bench_configuration_kernels_and_solve():
    import paper_1901_01685_amd as pmg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    s = pmg.Solver(2, 5, 1024, device=0)
    n = s.n
    print("bench configuration n", n, "chunks", s.info.chunks_l, s.info.chunks_u, flush=True)
    A = s.export(pmg.OP_A).tocsr()
    L = s.export(pmg.OP_L).tocsr()
    U = s.export(pmg.OP_U).tocsr()
    perm = s.export_perm()
    rng = np.random.default_rng(7)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    s.rhs(b)
    bh = b.cpu().numpy()
    x0 = rng.uniform(-1, 1, n)
    x = torch.tensor(x0, device=dev)
    # a1: residual
    r = torch.empty_like(b)
    nrm = s.residual(b, x, r, norm=True)
    rh = r.cpu().numpy()
    r_ref = bh - A @ x0
    assert np.linalg.norm(rh - r_ref) <= 1e-12 * np.linalg.norm(r_ref)
    assert abs(nrm - np.linalg.norm(r_ref)) <= 1e-12 * np.linalg.norm(r_ref)
    # a2: forward substitution, (I + L) y = P r
    y = torch.empty_like(b)
    s.lower_solve(r, y)
    yh = y.cpu().numpy()
    pr = rh[perm]
    assert np.linalg.norm(yh + L @ yh - pr) <= 1e-12 * np.linalg.norm(pr)
    # a3: backward substitution, U e = y and x += P^T e
    s.upper_solve(y, x)
    e_perm = (x.cpu().numpy() - x0)[perm]
    assert np.linalg.norm(U @ e_perm - yh) <= 1e-11 * np.linalg.norm(yh)
    # whole solve from zero, residual recomputed on the host
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    st, it, rel, *_ = s.solve(b, x, tol=1e-8)
    xh = x.cpu().numpy()
    rel_cpu = np.linalg.norm(bh - A @ xh) / np.linalg.norm(bh)
    print(f"bench configuration: {it} V-cycles, relres {rel:.3e}, host {rel_cpu:.3e}", flush=True)
    assert st == pmg.OK and rel <= 1e-8 and rel_cpu <= 1.01e-8
    assert it <= 8
