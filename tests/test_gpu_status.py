"""Status branches of the solve on the GPU, through the C ABI, against the
oracle on the same inputs (Section 5: a solve has diverged when the relative
residual exceeds 1e10 at the end of a V-cycle).

The divergence branch is reached with an injected operator
(pmg_setup_from_csr): A_p - 2 lambda_min(A_p) I is indefinite, the positive
definite degree-1 coarse correction no longer matches it, and the V-cycle
iteration grows by about 1.4 per cycle until it passes 1e10."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla
import torch

import oracle as O
import paper_1901_01685_amd as pmg

pytestmark = pytest.mark.gpu


def _shifted(A, c):
    lmin = sla.eigsh(A, k=1, sigma=0, which="LM")[0][0]
    return (A - c * lmin * sp.eye(A.shape[0])).tocsr()


def test_diverged_on_both_sides_at_the_same_cycle():
    o = O.Oracle(2, 3, 32)
    B = _shifted(o.A(), 2.0)
    assert o.set_operator(B)[0] == 0
    f = o.f()
    xo, sto, ito, ho = o.solve(f, tol=1e-8)
    assert sto == O.EDIVERGED and 10 < ito < 100
    s = pmg.Solver(2, 3, 32, operator=B, device=0)
    dev = torch.device("cuda:0")
    b = torch.tensor(f, device=dev)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    st, it, rel, r0, _, h = s.solve(b, x, tol=1e-8)
    print(f"gpu {st} {it} {rel:.3e}  oracle {sto} {ito} {ho[-1]:.3e}", flush=True)
    assert st == pmg.EDIVERGED and abs(it - ito) <= 1, (st, it, ito)
    k = min(len(h), len(ho))
    assert np.allclose(h[:k], ho[:k], rtol=1e-8, atol=0), np.abs(h[:k] / ho[:k] - 1).max()
    if it == ito:  # the last iterate is returned
        xg = x.cpu().numpy()
        assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)


def test_divergence_ratio_is_strict_and_relative():
    o = O.Oracle(2, 3, 32)
    B = _shifted(o.A(), 2.0)
    o.set_operator(B)
    f = o.f()
    _, _, _, ho = o.solve(f, tol=1e-8)
    dev = torch.device("cuda:0")
    s = pmg.Solver(2, 3, 32, operator=B, device=0, diverge_ratio=float(ho[1]))
    b = torch.tensor(f, device=dev)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    st, it, *_ = s.solve(b, x, tol=1e-8)
    assert st == pmg.EDIVERGED and it == 2, (st, it)


def test_server_uses_its_divergence_ratio():
    srv = pmg.Server(budget_bytes=2 << 30, max_slots=2, diverge_ratio=1e-6)
    try:
        st, t = srv.submit(2, 2, 32)
        assert st == pmg.OK
        st, info, _ = srv.wait(t)
        assert st == pmg.EDIVERGED and info["iterations"] == 1, (st, info)
    finally:
        srv.close()
    srv = pmg.Server(budget_bytes=2 << 30, max_slots=2)
    try:
        st, t = srv.submit(2, 2, 32)
        res = None
        while res is None:
            res = srv.poll(t)
        st, info, x = res
        assert st == pmg.OK and info["relres"] <= 1e-10
    finally:
        srv.close()
