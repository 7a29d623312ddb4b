"""Tiled smoothing on 2-D degree-1 levels (gs_tile_down / gs_tile_up) gives
exactly what the launch-per-colour and launch-per-transfer kernels give
(stated tolerance: bitwise; the same per-node arithmetic in the same order),
also where the tiled kernels form the level's values from its 1-D Kronecker
factors (2-D unit box, Poisson).
Cases cover ragged last blocks, a one-node last block (the 511-node coarse
level of h = 1/1024 in blocks of 30), two sweeps, and a 3-D problem (which
always takes the launch-per-phase path)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    # dim, degree, n_elem, geometry, extra options
    (2, 2, 256, 0, {}),
    (2, 3, 128, 1, {}),
    (2, 2, 256, 0, {"nu1": 2, "nu2": 1}),
    (2, 2, 1024, 0, {}),
    (3, 2, 16, 0, {}),
    (2, 2, 256, 0, {"pde": 1}),   # non-symmetric CDR stencils (benchmark 2)
]


def _id(c):
    return "d%dp%dn%dg%d" % c[:4] + ("".join("-%s%d" % kv for kv in sorted(c[4].items())))


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_tiled_coarse_and_vcycles_match_per_phase(case):
    import paper_1901_01685_amd as pmg
    _need_gpu()
    dim, p, nel, g, kw = case
    st = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, device=0, tiled_gs=1, **kw)
    sp = pmg.Solver(dim, p, nel, geometry=g, rhs_kind=g, device=0, tiled_gs=0, **kw)
    # on the 2-D unit box (Poisson) the tiled kernels form every level's
    # values from the level's 1-D factors, the per-phase kernels read them
    kron = dim == 2 and g == 0 and kw.get("pde", 0) == 0
    assert (st.info.coarse_kron_levels > 0) == kron
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    # the coarse solve alone (two h-multigrid cycles on the degree-1 problem)
    r1 = torch.tensor(rng.uniform(-1, 1, st.n1), device=dev)
    et, ep = torch.empty_like(r1), torch.empty_like(r1)
    st.coarse(r1, et)
    sp.coarse(r1, ep)
    torch.cuda.synchronize()
    assert torch.isfinite(et).all()
    assert torch.equal(et, ep)
    # whole V-cycles from a random start
    b = torch.empty(st.n, dtype=torch.float64, device=dev)
    st.rhs(b)
    x0 = torch.tensor(rng.uniform(-1, 1, st.n), device=dev)
    xt, xp = x0.clone(), x0.clone()
    rt, rp = torch.empty_like(b), torch.empty_like(b)
    st.residual(b, xt, rt)
    sp.residual(b, xp, rp)
    for it in range(3):
        nt = st.vcycle(b, xt, rt, norm=True)
        npp = sp.vcycle(b, xp, rp, norm=True)
        torch.cuda.synchronize()
        assert torch.equal(xt, xp) and torch.equal(rt, rp), it
        assert nt == npp
