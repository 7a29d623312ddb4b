"""GPU parity of every solve-phase step against the FP64 oracle, through the C
ABI.  Operators on both sides are built independently (library host setup vs
oracle); CPU tests pin that they agree to rounding with identical ILUT
patterns.  Tolerances: FP64 steps normwise 1e-12 relative (the only
differences are summation order and reciprocal scaling); whole solves by the
residual-history metric max_k ||r_k^gpu - r_k^orc|| / ||r_0|| <= 1e-10 and
iteration counts within one."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # (dim, p, nel, geom): several 64-row chunks per line, ragged tails
    (2, 2, 16, 0),     # the smallest workload: 256 unknowns, one partial chunk per line
    (2, 3, 128, 0),    # 129-row lines: 2 full chunks + 1-row tail
    (2, 5, 64, 0),     # 67-row lines
    (2, 4, 32, 1),     # quarter annulus
    (3, 2, 16, 0),     # unit cube
    (3, 3, 12, 0),
    # benchmark 2: non-symmetric CDR operator on the unit square (pde = 1)
    (2, 2, 16, 0, 1),
    (2, 4, 64, 0, 1),
    (2, 5, 128, 0, 1),  # degree-1 levels 127 and 63: tiled smoothing and the LDS cycle
]


def _id(c):
    return "d%dp%dn%dg%d" % c[:4] + ("cdr" if len(c) > 4 and c[4] else "")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


_cache = {}


def _pair(dim, p, nel, geom, pde=0, **kw):
    import paper_1901_01685_amd as pmg
    key = (dim, p, nel, geom, pde, tuple(sorted(kw.items())))
    if key not in _cache:
        s = pmg.Solver(dim, p, nel, geometry=geom, rhs_kind=geom, pde=pde, device=0, **kw)
        o = O.Oracle(dim, p, nel, geom=geom, rhs=geom, pde=pde)
        _cache[key] = (s, o)
    return _cache[key]


def _t(a, dev):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=dev)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_steps_match_oracle(case):
    dev = _dev()
    s, o = _pair(*case)
    print("case", case, "n", s.n, flush=True)
    rng = np.random.default_rng(11)
    n, n1 = s.n, s.n1
    b = o.f()
    x = rng.uniform(-1, 1, n)
    # a1: residual
    bt, xt, rt = _t(b, dev), _t(x, dev), torch.empty(n, dtype=torch.float64, device=dev)
    nrm = s.residual(bt, xt, rt, norm=True)
    r_or = o.residual(b, x)
    assert _rel(rt.cpu().numpy(), r_or) < 1e-12
    assert abs(nrm - np.linalg.norm(r_or)) <= 1e-12 * np.linalg.norm(r_or)
    # a2 + a3: ILUT smoothing step
    xs = xt.clone()
    s.smooth(_t(r_or, dev), xs)
    torch.cuda.synchronize()
    assert _rel(xs.cpu().numpy(), o.smooth(r_or, x)) < 1e-12
    # a4: restriction
    r1 = torch.empty(n1, dtype=torch.float64, device=dev)
    s.restrict(_t(r_or, dev), r1)
    r1_or = (o.R() @ r_or) / o.ml1()
    assert _rel(r1.cpu().numpy(), r1_or) < 1e-12
    # a5: coarse correction (h-multigrid)
    e1 = torch.empty(n1, dtype=torch.float64, device=dev)
    s.coarse(_t(r1_or, dev), e1)
    e1_or = o.coarse(r1_or)
    assert _rel(e1.cpu().numpy(), e1_or) < 1e-12
    # a6: prolongation
    xp = xt.clone()
    s.prolong(_t(e1_or, dev), xp)
    xp_or = x + (o.P() @ e1_or) / o.mlp()
    assert _rel(xp.cpu().numpy(), xp_or) < 1e-13
    # whole V-cycle
    xv = xt.clone()
    rv = _t(r_or, dev)
    nv = s.vcycle(bt, xv, rv, norm=True)
    xv_or, rv_or = o.vcycle(b, x, r_or)
    assert _rel(xv.cpu().numpy(), xv_or) < 1e-11
    assert np.linalg.norm(rv.cpu().numpy() - rv_or) <= 1e-10 * np.linalg.norm(r_or)
    assert abs(nv - np.linalg.norm(rv_or)) <= 1e-10 * np.linalg.norm(r_or)


@pytest.mark.parametrize("case", CASES, ids=_id)
@pytest.mark.parametrize("x0kind", ["zero", "random"])
def test_solve_history_matches_oracle(case, x0kind):
    dev = _dev()
    s, o = _pair(*case)
    print("case", case, x0kind, flush=True)
    n = s.n
    x0 = np.zeros(n) if x0kind == "zero" else np.random.default_rng(0).uniform(-1, 1, n)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    s.rhs(b)
    assert _rel(b.cpu().numpy(), o.f()) < 1e-13
    x = _t(x0, dev)
    st, it, rel, r0, _, hist = s.solve(b, x, tol=1e-8)
    xo, sto, ito, histo = o.solve(o.f(), x0=x0, tol=1e-8)
    assert st == 0 and sto == 0
    assert abs(it - ito) <= 1, (it, ito)
    k = min(len(hist), len(histo))
    assert np.abs(hist[:k] - histo[:k]).max() <= 1e-10, (hist, histo)
    assert hist[-1] <= 1e-8
    assert _rel(x.cpu().numpy(), xo) <= 1e-7


def test_edge_cases_status_codes():
    import paper_1901_01685_amd as pmg
    dev = _dev()
    s, o = _pair(2, 2, 16, 0)
    n = s.n
    # zero right-hand side and zero guess: converged before any V-cycle
    b = torch.zeros(n, dtype=torch.float64, device=dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    st, it, rel, r0, _, _ = s.solve(b, x)
    assert st == pmg.OK and it == 0 and r0 == 0.0
    # NaN in b
    b = torch.empty(n, dtype=torch.float64, device=dev)
    s.rhs(b)
    b[5] = float("nan")
    st, it, *_ = s.solve(b, x)
    assert st == pmg.ENAN and it == 0
    # max_iter
    s2 = pmg.Solver(2, 2, 16, device=0, max_iter=1)
    s2.rhs(b)
    st, it, rel, *_ = s2.solve(b, torch.zeros(n, dtype=torch.float64, device=dev), tol=1e-14)
    assert st == pmg.EMAXIT and it == 1 and 0 < rel < 1
    # initial guess = converged solution: V-cycles stay at the rounding floor
    # (the relative criterion cannot be met again, so the solve ends at max_iter)
    s.rhs(b)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    s.solve(b, x, tol=1e-13)
    r = torch.empty_like(b)
    rn0 = s.residual(b, x, r, norm=True)
    bn = float(torch.linalg.norm(b))
    assert rn0 <= 1e-12 * bn
    rn1 = s.vcycle(b, x, r, norm=True)
    assert rn1 <= 1e-12 * bn


def test_smallest_problem_single_level():
    """n_el <= 8: the degree-1 problem is solved directly (one level)."""
    dev = _dev()
    s, o = _pair(2, 3, 8, 1)
    assert s.info.nlev == 1
    b = torch.empty(s.n, dtype=torch.float64, device=dev)
    s.rhs(b)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    st, it, rel, r0, _, hist = s.solve(b, x, tol=1e-8)
    _, sto, ito, histo = o.solve(o.f(), tol=1e-8)
    k = min(len(hist), len(histo))
    assert st == 0 and abs(it - ito) <= 1 and np.abs(hist[:k] - histo[:k]).max() <= 1e-10


def test_repeated_solves_are_bitwise_reproducible():
    dev = _dev()
    s, _ = _pair(2, 5, 64, 0)
    b = torch.empty(s.n, dtype=torch.float64, device=dev)
    s.rhs(b)
    outs = []
    for _ in range(3):
        x = torch.zeros(s.n, dtype=torch.float64, device=dev)
        st, it, rel, *_ = s.solve(b, x, tol=1e-10)
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
