"""Pins of the oracle's convection-diffusion-reaction operator (benchmark 2 of
Section 2: unit square, D = [1.2 -0.7; -0.4 0.9], v = (0.4, -0.2), R = 0.3,
u = sin(pi x) sin(pi y)).

What fixes it independently of the oracle's own formulas:
  * the closed-form right-hand side against central differences of the exact
    solution pushed through the differential operator;
  * the Galerkin solution converging to the exact solution at the optimal L2
    rate h^(p+1) (a wrong sign or size of any coefficient, or a transposed
    convection term, converges to another function and stalls);
  * coercivity: D's symmetric part is positive definite and R > 0, while the
    convection form is skew on H^1_0, so the symmetric part of A is positive
    definite and A itself is not symmetric;
  * the paper's iteration counts for benchmark 2 (Tables 4 and 5)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_vcycles.json")
D = np.array([[1.2, -0.7], [-0.4, 0.9]])
V = np.array([0.4, -0.2])
R = 0.3


def _u(k, x, y):
    return np.sin(k[0] * np.pi * x) * np.sin(k[1] * np.pi * y)


@pytest.mark.parametrize("k", [(1, 1), (2, 1), (1, 3)])
def test_rhs_is_the_operator_applied_to_the_solution(k):
    rng = np.random.default_rng(1)
    h = 1e-4
    for x, y in rng.uniform(0.05, 0.95, (20, 2)):
        uxx = (_u(k, x + h, y) - 2 * _u(k, x, y) + _u(k, x - h, y)) / h**2
        uyy = (_u(k, x, y + h) - 2 * _u(k, x, y) + _u(k, x, y - h)) / h**2
        uxy = (_u(k, x + h, y + h) - _u(k, x + h, y - h) - _u(k, x - h, y + h) + _u(k, x - h, y - h)) / (4 * h**2)
        ux = (_u(k, x + h, y) - _u(k, x - h, y)) / (2 * h)
        uy = (_u(k, x, y + h) - _u(k, x, y - h)) / (2 * h)
        fd = -(D[0, 0] * uxx + (D[0, 1] + D[1, 0]) * uxy + D[1, 1] * uyy) + V[0] * ux + V[1] * uy + R * _u(k, x, y)
        f = O.cdr_f(k, (x, y))
        assert abs(f - fd) <= 2e-5 * max(1.0, abs(f)), (k, x, y, f, fd)


@pytest.mark.parametrize("p", [2, 3])
def test_galerkin_solution_converges_at_rate_p_plus_1(p):
    errs = []
    for nel in (8, 16, 32):
        o = O.Oracle(2, p, nel, pde=O.PDE_CDR, ilut=False)
        u = spla.spsolve(o.A().tocsc(), o.f())
        errs.append(o.l2_error(u))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(r >= p + 1 - 0.3 for r in rates), (p, errs, rates)


def test_symmetric_part_positive_definite_and_operator_not_symmetric():
    o = O.Oracle(2, 2, 8, pde=O.PDE_CDR, ilut=False)
    A = o.A().toarray()
    S, K = (A + A.T) / 2, (A - A.T) / 2
    assert np.linalg.eigvalsh(S).min() > 0
    assert np.abs(K).max() > 1e-3 * np.abs(A).max()
    # the Poisson operator of the same space stays symmetric
    P = O.Oracle(2, 2, 8, ilut=False).A().toarray()
    assert np.abs(P - P.T).max() <= 1e-14 * np.abs(P).max()


def test_degree1_hierarchy_uses_the_same_operator():
    o = O.Oracle(2, 2, 32, pde=O.PDE_CDR, ilut=False)
    for lev in range(o.nlev):
        A1 = o.A1(lev).toarray()
        assert np.abs(A1 - A1.T).max() > 0, lev
        assert np.linalg.eigvalsh((A1 + A1.T) / 2).min() > 0, lev


def test_paper_iteration_counts_benchmark_2():
    gold = json.load(open(GOLD))
    g4, g5 = gold["cdr"], gold["bicgstab_cdr"]
    for p in (2, 3, 4, 5):
        o = O.Oracle(2, p, 64, pde=O.PDE_CDR)
        x0 = np.random.default_rng(0).uniform(-1, 1, o.n)
        _, st, it, _ = o.solve(o.f(), x0=x0, tol=1e-8)
        paper = g4["ilut"][g4["h"].index(64)][g4["p"].index(p)]
        assert st == 0 and abs(it - paper) <= 2, ("vcycles", p, it, paper)
        _, st, it, _ = o.bicgstab(o.f(), x0=x0, tol=1e-8)
        paper = g5["ilut"][g5["h"].index(64)][g5["p"].index(p)]
        assert st == 0 and abs(it - paper) <= 1, ("bicgstab", p, it, paper)


def test_invalid_cdr_configurations_rejected():
    for kw in ({"dim": 3, "p": 2, "nel": 4}, {"dim": 2, "p": 2, "nel": 8, "geom": 1, "rhs": 1}):
        dim, p, nel = kw.pop("dim"), kw.pop("p"), kw.pop("nel")
        with pytest.raises(ValueError):
            O.Oracle(dim, p, nel, pde=O.PDE_CDR, ilut=False, **kw)
