"""Residual and p-transfers from Kronecker factors on the unit box
(pmg_options.kron_residual): the coefficients of A = sum over directions of
(1-D stiffness) x (1-D mass), and of the transfers P = X x X and R = P^T, are
formed in the kernels from the 1-D factors with the assembly's products and
sums, so they equal the stored values and the residual, the V-cycle and whole
solves agree bit for bit with the stencil layouts that read them (FP64 and
FP32-in-FP64; 2-D and 3-D; every unrolled stencil width).  Problems that are
not Kronecker sums (annulus; benchmark 2's operator) keep the stencil layout
for A."""
import numpy as np
import pytest

import paper_1901_01685_amd as pmg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [(2, 2, 16), (2, 3, 40), (2, 4, 24), (2, 5, 64), (3, 2, 12), (3, 3, 16)]


@pytest.mark.parametrize("dim,p,nel", CASES)
def test_kron_residual_equals_the_stencil_residual_bitwise(dim, p, nel):
    dev = torch.device("cuda:0")
    k = pmg.Solver(dim, p, nel, device=0, kron_residual=1)
    s = pmg.Solver(dim, p, nel, device=0, kron_residual=0)
    assert k.info.residual_layout == 2 and s.info.residual_layout == 1
    assert k.info.resid_rows == 1 and s.info.resid_rows == 1
    assert k.info.transfer_layout == 2 and s.info.transfer_layout in (0, 1)
    assert k.info.bytes_spmv < s.info.bytes_spmv and k.info.bytes_restrict < s.info.bytes_restrict
    g = torch.Generator(device="cpu").manual_seed(dim * 100 + p * 10 + nel)
    x = torch.randn(k.n, generator=g, dtype=torch.float64).to(dev)
    b = torch.randn(k.n, generator=g, dtype=torch.float64).to(dev)
    rk, rs = torch.empty_like(b), torch.empty_like(b)
    nk = k.residual(b, x, rk, norm=True)
    ns = s.residual(b, x, rs, norm=True)
    torch.cuda.synchronize()
    assert torch.equal(rk, rs) and nk == ns
    # V-cycles (FP64) from the same start: the transfers formed from their
    # Kronecker factor agree bit for bit with the stencil layout (with CSR
    # transfers, chosen on some small grids, only to rounding)
    xk, xs = x.clone(), x.clone()
    for _ in range(2):
        k.vcycle(b, xk, rk, norm=True)
        s.vcycle(b, xs, rs, norm=True)
    torch.cuda.synchronize()
    if s.info.transfer_layout == 1:
        assert torch.equal(xk, xs)
    else:
        assert torch.allclose(xk, xs, rtol=1e-12, atol=1e-12 * float(xs.abs().max()))


@pytest.mark.parametrize("dim,p,nel", [(2, 5, 48), (3, 2, 12)])
def test_kron_residual_mixed_precision_solves_bitwise(dim, p, nel):
    dev = torch.device("cuda:0")
    k = pmg.Solver(dim, p, nel, device=0, kron_residual=1, precision=pmg.FP32_IN_FP64)
    s = pmg.Solver(dim, p, nel, device=0, kron_residual=0, precision=pmg.FP32_IN_FP64)
    b = torch.empty(k.n, dtype=torch.float64, device=dev)
    k.rhs(b)
    xk, xs = torch.zeros_like(b), torch.zeros_like(b)
    stk, itk, relk, *_ = k.solve(b, xk, tol=1e-10)
    sts, its, rels, *_ = s.solve(b, xs, tol=1e-10)
    assert stk == pmg.OK and sts == pmg.OK and itk == its and relk == rels
    assert torch.equal(xk, xs)


def test_non_kronecker_problems_keep_the_stencil_layout():
    a = pmg.Solver(2, 3, 32, device=0, geometry=pmg.GEOM_QUARTER_ANNULUS, rhs_kind=pmg.RHS_ANNULUS)
    c = pmg.Solver(2, 3, 32, device=0, pde=pmg.PDE_CDR)
    assert a.info.residual_layout != 2 and c.info.residual_layout != 2
    # benchmark 2's transfers are the box's: they keep their Kronecker factor
    assert a.info.transfer_layout != 2 and c.info.transfer_layout == 2


@pytest.mark.parametrize("dim,p,nel", [(2, 5, 48), (3, 2, 16)])
def test_kron_products_in_bicgstab_bitwise(dim, p, nel):
    """BiCGSTAB's products with A (r = A x, no right-hand side) take the same
    Kronecker path."""
    dev = torch.device("cuda:0")
    k = pmg.Solver(dim, p, nel, device=0, kron_residual=1)
    s = pmg.Solver(dim, p, nel, device=0, kron_residual=0)
    assert k.info.residual_layout == 2 and s.info.residual_layout == 1
    b = torch.empty(k.n, dtype=torch.float64, device=dev)
    k.rhs(b)
    xk, xs = torch.zeros_like(b), torch.zeros_like(b)
    stk, itk, relk, *_ = k.bicgstab(b, xk, tol=1e-10)
    sts, its, rels, *_ = s.bicgstab(b, xs, tol=1e-10)
    assert stk == pmg.OK and sts == pmg.OK and itk == its and relk == rels
    assert torch.equal(xk, xs)


def test_four_rows_per_thread_on_a_large_grid():
    """On a grid large enough that a residual thread takes four rows in y
    (p = 3, h = 1/896: 897 lines, not a multiple of four), both layouts agree bit for
    bit, FP64 and FP32, and the residual matches the host product with the
    exported A to summation order."""
    dev = torch.device("cuda:0")
    k = pmg.Solver(2, 3, 896, device=0, kron_residual=1, precision=pmg.FP32_IN_FP64)
    s = pmg.Solver(2, 3, 896, device=0, kron_residual=0, precision=pmg.FP32_IN_FP64)
    assert k.info.residual_layout == 2 and s.info.residual_layout == 1
    assert k.info.resid_rows == 4 and s.info.resid_rows == 4
    print("four rows per thread: n", k.n, flush=True)
    g = torch.Generator(device="cpu").manual_seed(896)
    xh = torch.rand(k.n, generator=g, dtype=torch.float64) * 2 - 1
    bh = torch.rand(k.n, generator=g, dtype=torch.float64) * 2 - 1
    x, b = xh.to(dev), bh.to(dev)
    rk, rs = torch.empty_like(b), torch.empty_like(b)
    nk = k.residual(b, x, rk, norm=True)
    ns = s.residual(b, x, rs, norm=True)
    torch.cuda.synchronize()
    assert torch.equal(rk, rs) and nk == ns
    A = s.export(pmg.OP_A).tocsr()
    r_ref = bh.numpy() - A @ xh.numpy()
    assert np.linalg.norm(rk.cpu().numpy() - r_ref) <= 1e-12 * np.linalg.norm(r_ref)
    assert abs(nk - np.linalg.norm(r_ref)) <= 1e-12 * np.linalg.norm(r_ref)
    # FP32 V-cycles inside FP64 defect correction: the float kernels
    k.rhs(b)
    xk, xs = torch.zeros_like(b), torch.zeros_like(b)
    stk, itk, relk, *_ = k.solve(b, xk, tol=1e-10)
    sts, its, rels, *_ = s.solve(b, xs, tol=1e-10)
    assert stk == pmg.OK and sts == pmg.OK and itk == its and relk == rels
    assert torch.equal(xk, xs)
