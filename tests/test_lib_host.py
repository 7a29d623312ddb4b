"""CPU tests of the library: the C ABI is exported as declared in
include/pmg.h, the host setup (assembly, lumping, transfers, degree-1
hierarchy, ILUT) agrees with the independently written oracle, and the
argument checks return the documented status codes.  No device is touched:
handles are set up with device = -1 (host-only)."""
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1901_01685_amd as P

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pmg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^\s*(?:pmg_status|double|const char\s*\*)\s*(pmg_\w+)\s*\(", src, flags=re.M))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "pmg_setup" in names and "pmg_solve" in names and len(names) >= 15
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    assert names == set(P.SIGNATURES), names ^ set(P.SIGNATURES)


def _rel(a, b):
    a = a.toarray() if hasattr(a, "toarray") else np.asarray(a)
    b = b.toarray() if hasattr(b, "toarray") else np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _same_pattern(a, b):
    a.sort_indices(); b.sort_indices()
    return np.array_equal(a.indptr, b.indptr) and np.array_equal(a.indices, b.indices)


SETUP_CASES = [(2, 2, 16, 0), (2, 3, 32, 0), (2, 5, 16, 1), (2, 4, 32, 1), (3, 2, 8, 0),
               (3, 2, 16, 0), (3, 3, 12, 0), (2, 5, 64, 0)]


@pytest.mark.parametrize("case", SETUP_CASES, ids=lambda c: "d%dp%dn%dg%d" % c)
def test_host_setup_matches_oracle(case):
    dim, p, nel, g = case
    s = P.Solver(dim, p, nel, geometry=g, rhs_kind=g, device=-1)
    o = O.Oracle(dim, p, nel, geom=g, rhs=g)
    assert (s.n, s.n1, s.info.nlev) == (o.n, o.n1, o.nlev)
    assert _same_pattern(s.export(P.OP_A), o.A()) and _rel(s.export(P.OP_A), o.A()) < 1e-13
    assert _rel(s.export_vec(P.VEC_F), o.f()) < 1e-13
    assert _rel(s.export_vec(P.VEC_MLP), o.mlp()) < 1e-13
    assert _rel(s.export_vec(P.VEC_ML1), o.ml1()) < 1e-13
    assert _same_pattern(s.export(P.OP_R), o.R()) and _rel(s.export(P.OP_R), o.R()) < 1e-13
    assert _same_pattern(s.export(P.OP_P), o.P()) and _rel(s.export(P.OP_P), o.P()) < 1e-13
    for lev in range(o.nlev):
        assert _rel(s.export(P.OP_A1, lev), o.A1(lev)) < 1e-13
    for lev in range(o.nlev - 1):
        assert _rel(s.export(P.OP_PH, lev), o.Ph(lev)) == 0.0
    C = o.chol()
    inv = np.linalg.inv(C @ C.T)
    nc = C.shape[0]
    assert _rel(s.export_vec(P.VEC_COARSE_INV).reshape(nc, nc), inv) < 1e-12
    # ILUT ordering and factors: identical permutation and patterns, values to rounding
    assert np.array_equal(s.export_perm(), o.perm())
    for a, b in ((s.export(P.OP_L), o.L()), (s.export(P.OP_U), o.U())):
        assert _same_pattern(a, b)
        assert _rel(a, b) < 1e-12


def test_ilut_independent_of_thread_count():
    a = P.Solver(2, 4, 48, geometry=1, rhs_kind=1, device=-1, setup_threads=1)
    b = P.Solver(2, 4, 48, geometry=1, rhs_kind=1, device=-1, setup_threads=7)
    for op in (P.OP_L, P.OP_U):
        x, y = a.export(op), b.export(op)
        assert np.array_equal(x.indptr, y.indptr) and np.array_equal(x.indices, y.indices)
        assert np.array_equal(x.data, y.data)


@pytest.mark.parametrize("ordering", [0, 1])
def test_orderings_match_oracle(ordering):
    for (dim, p, nel) in [(2, 3, 40), (3, 2, 14), (2, 5, 100)]:
        s = P.Solver(dim, p, nel, device=-1, ordering=ordering)
        o = O.Oracle(dim, p, nel, opts=O.Options(ordering=ordering), ilut=False)
        assert np.array_equal(s.export_perm(), o.perm())


def test_info_sizes_and_bytes():
    s = P.Solver(2, 5, 64, device=-1, ordering=0)
    i = s.info
    assert i.n == (64 + 5 - 2) ** 2 and i.n1 == 63 ** 2
    assert i.seg_len == 67 and i.segments == 67
    # lower bound on the natural-order DAG depth of the ILU(0) pattern
    assert i.dag_levels_l >= (5 + 2) * (67 - 1) + 1
    # on the box the residual forms A's coefficients from the 1-D factors of
    # its Kronecker sum (two bands of 67 x 11 entries) and reads the vectors
    assert i.residual_layout == 2 and i.bytes_spmv == 2 * 8 * 67 * 11 + 24 * i.n
    # otherwise it reads A in stencil layout (8 bytes per offset slot, 11^2
    # slots per row) when that is fewer bytes than CSR (12 per non-zero)
    k = P.Solver(2, 5, 64, device=-1, ordering=0, kron_residual=0).info
    stencil = 8 * 11 ** 2 * k.n + 24 * k.n
    csr = 12 * k.nnz_a + 4 * (k.n + 1) + 24 * k.n
    assert k.residual_layout == 1 and stencil < csr and k.bytes_spmv == stencil
    assert k.bytes_vcycle > 3 * k.bytes_spmv
    # on a small 3-D grid the zero slots at the boundary make CSR cheaper
    j = P.Solver(3, 3, 8, device=-1, kron_residual=0).info
    assert j.residual_layout == 0 and j.bytes_spmv == 12 * j.nnz_a + 4 * (j.n + 1) + 24 * j.n
    assert P.Solver(3, 3, 8, device=-1).info.residual_layout == 2
    # a residual thread takes one row on these small grids (four only where
    # that still leaves three waves per SIMD of the 256 CUs); none with CSR
    assert i.resid_rows == 1 and k.resid_rows == 1 and j.resid_rows == 0


def test_status_codes_host():
    with pytest.raises(P.PmgError) as e:
        P.Solver(4, 2, 16, device=-1)
    assert e.value.status == P.EINVAL
    with pytest.raises(P.PmgError) as e:
        P.Solver(3, 2, 16, geometry=P.GEOM_QUARTER_ANNULUS, device=-1)
    assert e.value.status == P.EINVAL
    # 26 -> 13 stops at the odd mesh: 12^2 = 144 unknowns is fine in 2-D ...
    s = P.Solver(2, 2, 26, device=-1)
    assert s.info.nlev == 2 and s.info.n_coarsest == 144
    with pytest.raises(P.PmgError) as e:
        P.Solver(3, 2, 26, device=-1)           # ... but 12^3 = 1728 exceeds the limit in 3-D
    assert e.value.status == P.EINVAL
    s = P.Solver(2, 2, 16, device=-1)
    st = P.lib().pmg_solve(s._h, None, None, 1e-8, None, None, None)
    assert st == P.EDEVICE
    assert P.lib().pmg_get_info(None, None) == P.EINVAL
    assert P.lib().pmg_status_str(P.EZEROPIVOT) == b"zero pivot in ILUT"


@pytest.mark.parametrize("case", [(2, 16), (3, 32), (5, 16), (4, 64)], ids=lambda c: "p%dn%d" % c)
def test_host_setup_matches_oracle_cdr(case):
    """Benchmark 2 (CDR operator): the library's Kronecker assembly against the
    oracle's element loop, at degree p and on every degree-1 level, the load
    vector of the CDR right-hand side, the non-symmetric coarsest inverse, and
    the ILUT factors of the non-symmetric operator."""
    p, nel = case
    s = P.Solver(2, p, nel, pde=P.PDE_CDR, device=-1)
    o = O.Oracle(2, p, nel, pde=O.PDE_CDR)
    A = s.export(P.OP_A)
    assert _same_pattern(A, o.A()) and _rel(A, o.A()) < 1e-13
    assert abs(A - A.T).max() > 1e-3 * abs(A).max()      # genuinely non-symmetric
    assert _rel(s.export_vec(P.VEC_F), o.f()) < 1e-12
    for lev in range(o.nlev):
        assert _rel(s.export(P.OP_A1, lev), o.A1(lev)) < 1e-13
    nc = o.level_n[o.nlev - 1]
    inv = np.linalg.inv(o.A1(o.nlev - 1).toarray())
    assert _rel(s.export_vec(P.VEC_COARSE_INV).reshape(nc, nc), inv) < 1e-11
    assert np.array_equal(s.export_perm(), o.perm())
    for a, b in ((s.export(P.OP_L), o.L()), (s.export(P.OP_U), o.U())):
        assert _same_pattern(a, b)
        assert _rel(a, b) < 1e-12


def test_cdr_configurations_checked():
    for kw in ({"dim": 3, "degree": 2, "n_elem": 8}, {"dim": 2, "degree": 2, "n_elem": 8, "geometry": 1, "rhs_kind": 1}):
        with pytest.raises(P.PmgError) as e:
            P.Solver(pde=P.PDE_CDR, device=-1, **kw)
        assert e.value.status == P.EINVAL
    with pytest.raises(P.PmgError) as e:
        P.Solver(2, 2, 8, pde=7, device=-1)
    assert e.value.status == P.EINVAL


def test_mass_transfer_options_checked():
    with pytest.raises(P.PmgError) as e:
        P.Solver(2, 2, 8, mass_transfer=2, device=-1)
    assert e.value.status == P.EINVAL
    with pytest.raises(P.PmgError) as e:       # consistent masses run in FP64 only
        P.Solver(2, 2, 8, mass_transfer=P.MASS_CONSISTENT, precision=P.FP32_IN_FP64, device=-1)
    assert e.value.status == P.EINVAL
    s = P.Solver(2, 3, 16, geometry=1, rhs_kind=1, mass_transfer=P.MASS_CONSISTENT, device=-1)
    assert s.options.mass_transfer == P.MASS_CONSISTENT


@pytest.mark.parametrize("case", [(2, 3, 16, 0), (2, 4, 16, 1), (3, 3, 6, 0)], ids=lambda c: "d%dp%dn%dg%d" % c)
def test_host_setup_matches_oracle_indirect(case):
    """Indirect projection (Appendix A): the degree-p level transfers to
    degree p-1 (transfer matrix and lumped masses against the oracle's), has
    no degree-1 hierarchy of its own, and the options are checked."""
    dim, p, nel, g = case
    s = P.Solver(dim, p, nel, geometry=g, rhs_kind=g, projection=P.PROJ_INDIRECT, device=-1)
    o = O.Oracle(dim, p, nel, geom=g, rhs=g, opts=O.Options(projection=1), ilut=False)
    assert s.n1 == o.n1 == (nel + p - 3) ** dim
    assert s.info.nlev == 0
    assert _same_pattern(s.export(P.OP_P), o.P()) and _rel(s.export(P.OP_P), o.P()) < 1e-13
    assert _same_pattern(s.export(P.OP_R), o.R()) and _rel(s.export(P.OP_R), o.R()) < 1e-13
    assert _rel(s.export_vec(P.VEC_ML1), o.ml1()) < 1e-13
    with pytest.raises(P.PmgError) as e:
        P.Solver(2, 3, 8, projection=5, device=-1)
    assert e.value.status == P.EINVAL
