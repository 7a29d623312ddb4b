"""Fault paths of the triangular solves and of the device ILUT
(include/pmg.h, pmg_options.poll_limit).

A wave that waits longer than its poll bound for an entry of another chunk
marks the solve as faulted and stops waiting, and so does every other wave,
so the kernels end; the next synchronising call returns PMG_EDEVICE.  The
bound is forced down from the host (poll_limit = 1: a wave that still finds
a pending entry after one reload gives up) on a problem whose schedule makes
waves wait, natural ordering, where nearly every chunk waits on the line
before it and nearly every ILUT row on the row before it.  The solve test
factors on the host so that only the solve meets the small bound.  Nothing
faults the GPU: every kernel exits normally.
"""
import numpy as np
import pytest
import torch

import paper_1901_01685_amd as pmg

pytestmark = pytest.mark.gpu


def test_poll_bound_reports_edevice_and_the_handle_recovers():
    dev = torch.device("cuda:0")
    s = pmg.Solver(2, 3, 64, device=0, poll_limit=1, ordering=pmg.ORDER_NATURAL, ilut_on_device=0)
    b = torch.empty(s.n, dtype=torch.float64, device=dev)
    s.rhs(b)
    x = torch.zeros(s.n, dtype=torch.float64, device=dev)
    st, *_ = s.solve(b, x, tol=1e-8, check=False)
    assert st == pmg.EDEVICE, st
    assert "poll bound" in pmg.lib().pmg_last_error().decode()
    # the fault word was cleared and the counters reset: a call without a
    # triangular solve synchronises cleanly on the same handle
    r = torch.empty_like(b)
    nrm = s.residual(b, torch.zeros_like(b), r, norm=True)
    assert np.isclose(nrm, torch.linalg.vector_norm(b).item(), rtol=1e-12)
    # the default bound on the same problem converges as usual
    t = pmg.Solver(2, 3, 64, device=0, ordering=pmg.ORDER_NATURAL)
    x.zero_()
    st, it, rel, *_ = t.solve(b, x, tol=1e-8)
    assert st == pmg.OK and rel <= 1e-8, (st, rel)


def test_negative_poll_limit_is_rejected():
    with pytest.raises(pmg.PmgError) as e:
        pmg.Solver(2, 2, 8, device=0, poll_limit=-1)
    assert e.value.status == pmg.EINVAL


def test_device_ilut_poll_bound_fails_setup_and_the_device_recovers():
    with pytest.raises(pmg.PmgError) as e:
        pmg.Solver(2, 3, 64, device=0, poll_limit=1, ordering=pmg.ORDER_NATURAL, ilut_on_device=1)
    assert e.value.status == pmg.EDEVICE, e.value
    assert "poll bound" in str(e.value)
    # the kernel ended normally: the next setup on the device factors as usual
    t = pmg.Solver(2, 3, 64, device=0, ordering=pmg.ORDER_NATURAL, ilut_on_device=1)
    assert t.info.ilut_on_device == 1
    b = torch.empty(t.n, dtype=torch.float64, device="cuda:0")
    t.rhs(b)
    x = torch.zeros_like(b)
    st, it, rel, *_ = t.solve(b, x, tol=1e-8)
    assert st == pmg.OK and rel <= 1e-8, (st, rel)
