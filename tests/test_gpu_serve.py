"""Request server (continuous batching): every result is checked against the
FP64 oracle (relative residual of the returned x <= 1e-10, recomputed by the
oracle), a request gives the same solution alone and inside a mix of other
classes (stated tolerance: bitwise, since every reduction has a fixed order
and each slot has its own workspace), requests overlap on the device,
classes above the budget are rejected, and least recently used idle classes
are evicted and set up again when memory is needed."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_oracles = {}


def _oracle_relres(dim, p, nel, geom, freq, x):
    key = (dim, p, nel, geom)
    if key not in _oracles:
        _oracles[key] = O.Oracle(dim, p, nel, geom=geom, rhs=0, ilut=False)
    o = _oracles[key]
    # right-hand side of this request's frequencies
    of = O.Oracle(dim, p, nel, geom=geom, rhs=0, freq=freq, ilut=False).f() if tuple(freq) != (1, 1, 1) else o.f()
    return np.linalg.norm(o.residual(of, x)) / np.linalg.norm(of)


MIX = [  # (dim, p, nel, geom, freq)
    (2, 3, 32, 0, (2, 1, 1)),
    (3, 2, 12, 0, (1, 3, 2)),
    (2, 5, 32, 1, (1, 1, 1)),
    (2, 2, 64, 0, (4, 4, 1)),
    (2, 4, 16, 0, (3, 1, 1)),
    (3, 3, 8, 0, (2, 2, 2)),
    (2, 3, 32, 0, (2, 1, 1)),   # same class and right-hand side as the first
    (2, 2, 32, 1, (1, 1, 1)),
    (3, 2, 16, 0, (1, 1, 4)),
    (2, 5, 16, 0, (1, 2, 1)),
]


def test_alone_and_in_the_mix_agree_and_match_oracle():
    import paper_1901_01685_amd as pmg
    _need_gpu()
    srv = pmg.Server(max_slots=4)
    try:
        # alone
        dim, p, nel, g, fr = MIX[0]
        st, t = srv.submit(dim, p, nel, g, freq=fr)
        assert st == pmg.OK
        st, info, x_alone = srv.wait(t)
        assert st == pmg.OK and info["relres"] <= 1e-10
        print("alone:", info, flush=True)
        # in a mix of ten requests of eight classes, all in flight together
        tickets = []
        for (dim, p, nel, g, fr) in MIX:
            st, t = srv.submit(dim, p, nel, g, freq=fr)
            assert st == pmg.OK
            tickets.append(t)
        results = [srv.wait(t) for t in tickets]
        for (case, (st, info, x)) in zip(MIX, results):
            dim, p, nel, g, fr = case
            assert st == pmg.OK, (case, info)
            assert info["relres"] <= 1e-10
            rel = _oracle_relres(dim, p, nel, g, fr, x)
            print(case, "outer", info["iterations"], "relres", info["relres"], "oracle", rel,
                  "latency %.2f ms" % (1e3 * (info["t_finish"] - info["t_submit"])), flush=True)
            assert rel <= 1.01e-10
        # same request alone and in the mix: identical solutions
        assert np.array_equal(results[0][2], x_alone)
        assert np.array_equal(results[6][2], x_alone)
        # requests in flight together share the slots: a burst of requests of a
        # resident class with right-hand sides given by the caller (so every
        # submit returns at once) is admitted side by side, and equal inputs
        # give equal results whatever the company
        dim, p, nel, g, fr = MIX[0]
        rng = np.random.default_rng(2)
        bs = [rng.uniform(-1, 1, (nel + p - 2) ** dim) for _ in range(2)]
        burst = [srv.submit(dim, p, nel, g, b=bs[k % 2]) for k in range(6)]
        assert all(st == pmg.OK for st, _ in burst)
        out = [srv.wait(t) for _, t in burst]
        assert all(st == pmg.OK and info["relres"] <= 1e-10 for st, info, _ in out)
        for k in range(2, 6):
            assert np.array_equal(out[k][2], out[k % 2][2])
        infos = [info for _, info, _ in out]
        assert any(a["t_admit"] < b["t_finish"] and b["t_admit"] < a["t_finish"]
                   for i, a in enumerate(infos) for b in infos[i + 1:])
        stt = srv.stats()
        assert stt["completed"] == len(MIX) + 1 + len(burst) and stt["failed"] == 0
    finally:
        srv.close()


def test_budget_rejection_and_eviction():
    import paper_1901_01685_amd as pmg
    _need_gpu()
    # small budget: a 3-D p = 5, h = 1/64 class (estimated ~20 GB) is rejected
    srv = pmg.Server(max_slots=2, budget_bytes=200 << 20, max_class_bytes=120 << 20)
    try:
        st, t = srv.submit(3, 5, 64)
        assert st == pmg.EBUDGET and t == -1
        # classes of ~50-90 MB each: the budget holds only a few, so older idle
        # classes are evicted and set up again later; results stay correct
        seq = [(2, 4, 128), (2, 5, 96), (2, 3, 160), (2, 4, 128), (2, 5, 96)]
        xs = []
        for (dim, p, nel) in seq:
            st, t = srv.submit(dim, p, nel)
            assert st == pmg.OK
            st, info, x = srv.wait(t)
            assert st == pmg.OK and info["relres"] <= 1e-10
            xs.append(x)
        stt = srv.stats()
        print(stt, flush=True)
        assert stt["rejected"] == 1
        assert stt["evictions"] >= 1
        assert stt["bytes_in_use"] <= 200 << 20
        # a class set up again gives the same solution as before
        assert np.array_equal(xs[0], xs[3]) and np.array_equal(xs[1], xs[4])
    finally:
        srv.close()


def test_fp64_single_slot_mode():
    import paper_1901_01685_amd as pmg
    _need_gpu()
    srv = pmg.Server(max_slots=4)
    try:
        srv.configure(1, pmg.FP64)
        st, t = srv.submit(2, 4, 32, freq=(1, 2, 1))
        assert st == pmg.OK
        st, info, x = srv.wait(t)
        assert st == pmg.OK and info["relres"] <= 1e-10
        assert _oracle_relres(2, 4, 32, 0, (1, 2, 1), x) <= 1.01e-10
    finally:
        srv.close()


def test_cdr_requests_are_their_own_class():
    """Benchmark 2 requests share (dim, p, n_el, geometry) with Poisson ones but
    not the operator: the class key includes the pde, and each result matches
    its own oracle."""
    import paper_1901_01685_amd as pmg
    _need_gpu()
    srv = pmg.Server(max_slots=2)
    try:
        t_p = srv.submit(2, 3, 32)[1]
        t_c = srv.submit(2, 3, 32, pde=pmg.PDE_CDR)[1]
        (st_p, info_p, x_p), (st_c, info_c, x_c) = srv.wait(t_p), srv.wait(t_c)
        assert st_p == pmg.OK and st_c == pmg.OK
        assert srv.stats()["classes_resident"] >= 2
        o = O.Oracle(2, 3, 32, pde=O.PDE_CDR, ilut=False)
        f = o.f()
        assert np.linalg.norm(o.residual(f, x_c)) <= 1.01e-10 * np.linalg.norm(f)
        assert _oracle_relres(2, 3, 32, 0, (1, 1, 1), x_p) <= 1.01e-10
    finally:
        srv.close()


def test_effective_options_take_the_budget_from_the_device():
    import paper_1901_01685_amd as pmg
    _need_gpu()
    total = torch.cuda.get_device_properties(0).total_memory
    srv = pmg.Server(max_slots=3)
    try:
        o = srv.effective_options()
        # 70 % of the device's memory, a quarter of it per class, one wave per
        # CU per slot grid; the requested fields unchanged
        assert abs(o.budget_bytes - 0.7 * total) <= 1 << 20, (o.budget_bytes, total)
        assert o.max_class_bytes == o.budget_bytes // 4
        assert o.tri_waves_per_cu == 1 and o.max_slots == 3 and o.precision == pmg.FP32_IN_FP64
    finally:
        srv.close()
    srv = pmg.Server(max_slots=2, budget_bytes=300 << 20, max_class_bytes=100 << 20, tri_waves_per_cu=0)
    try:
        o = srv.effective_options()
        assert o.budget_bytes == 300 << 20 and o.max_class_bytes == 100 << 20 and o.tri_waves_per_cu == 0
        st, t = srv.submit(2, 3, 32)
        assert st == pmg.OK
        st, info, _ = srv.wait(t)
        assert st == pmg.OK and info["relres"] <= 1e-10
    finally:
        srv.close()
    with pytest.raises(pmg.PmgError) as e:
        pmg.Server(tri_waves_per_cu=-1)
    assert e.value.status == pmg.EINVAL
