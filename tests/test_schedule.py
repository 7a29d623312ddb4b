"""Host logic of the triangular solves (no GPU): the chunk schedule and the
chunk-sliced factors exported by the library, run through a CPU emulation of
what the kernels do.

* Deadlock freedom: a wave holding ticket k only waits for entries of chunks
  whose tickets are below k.  Running the chunks one after the other in
  ticket order must therefore find every entry it reads already final.
* Layout: replaying the kernels' arithmetic on the exported slots (gather
  over off-chunk slots, in-chunk recurrence on the staged tile, and for the
  upper factor the in-chunk values divided by their column's diagonal) gives
  the triangular solves of the exported L and U, as computed by scipy
  (stated tolerance 1e-13 relative: only the summation order differs).
* The dependency lists name exactly the chunks each chunk reads, and the
  previous chunk of the own segment is always among them.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import paper_1901_01685_amd as pmg

CASES = [(2, 2, 16), (2, 3, 40), (2, 5, 24), (3, 2, 12)]


def _emulate(s, factor, rhs):
    S = s.export_schedule(factor)
    nseg, seg = s.info.segments, s.info.seg_len
    nch = (seg + 63) // 64
    nq = nseg * nch
    upper = factor == 1
    order = S["order"]
    assert np.array_equal(np.sort(order), np.arange(nq)), "ticket order is not a permutation of the chunks"
    ticket = np.empty(nq, dtype=np.int64)
    ticket[order] = np.arange(nq)
    final = np.zeros(s.n, dtype=bool)
    out = np.zeros(s.n)
    for tk, q in enumerate(order):
        sg, c = divmod(int(q), nch)
        r0, nrow = sg * seg + c * 64, min(64, seg - c * 64)
        # dependency list: chunks of other tickets, all earlier
        W = S["waits"][S["wptr"][q]:S["wptr"][q + 1]]
        deps = set()
        for (sc, need) in W:
            dq = sc * nch + ((need - 1) // 64 if not upper else (seg - need) // 64)
            assert ticket[dq] < tk, "chunk %d waits for chunk %d taken later" % (q, dq)
            deps.add(int(dq))
        own_prev = (q - 1 if c > 0 else None) if not upper else (q + 1 if c < nch - 1 else None)
        if own_prev is not None:
            assert own_prev in deps, "chunk %d does not wait for its segment's previous chunk" % q
        w, base = S["off_w"][q], S["off_ptr"][q]
        t = np.zeros(64)
        t[:nrow] = rhs[r0:r0 + nrow]
        read = set()
        for u in range(w):
            cols = S["off_col"][base + u * 64: base + u * 64 + 64]
            vals = S["off_val"][base + u * 64: base + u * 64 + 64]
            for l in range(64):
                if cols[l] < 0:
                    assert vals[l] == 0.0
                    continue
                assert l < nrow
                col = int(cols[l])
                assert final[col], "ticket %d reads entry %d before it is final" % (tk, col)
                read.add((col // seg) * nch + (col % seg) // 64)
                t[l] -= vals[l] * out[col]
        assert read <= deps, "chunk %d reads chunks missing from its dependency list" % q
        tile = np.zeros((64, 64))
        ib = S["in_ptr"][q]
        for u in range(S["in_w"][q]):
            jj = S["in_j"][ib + u * 64: ib + u * 64 + 64]
            vv = S["in_val"][ib + u * 64: ib + u * 64 + 64]
            for l in range(64):
                if jj[l] >= 0:
                    assert l < nrow and 0 <= jj[l] < nrow
                    assert (jj[l] < l) if not upper else (jj[l] > l), "in-chunk entry on the wrong side"
                    tile[jj[l], l] = vv[l]
        steps = range(63) if not upper else range(63, 0, -1)
        for j in steps:
            t -= tile[j] * t[j]
        if upper:
            d = np.ones(64)
            d[:nrow] = S["diag"][r0:r0 + nrow]
            t = t / d
        out[r0:r0 + nrow] = t[:nrow]
        final[r0:r0 + nrow] = True
    assert final.all()
    # padding entries at the end of the sliced arrays
    assert np.all(S["off_col"][-64:] == -1) and np.all(S["off_val"][-64:] == 0)
    assert np.all(S["in_j"][-64:] == -1) and np.all(S["in_val"][-64:] == 0)
    return out


@pytest.mark.parametrize("case", CASES, ids=lambda c: "d%dp%dn%d" % c)
def test_schedule_is_deadlock_free_and_layout_solves(case):
    s = pmg.Solver(*case, device=-1)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(s.n)
    perm = s.export_perm()
    L = s.export(pmg.OP_L)
    U = s.export(pmg.OP_U)
    y = _emulate(s, 0, r[perm])
    y_ref = spla.spsolve_triangular((L + sp.eye(s.n)).tocsr(), r[perm], lower=True)
    assert np.linalg.norm(y - y_ref) <= 1e-13 * np.linalg.norm(y_ref)
    e = _emulate(s, 1, y)
    e_ref = spla.spsolve_triangular(U.tocsr(), y, lower=False)
    assert np.linalg.norm(e - e_ref) <= 1e-13 * np.linalg.norm(e_ref)


def test_chunk_order_is_by_level():
    """Tickets follow the level of the chunk dependency graph, so the waves in
    flight at any time work on the same few levels."""
    s = pmg.Solver(2, 3, 64, device=-1)
    for f in (0, 1):
        S = s.export_schedule(f)
        seg = s.info.seg_len
        nch = (seg + 63) // 64
        nq = s.info.segments * nch
        lev = np.zeros(nq, dtype=np.int64)
        for q in S["order"]:
            W = S["waits"][S["wptr"][q]:S["wptr"][q + 1]]
            if len(W):
                dq = W[:, 0] * nch + ((W[:, 1] - 1) // 64 if f == 0 else (seg - W[:, 1]) // 64)
                lev[q] = lev[dq].max() + 1
        assert np.all(np.diff(lev[S["order"]]) >= 0)
