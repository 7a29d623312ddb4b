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
    line = s.info.seg_len
    upper = factor == 1
    row0, nrows = S["chunk_row"], S["chunk_len"]
    nq = len(row0)
    assert nq == (s.info.chunks_u if upper else s.info.chunks_l)
    # segments are runs of whole grid lines covering the rows
    ss = S["seg_start"]
    assert len(ss) == s.info.segments + 1 and ss[0] == 0 and ss[-1] == s.n
    assert np.all(np.diff(ss) > 0) and np.all(ss % line == 0)
    segof = lambda r: np.searchsorted(ss, r, side="right") - 1
    # chunks tile the rows, never cross a segment, hold at most 64 rows
    assert row0[0] == 0 and np.all(row0[1:] == row0[:-1] + nrows[:-1]) and row0[-1] + nrows[-1] == s.n
    assert np.all((nrows >= 1) & (nrows <= 64))
    assert np.all(segof(row0) == segof(row0 + nrows - 1))
    row_chunk = np.repeat(np.arange(nq), nrows)
    order = S["order"]
    assert np.array_equal(np.sort(order), np.arange(nq)), "ticket order is not a permutation of the chunks"
    ticket = np.empty(nq, dtype=np.int64)
    ticket[order] = np.arange(nq)
    final = np.zeros(s.n, dtype=bool)
    out = np.zeros(s.n)
    for tk, q in enumerate(order):
        r0, nrow = int(row0[q]), int(nrows[q])
        sg = segof(r0)
        # dependency list: chunks of other tickets, all earlier
        deps = set(int(d) for d in S["deps"][S["wptr"][q]:S["wptr"][q + 1]])
        for dq in deps:
            assert ticket[dq] < tk, "chunk %d waits for chunk %d taken later" % (q, dq)
        own_prev = q - 1 if not upper else q + 1
        if 0 <= own_prev < nq and segof(row0[own_prev]) == sg:
            assert own_prev in deps, "chunk %d does not wait for its segment's previous chunk" % q
        w, base = S["off_w"][q], S["off_ptr"][q]
        if w:
            # each row's entries fill its last slots: no padding after an entry
            cw = S["off_col"][base:base + 64 * w].reshape(w, 64)
            seen = np.maximum.accumulate(cw >= 0, axis=0)
            assert not np.any(seen & (cw < 0)), "chunk %d: off-chunk slots are not right-aligned" % q
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
                read.add(int(row_chunk[col]))
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
    flight at any time work on the same few levels; the reported depth is
    that graph's."""
    s = pmg.Solver(2, 3, 64, device=-1)
    for f in (0, 1):
        S = s.export_schedule(f)
        nq = len(S["chunk_row"])
        lev = np.zeros(nq, dtype=np.int64)
        for q in S["order"]:
            d = S["deps"][S["wptr"][q]:S["wptr"][q + 1]]
            lev[q] = (lev[d].max() if len(d) else 0) + 1
        assert np.all(np.diff(lev[S["order"]]) >= 0)
        assert lev.max() == (s.info.chunk_levels_u if f else s.info.chunk_levels_l)


def test_skewed_chunks_shorten_the_chain():
    """Chunk boundaries shifted per segment (first chunk shorter) so that a
    chunk waits for one chunk of each previous grid line instead of two:
    the chunk graph is markedly shallower than with aligned 64-row chunks,
    whose depth is recomputed here from the exported factors."""
    s = pmg.Solver(2, 5, 128, device=-1)
    seg = s.info.seg_len
    for f, T in ((0, s.export(pmg.OP_L)), (1, s.export(pmg.OP_U))):
        T = T.tocsr()
        nch = (seg + 63) // 64
        chunk = lambda i: (i // seg) * nch + (i % seg) // 64
        nq = s.info.segments * nch
        lev = np.zeros(nq, dtype=np.int64)
        qs = range(nq) if f == 0 else range(nq - 1, -1, -1)
        for q in qs:
            sg, c = divmod(q, nch)
            r0, r1 = sg * seg + c * 64, min(sg * seg + seg, sg * seg + c * 64 + 64)
            cols = T.indices[T.indptr[r0] + (1 if f else 0): T.indptr[r1]] if not f else \
                np.concatenate([T.indices[T.indptr[i] + 1: T.indptr[i + 1]] for i in range(r0, r1)])
            cq = np.unique([chunk(c_) for c_ in cols if not (r0 <= c_ < r1)])
            lev[q] = (lev[cq].max() if len(cq) else 0) + 1
        skewed = s.info.chunk_levels_u if f else s.info.chunk_levels_l
        assert skewed <= 0.85 * lev.max(), (skewed, lev.max())


def _drain(order, deps_of, waves, resident, rng):
    """Replays the ticket protocol of the triangular-solve kernels: the grid
    has `waves` waves, of which at most `resident` run at once (the others
    start only as running waves exit, as when other kernels hold the rest of
    the device).  A running wave draws the next ticket from the one counter,
    exits once the tickets run out, and finishes its chunk once every chunk
    it reads is finished; the step taken next is random.  Returns the chunks
    in finishing order, or None if no running wave can move while chunks
    remain (a deadlock)."""
    nq = len(order)
    count = 0
    held = {}                      # running wave -> ticket or None
    waiting = list(range(waves))   # waves not started yet
    done = np.zeros(nq, dtype=bool)
    finished = []
    while held or waiting:
        while waiting and len(held) < resident:
            held[waiting.pop(0)] = None
        movable = [w for w, t in held.items()
                   if t is None or all(done[d] for d in deps_of[order[t]])]
        if not movable:
            return None
        w = movable[rng.integers(len(movable))]
        if held[w] is None:
            t = count
            count += 1
            if t >= nq:
                del held[w]
            else:
                held[w] = t
        else:
            q = order[held[w]]
            done[q] = True
            finished.append(q)
            held[w] = None
    return finished


@pytest.mark.parametrize("factor", [0, 1])
def test_tickets_never_deadlock_under_partial_residency(factor):
    """One ticket counter (trisolve kernels): with any grid size and any
    number of waves resident at once, down to one, every interleaving drains
    all chunks, so the solves cannot wait on a wave that never runs."""
    s = pmg.Solver(2, 3, 40, device=-1)
    S = s.export_schedule(factor)
    order = [int(q) for q in S["order"]]
    deps_of = {q: [int(d) for d in S["deps"][S["wptr"][q]:S["wptr"][q + 1]]] for q in range(len(order))}
    rng = np.random.default_rng(11)
    for waves, resident in ((1, 1), (8, 1), (8, 3), (13, 2), (13, 13), (64, 5)):
        for _ in range(3):
            fin = _drain(order, deps_of, waves, resident, rng)
            assert fin is not None, "deadlock with %d waves, %d resident" % (waves, resident)
            assert sorted(fin) == list(range(len(order)))


def test_ticket_order_is_what_makes_it_safe():
    """The model detects a deadlock when the order breaks the dependencies:
    with the tickets of a chunk and a chunk it reads swapped, one resident
    wave waits forever (the kernels' poll bound turns this into a fault)."""
    s = pmg.Solver(2, 3, 40, device=-1)
    S = s.export_schedule(0)
    order = [int(q) for q in S["order"]]
    deps_of = {q: [int(d) for d in S["deps"][S["wptr"][q]:S["wptr"][q + 1]]] for q in range(len(order))}
    pos = {q: t for t, q in enumerate(order)}
    q = next(q for q in order if deps_of[q])
    d = deps_of[q][0]
    bad = list(order)
    bad[pos[q]], bad[pos[d]] = d, q
    assert _drain(bad, deps_of, 4, 1, np.random.default_rng(0)) is None
