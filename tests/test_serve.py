"""Serving loop (admission by output bytes, continuous batching) driven on the
host: every query's result equals the plain scan-and-lookup of Sec. 2.2 on the
raw values, alone or in a mix, and the scheduler keeps its memory budget."""
import numpy as np
import pytest

from oracle.scan import scan_values
from paper_2209_00220_amd.serve import Query, Server, latency_summary, poisson_arrivals, run_serial


class HostExecutor:
    """Executes the server's steps with plain numpy on raw value columns."""

    def __init__(self, tables, step_cost=0.0, clock=None):
        self.tables = tables
        self.steps = []
        self.finishes = []
        self.step_cost = step_cost
        self.clock = clock

    def n_rows(self, t):
        return next(iter(self.tables[t].values())).shape[0]

    def bv_bytes(self, t):
        return 8 * ((self.n_rows(t) + 63) // 64)

    def new_bv(self, t):
        return np.zeros(self.n_rows(t), dtype=bool)

    def scan_step(self, items):
        self.steps.append([(t, c, op, lo, hi, inb is not None) for t, c, op, lo, hi, inb, _ in items])
        for t, c, op, lo, hi, inb, out in items:
            out[:] = scan_values(self.tables[t][c], op, lo, hi, in_mask=inb)
        if self.clock is not None:
            self.clock.t += self.step_cost
        return object()

    def finish(self, t, bv, columns, cap):
        self.finishes.append((t, tuple(columns), cap))
        count = int(bv.sum())
        vals = {c: self.tables[t][c][bv].copy() for c in columns}
        return (count, None if (columns and count > cap) else vals)

    def result(self, token):
        return token

    def is_done(self, token):
        return True

    def wait(self, token):
        pass


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def _tables(seed=0):
    rng = np.random.default_rng(seed)
    return {
        "a": {c: rng.integers(0, 1 << 12, 5000, dtype=np.uint32) for c in ("c0", "c1", "c2")},
        "b": {c: rng.integers(0, 1 << 20, 3001, dtype=np.uint32) for c in ("d0", "d1")},
    }


def _queries(tables, n, seed, arrivals=None):
    rng = np.random.default_rng(seed)
    ops = ["lt", "le", "gt", "ge", "eq", "ne", "between"]
    qs = []
    for i in range(n):
        t = ["a", "b"][int(rng.integers(0, 2))]
        cols = list(tables[t])
        preds = []
        for _ in range(int(rng.integers(1, 5))):
            c = cols[int(rng.integers(0, len(cols)))]
            x = tables[t][c]
            lo, hi = sorted(int(v) for v in x[rng.integers(0, x.shape[0], 2)])
            op = ops[int(rng.integers(0, len(ops)))]
            preds.append((c, op, lo, hi if op == "between" else None))
        look = [cols[int(j)] for j in rng.choice(len(cols), size=int(rng.integers(1, 3)), replace=False)]
        qs.append(Query(i, t, preds, look, 0.0 if arrivals is None else float(arrivals[i])))
    return qs


def _plain(tables, q):
    sel = None
    for c, op, lo, hi in q.preds:
        sel = scan_values(tables[q.table][c], op, lo, hi, in_mask=sel)
    return {c: tables[q.table][c][sel] for c in q.lookups}, int(sel.sum())


def test_results_equal_plain_scan_and_lookup():
    tables = _tables()
    qs = _queries(tables, 40, seed=1)
    res = Server(HostExecutor(tables), budget_bytes=1 << 30).run(qs)
    for q in qs:
        want, cnt = _plain(tables, q)
        assert res[q.qid].count == cnt
        for c in q.lookups:
            assert np.array_equal(res[q.qid].values[c], want[c])


def test_alone_equals_in_mix():
    tables = _tables(3)
    qs = _queries(tables, 30, seed=4)
    mix = Server(HostExecutor(tables), budget_bytes=1 << 30).run(qs)
    for q in qs:
        alone = Server(HostExecutor(tables), budget_bytes=1 << 30).run([q])[q.qid]
        assert alone.count == mix[q.qid].count
        for c in q.lookups:
            assert np.array_equal(alone.values[c], mix[q.qid].values[c])
    serial = run_serial(HostExecutor(tables), qs)
    for q in qs:
        assert serial[q.qid].count == mix[q.qid].count


def test_continuous_batching_one_predicate_per_step():
    tables = _tables()
    qs = _queries(tables, 10, seed=2)
    ex = HostExecutor(tables)
    Server(ex, budget_bytes=1 << 30).run(qs)
    # all arrive at 0: step s carries the s-th predicate of every query with more than s
    for s, step in enumerate(ex.steps):
        assert len(step) == sum(1 for q in qs if len(q.preds) > s)
        assert all(has_in == (s > 0) for *_, has_in in step)
    assert len(ex.steps) == max(len(q.preds) for q in qs)


def test_budget_limits_admission():
    tables = _tables()
    qs = _queries(tables, 12, seed=5)
    per_query = 2 * 8 * ((5000 + 63) // 64)   # the larger table's two bitvectors
    ex = HostExecutor(tables)
    # no lookup outputs reserved up front: admission counts the bitvectors only
    srv = Server(ex, budget_bytes=6 * per_query, lookup_cap_rows=0)   # reservations may hold half: three queries
    res = srv.run(qs)
    assert len(res) == len(qs)
    assert max(len(s) for s in ex.steps) <= 3
    # bitvector reservations never exceed the budget (lookup bytes may, for the oldest query)
    assert srv.in_use == 0 and srv.scan_in_use == 0
    # admission in arrival order
    adm = [res[q.qid].admitted for q in sorted(qs, key=lambda q: q.qid)]
    assert adm == sorted(adm)


def test_lookups_keep_their_share_of_the_budget():
    # one-predicate queries all arriving at once: the bitvectors of the admitted
    # queries hold at most the scan share, so every query's lookup fits in the
    # rest and it completes in the step its scan ran
    tables = _tables()
    clock = FakeClock()
    qs = [q for q in _queries(tables, 40, seed=11) if q.table == "a"][:12]
    for q in qs:
        q.preds = q.preds[:1]
    per_query = 2 * 8 * ((5000 + 63) // 64)
    budget = 1 << 20
    ex = HostExecutor(tables, step_cost=0.01, clock=clock)
    srv = Server(ex, budget_bytes=budget, scan_share=4 * per_query / budget, lookup_cap_rows=0, clock=clock,
                 sleep=clock.sleep)
    res = srv.run(qs)
    assert len(qs) == 12 and max(len(s) for s in ex.steps) == 4 and len(ex.steps) == 3
    for q in qs:
        assert res[q.qid].done == pytest.approx(res[q.qid].admitted + 0.01)
        assert res[q.qid].count == _plain(tables, q)[1]
    with pytest.raises(ValueError):
        Server(ex, budget_bytes=budget, scan_share=0.0)


def test_single_query_over_budget_still_runs():
    tables = _tables()
    q = _queries(tables, 1, seed=6)[0]
    res = Server(HostExecutor(tables), budget_bytes=1).run([q])
    assert res[q.qid].count == _plain(tables, q)[1]


def test_late_arrivals_join_between_steps():
    tables = _tables()
    clock = FakeClock()
    arr = [0.0, 0.0, 0.005, 0.5]
    qs = _queries(tables, 4, seed=7, arrivals=arr)
    for q in qs:   # three predicates each, so the early queries are still scanning
        q.preds = (q.preds * 3)[:3]
    ex = HostExecutor(tables, step_cost=0.01, clock=clock)
    res = Server(ex, budget_bytes=1 << 30, clock=clock, sleep=clock.sleep).run(qs)
    # query 2 arrives during the first step and joins at the second
    assert [len(s) for s in ex.steps[:3]] == [2, 3, 3]
    assert res[3].admitted >= 0.5
    assert res[2].admitted == pytest.approx(0.01)
    for q in qs:
        assert res[q.qid].count == _plain(tables, q)[1]


def test_poisson_and_summary():
    a = poisson_arrivals(1000, 200.0, seed=9)
    b = poisson_arrivals(1000, 200.0, seed=9)
    assert np.array_equal(a, b) and np.all(np.diff(a) >= 0)
    assert 3.5 < a[-1] < 6.5   # about 1000 / 200 s
    tables = _tables()
    res = Server(HostExecutor(tables), budget_bytes=1 << 30).run(_queries(tables, 20, seed=8))
    s = latency_summary(res)
    assert s["queries"] == 20 and s["p50_ms"] <= s["p99_ms"]


def test_query_without_predicate_rejected():
    with pytest.raises(ValueError):
        Server(HostExecutor(_tables()), budget_bytes=1 << 20).run([Query(0, "a", [], ["c0"])])


class _Token:
    def __init__(self, idx, value=None):
        self.idx, self.value, self.done = idx, value, False


class LazyExecutor(HostExecutor):
    """Work completes only when the loop waits for it (in enqueue order), so
    scan steps really are in flight between iterations."""

    def __init__(self, tables):
        super().__init__(tables)
        self.tokens = []
        self.max_scan_inflight = 0

    def _token(self, value=None):
        t = _Token(len(self.tokens), value)
        self.tokens.append(t)
        return t

    def scan_step(self, items):
        super().scan_step(items)
        t = self._token()
        t.scan = True
        inflight = sum(1 for x in self.tokens if getattr(x, "scan", False) and not x.done)
        self.max_scan_inflight = max(self.max_scan_inflight, inflight)
        return t

    def finish(self, t, bv, columns, cap):
        return self._token(super().finish(t, bv, columns, cap))

    def result(self, token):
        assert token.done
        return token.value

    def is_done(self, token):
        return token.done

    def wait(self, token):
        for t in self.tokens[: token.idx + 1]:
            t.done = True


@pytest.mark.parametrize("lookahead,lookahead_rows,bound", [(8, 10_000, 2), (3, 1 << 30, 3), (8, 1, 1)])
def test_scan_steps_in_flight_are_bounded(lookahead, lookahead_rows, bound):
    # one scan per step (5000 rows each): at most `bound` steps in flight, by
    # count or by rows, and one step always may go
    tables = _tables()
    qs = [q for q in _queries(tables, 30, seed=13) if q.table == "a"][:8]
    for q in qs:
        q.preds = (q.preds * 3)[:3]
    ex = LazyExecutor(tables)
    res = Server(ex, budget_bytes=1 << 30, max_batch=1, lookahead=lookahead, lookahead_rows=lookahead_rows).run(qs)
    assert ex.max_scan_inflight == bound
    for q in qs:
        want, cnt = _plain(tables, q)
        assert res[q.qid].count == cnt
        for c in q.lookups:
            assert np.array_equal(res[q.qid].values[c], want[c])



def test_lookup_outputs_reserved_at_admission():
    """A query reserves its bitvectors and the lookup outputs of up to
    lookup_cap_rows rows when admitted; its lookups then follow its last scan
    with no count read in between (one finish per query).  A query with more
    rows looks up again with the exact count, and its result is unchanged."""
    tables = _tables()
    qs = _queries(tables, 30, seed=21)
    for cap_rows, expect_relookup in ((1 << 25, False), (40, True)):
        ex = HostExecutor(tables)
        srv = Server(ex, budget_bytes=1 << 30, lookup_cap_rows=cap_rows)
        res = srv.run(qs)
        for q in qs:
            want, cnt = _plain(tables, q)
            assert res[q.qid].count == cnt
            for c in q.lookups:
                assert np.array_equal(res[q.qid].values[c], want[c])
        big = sum(1 for q in qs if _plain(tables, q)[1] > cap_rows)
        assert srv.relookups == big and (big > 0) == expect_relookup
        assert len(ex.finishes) == len(qs) + big
        assert all(cap == min(ex.n_rows(t), cap_rows) for t, cols, cap in ex.finishes[:1])
        assert srv.in_use == 0 and srv.scan_in_use == 0
    # the reservation limits admission: each query of table "a" reserves two
    # bitvectors and 5000 rows of lookup outputs, so at most two fit at once
    one = [q for q in qs if q.table == "a" and len(q.lookups) == 1][:6]
    per = 2 * 8 * ((5000 + 63) // 64) + 4 * 5000 * 2
    ex = HostExecutor(tables)
    srv = Server(ex, budget_bytes=4 * per + 100, scan_share=0.5)
    srv.run(one)
    assert max(len(s) for s in ex.steps) <= 2 and srv.peak_in_use <= 4 * per + 100
