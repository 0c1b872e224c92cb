"""Host logic of the serving engine, on the CPU: the device library is
replaced by a stand-in that counts steps, so admission order, the memory
budget, chunking, the join of requests that arrive while a chunk runs, and
failure reporting can be checked without a GPU."""
import types

import pytest

from paper_2105_13484_amd import serve


class FakeState:
    def __init__(self, req_id, fail_after=None):
        self.req_id = req_id
        self.steps_done = 0
        self.fail_after = fail_after
        self.closed = False

    def sync(self):
        return 7 if self.fail_after is not None and self.steps_done >= self.fail_after else 0

    def read(self):
        return {"steps": self.steps_done}

    def close(self):
        self.closed = True


class FakeMesh:
    def close(self):
        pass


class FakeBatch:
    """Records every chunk: which members it advanced and by how much."""
    log = []
    clock = None

    def __init__(self, prec, engine):
        self.prec, self.engine, self.members, self.in_flight = prec, engine, [], None

    def add(self, st):
        self.members.append(st)

    def remove(self, st):
        assert self.in_flight is None, "members leave only after the chunk is synced"
        self.members.remove(st)

    def step_async(self, k):
        assert self.in_flight is None
        self.in_flight = (k, list(self.members))
        FakeBatch.log.append((self.prec, k, [m.req_id for m in self.members], self.engine.used_bytes))
        if FakeBatch.clock is not None:
            FakeBatch.clock.t += 1.0       # a chunk takes one time unit

    def query(self):
        return True             # a chunk has finished by the time anyone asks

    def sync(self):
        k, members = self.in_flight
        self.in_flight = None
        rc = 0
        for m in members:
            m.steps_done += k
            rc = rc or m.sync()
        return rc

    def close(self):
        pass


def fake_backend(fail=None):
    fail = fail or {}

    def state_from_case(case, device=None, stream=None):
        return FakeMesh(), FakeState(case.rid, fail.get(case.rid))

    return types.SimpleNamespace(footprint_bytes=lambda mesh, params: mesh.footprint,
                                 state_from_case=state_from_case)


def make_requests(specs):
    reqs = []
    for rid, (arrival, steps, prec, fp) in enumerate(specs):
        case = types.SimpleNamespace(rid=rid, mesh=types.SimpleNamespace(footprint=fp),
                                     params=types.SimpleNamespace(precision=prec), active_cell_layers=100)
        reqs.append(serve.Request(rid=rid, case=case, steps=steps, arrival=arrival))
    return reqs


@pytest.fixture
def engine(monkeypatch):
    def build(budget, chunk, fail=None):
        monkeypatch.setattr(serve, "ssprkse", fake_backend(fail))
        eng = serve.Engine(budget_bytes=budget, chunk_steps=chunk)

        def _batch(self, precision):
            if precision not in self._batches:
                self._streams[precision] = None
                self._batches[precision] = FakeBatch(precision, self)
            return self._batches[precision]

        monkeypatch.setattr(serve.Engine, "_batch", _batch)
        FakeBatch.log = []
        FakeBatch.clock = None
        return eng
    return build


class StepClock:
    """A clock that advances a fixed amount at every reading."""
    def __init__(self, dt):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


def test_every_request_gets_exactly_its_steps(engine):
    reqs = make_requests([(0.0, 7, 0, 10), (0.0, 3, 1, 10), (0.05, 12, 0, 10), (0.3, 5, 1, 10), (0.31, 1, 0, 10)])
    eng = engine(budget=100, chunk=4)
    stats = eng.run(reqs, clock=StepClock(0.01))
    assert stats["requests"] == 5 and stats["failed"] == 0
    for r in reqs:
        assert r.result == {"steps": r.steps}, r.rid
        assert r.arrival <= r.admitted <= r.done


def test_chunks_stop_at_the_nearest_completion(engine):
    reqs = make_requests([(0.0, 7, 0, 10), (0.0, 3, 0, 10)])
    eng = engine(budget=100, chunk=10)
    eng.run(reqs, clock=StepClock(0.001))
    # first chunk: both members, 3 steps (the shorter one ends); then 4 for the other
    assert [(k, ids) for _, k, ids, _ in FakeBatch.log] == [(3, [0, 1]), (4, [0])]


def test_budget_and_fifo_admission(engine):
    # the second request does not fit next to the first: it waits, and the
    # third, which would fit, does not overtake it
    reqs = make_requests([(0.0, 6, 0, 60), (0.0, 2, 0, 50), (0.0, 2, 0, 10)])
    eng = engine(budget=100, chunk=2)
    eng.run(reqs, clock=StepClock(0.001))
    assert all(used <= 100 for *_, used in FakeBatch.log)
    admitted = sorted(reqs, key=lambda r: r.admitted)
    assert [r.rid for r in admitted] == [0, 1, 2]
    first = FakeBatch.log[0][2]
    assert first == [0]


def test_requests_that_arrive_during_a_chunk_join_the_next(engine):
    # every chunk takes one time unit, so request 1 (arrival 0.5) arrives
    # while the first chunk runs: it is set up then, and only the next chunk
    # advances it
    reqs = make_requests([(0.0, 6, 0, 10), (0.5, 4, 0, 10)])
    eng = engine(budget=100, chunk=2)
    FakeBatch.clock = StepClock(1e-6)
    eng.run(reqs, clock=FakeBatch.clock)
    chunks = [ids for _, _, ids, _ in FakeBatch.log]
    assert chunks[0] == [0]
    assert 1 in chunks[1]
    assert reqs[1].result == {"steps": 4} and reqs[0].result == {"steps": 6}


def test_a_failing_member_is_reported_and_the_rest_finish(engine):
    reqs = make_requests([(0.0, 8, 0, 10), (0.0, 8, 0, 10), (0.0, 4, 1, 10)])
    eng = engine(budget=100, chunk=2, fail={1: 2})
    stats = eng.run(reqs, clock=StepClock(0.001))
    assert stats["failed"] == 1
    assert reqs[1].status == 7
    assert reqs[0].status == 0 and reqs[0].result == {"steps": 8}
    assert reqs[2].status == 0 and reqs[2].result == {"steps": 4}


def test_oversized_request_is_refused_up_front(engine):
    reqs = make_requests([(0.0, 2, 0, 500)])
    eng = engine(budget=100, chunk=2)
    with pytest.raises(ValueError):
        eng.run(reqs, clock=StepClock(0.001))


def test_a_batch_does_not_wait_for_the_other(engine, monkeypatch):
    """The FP64 batch's chunks take four polls to finish and the mixed
    batch's one: the mixed batch gets its next chunks while the FP64 one is
    still in flight."""
    reqs = make_requests([(0.0, 8, 0, 10), (0.0, 8, 1, 10)])
    eng = engine(budget=100, chunk=2)
    polls = {}

    def query(self):
        polls[self.prec] = polls.get(self.prec, 0) + 1
        return self.prec == 1 or polls[self.prec] % 4 == 0

    monkeypatch.setattr(FakeBatch, "query", query)
    monkeypatch.setattr(serve.time, "sleep", lambda s: None)
    stats = eng.run(reqs, clock=StepClock(0.001))
    assert stats["failed"] == 0
    order = [p for p, *_ in FakeBatch.log]
    assert order[:5] == [0, 1, 1, 1, 1]
    assert reqs[0].result == {"steps": 8} and reqs[1].result == {"steps": 8}
