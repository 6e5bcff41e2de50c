"""Host logic of the serving loop (paper_2211_00316_amd.serve.Server) on a simulated executor
and clock: admission by bytes within the budget, first come first served, continuous
batching at step boundaries, failure handling and the latency report; and the seeded
request draws of the serving mix."""
import numpy as np
import pytest

import phantoms as ph
from paper_2211_00316_amd.serve import Report, Request, Server


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, s):
        assert s >= 0
        self.t += s


class SimExecutor:
    """Steps cost the largest per-step cost of the batch; fail[rid] = step index at which
    that request's step fails."""

    def __init__(self, clock, cost=None, fail=None):
        self.clock = clock
        self.cost = cost or {}
        self.fail = fail or {}
        self.open_ids = set()
        self.batches = []
        self.bytes = {}

    def need_bytes(self, r):
        return self.bytes.get(r.tag, 100)

    def open(self, r):
        assert r.rid not in self.open_ids
        self.open_ids.add(r.rid)

    def step(self, reqs):
        assert all(r.rid in self.open_ids for r in reqs)
        self.batches.append([r.rid for r in reqs])
        self.clock.t += max(self.cost.get(r.tag, 1.0) for r in reqs)
        return [-4 if self.fail.get(r.rid) == r.steps_done else 0 for r in reqs]

    def close(self, r):
        self.open_ids.remove(r.rid)


def req(rid, arrival, n_steps, tag="a"):
    return Request(rid, arrival, None, None, None, [1.0] * n_steps, [1.0] * n_steps,
                   [1] * n_steps, tag=tag)


def run(reqs, budget=1000, max_batch=16, **kw):
    clk = SimClock()
    ex = SimExecutor(clk, **kw)
    rep = Server(ex, budget, max_batch=max_batch, clock=clk, sleep=clk.sleep).run(reqs)
    return rep, ex


def test_every_request_gets_its_steps_and_latency():
    reqs = [req(0, 0.0, 3), req(1, 0.0, 1), req(2, 0.5, 2)]
    rep, ex = run(reqs)
    assert [r.steps_done for r in rep.requests] == [3, 1, 2]
    assert rep.steps == 6 and not ex.open_ids
    # batches: {0,1} at t=0; 1 leaves; 2 arrived at 0.5, joins at t=1
    assert ex.batches == [[0, 1], [0, 2], [0, 2]]
    assert [r.t_done for r in rep.requests] == [3.0, 1.0, 3.0]
    assert [r.latency for r in rep.requests] == [3.0, 1.0, 2.5]
    assert rep.makespan == 3.0 and rep.steps_per_s == 2.0


def test_admission_keeps_within_budget_and_is_first_come_first_served():
    # each request needs 400 of 1000 bytes: at most two run at once; the third waits for a
    # slot, and the later small request does not overtake it
    reqs = [req(i, 0.0, 2, tag="big") for i in range(3)] + [req(3, 0.1, 1, tag="small")]
    clk = SimClock()
    ex = SimExecutor(clk)
    ex.bytes = {"big": 400, "small": 10}
    rep = Server(ex, 1000, clock=clk, sleep=clk.sleep).run(reqs)
    assert rep.peak_bytes <= 1000
    assert all(len([i for i in b if i < 3]) <= 2 for b in ex.batches)
    admits = [r.t_admit for r in sorted(rep.requests, key=lambda r: r.rid)]
    assert admits == sorted(admits)
    assert rep.requests[3].t_admit >= rep.requests[2].t_admit


def test_max_batch_and_idle_wait():
    reqs = [req(i, 5.0, 1) for i in range(5)]
    rep, ex = run(reqs, max_batch=2)
    assert max(len(b) for b in ex.batches) == 2
    assert min(r.t_admit for r in rep.requests) == 5.0   # the server slept until the arrival
    assert rep.steps == 5


def test_a_failed_step_ends_the_request_and_frees_its_bytes():
    reqs = [req(0, 0.0, 4), req(1, 0.0, 4)]
    rep, ex = run(reqs, fail={0: 1})
    r0, r1 = rep.requests
    assert r0.status == -4 and r0.steps_done == 1 and r0.t_done == 2.0
    assert r1.status == 0 and r1.steps_done == 4
    assert not ex.open_ids
    assert rep.summary()["failed"] == 1


def test_request_above_the_budget_is_refused():
    clk = SimClock()
    ex = SimExecutor(clk)
    ex.bytes = {"huge": 5000}
    with pytest.raises(ValueError):
        Server(ex, 1000, clock=clk, sleep=clk.sleep).run([req(0, 0.0, 1, tag="huge")])


def test_report_percentiles():
    rs = []
    for i, lat in enumerate([1.0, 2.0, 3.0, 10.0]):
        r = req(i, 0.0, 1)
        r.t_done = lat
        rs.append(r)
    rep = Report(rs, 10.0, 4, [4], 0, 1)
    assert rep.latency_pct(50) == pytest.approx(np.percentile([1, 2, 3, 10], 50))
    assert rep.latency_pct(99) == pytest.approx(np.percentile([1, 2, 3, 10], 99))


def test_serve_draws_are_seeded_and_in_range():
    a = ph.serve_draws(64, seed=5, rate=2.0)
    b = ph.serve_draws(64, seed=5, rate=4.0)
    assert [(d.cls, d.phantom_seed, d.n_steps) for d in a] == \
        [(d.cls, d.phantom_seed, d.n_steps) for d in b]
    assert np.allclose([2 * d.arrival for d in a], [4 * d.arrival for d in b])
    assert all(0 <= d.cls < 3 and 8 <= d.n_steps <= 32 for d in a)
    assert all(x.arrival <= y.arrival for x, y in zip(a, a[1:]))
    assert {d.cls for d in a} == {0, 1, 2}
    assert all(d.arrival == 0.0 for d in ph.serve_draws(8, seed=5))


def test_step_frequencies_span_the_list_low_to_high():
    for n in (1, 2, 8, 17, 32):
        idx = ph.step_frequencies(n, 32)
        assert len(idx) == n and idx[0] == 0 and (n == 1 or idx[-1] == 31)
        assert all(x < y for x, y in zip(idx, idx[1:]))
    assert ph.step_frequencies(32, 32) == list(range(32))


def test_serve_classes():
    names = [w.name for w in ph.SERVE_CLASSES]
    assert names == ["serve_ring256_grid256", "serve_ring512_grid512",
                     "serve_ring1024_grid1024"]
    for w in ph.SERVE_CLASSES:
        assert w.n_rays == w.n_trans and len(w.freqs) == 32 and w.freqs[0] == 100e3
        assert (w.nx - 1) * w.dx / 2 > w.radius     # the ring lies inside the grid
