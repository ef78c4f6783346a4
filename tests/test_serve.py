"""CPU checks of the serving scheduler (continuous batching) against a simulated device, the
request stream, the latency statistics and the library's footprint query (host-only)."""
import math

import numpy as np
import pytest

from paper_1211_4575_amd import inputs as I
from paper_1211_4575_amd import serve as S


class FakeDevice:
    """A device that runs enqueued batch steps one after another; a step takes
    ``a + b * (particles of its members)`` seconds.  The host clock only moves when the host
    sleeps or waits for the device (host work is free)."""

    def __init__(self, a=1e-3, b=1e-9, fail=()):
        self.a, self.b = a, b
        self.fail = set(fail)
        self.host = 0.0
        self.dev_free = 0.0
        self.members = {}
        self.steps_done = {}
        self.live_bytes = 0
        self.peak_live = 0
        self.admit_log = []
        self.max_members = 0

    def footprint(self, req):
        return 100 + req.n_per_beam

    def start(self):
        pass

    def now(self):
        return self.host

    def admit(self, req):
        h = req.rid
        self.members[h] = req
        self.steps_done[h] = 0
        self.live_bytes += self.footprint(req)
        self.peak_live = max(self.peak_live, self.live_bytes)
        self.admit_log.append((self.host, req.arrival, req.rid))
        return h

    def step(self):
        self.max_members = max(self.max_members, len(self.members))
        work = sum(2 * r.n_per_beam for r in self.members.values())
        start = max(self.host, self.dev_free)
        self.dev_free = start + self.a + self.b * work
        for h in self.members:
            self.steps_done[h] += 1
        return self.dev_free

    def leave(self, h):
        del self.members[h]

    def done(self, tok):
        return tok if tok <= self.host else None

    def wait(self, tok):
        self.host = max(self.host, tok)
        return tok

    def retire(self, h):
        self.live_bytes -= 100 + self._req(h).n_per_beam
        return (1 if h in self.fail else 0), dict(steps=self.steps_done[h])

    def _req(self, h):
        return self._reqs[h]

    def sleep_until(self, t):
        self.host = max(self.host, t)

    def finish(self):
        self.host = max(self.host, self.dev_free)


def _requests(count=40, rate=50.0, seed=7):
    return I.serving_requests(count=count, rate=rate, seed=seed, steps=(5, 40),
                              grids=((8, 8, 8), (16, 8, 8)), lattices=((1, 1, 1), (2, 2, 2)))


def _serve(reqs, budget=10**9, slots=64, **kw):
    dev = FakeDevice(**kw)
    dev._reqs = {r.rid: r for r in reqs}
    sch = S.Scheduler(dev, mem_budget=budget, max_slots=slots)
    return dev, sch, sch.run(reqs)


def test_every_request_completes_with_its_own_step_count():
    reqs = _requests()
    dev, sch, res = _serve(reqs)
    assert [r.rid for r in res] == [r.rid for r in reqs]
    for r, q in zip(res, reqs):
        assert r.status == "ok"
        assert r.info["steps"] == q.steps  # stepped exactly its steps while a member
        assert r.admitted >= q.arrival
        assert r.done > r.admitted
        assert r.latency >= q.steps * dev.a
    assert dev.live_bytes == 0 and not dev.members


def test_requests_overlap_on_the_device():
    # arrivals faster than service: several runs share batch steps
    reqs = _requests(rate=500.0)
    dev, sch, res = _serve(reqs)
    assert sch.peak_members > 4
    # fewer batch steps than the sum of the requests' steps
    assert sch.batch_steps < sum(q.steps for q in reqs) / 2


def test_memory_budget_and_slots_hold():
    reqs = _requests(rate=500.0)
    need = [100 + q.n_per_beam for q in reqs]
    budget = 3 * max(need)
    dev, sch, res = _serve(reqs, budget=budget)
    assert dev.peak_live <= budget and sch.peak_bytes <= budget
    assert all(r.status == "ok" for r in res)
    dev, sch, res = _serve(reqs, slots=3)
    assert dev.max_members <= 3 and sch.peak_members <= 3


def test_admission_in_arrival_order():
    reqs = _requests(rate=500.0)
    dev, sch, res = _serve(reqs, budget=2 * max(100 + q.n_per_beam for q in reqs))
    order = [rid for _, _, rid in dev.admit_log]
    assert order == [q.rid for q in sorted(reqs, key=lambda q: (q.arrival, q.rid))]
    times = [t for t, _, _ in dev.admit_log]
    assert times == sorted(times)


def test_too_large_rejected_and_failures_isolated():
    reqs = _requests()
    big = max(reqs, key=lambda q: q.n_per_beam)
    budget = 100 + big.n_per_beam - 1
    dev, sch, res = _serve(reqs, budget=budget, fail=(3,))
    for r, q in zip(res, reqs):
        if 100 + q.n_per_beam > budget:
            assert r.status == "rejected"
        elif q.rid == 3:
            assert r.status == "failed" and r.flags == 1
        else:
            assert r.status == "ok"


def test_cancelled_requests_leave_and_the_others_are_untouched():
    # request 2 cancelled while it waits, request 5 after 3 of its steps, request 9 from a
    # completion callback: each reported "cancelled" with the steps it ran; every other request
    # completes with its own step count, and the device ends empty
    reqs = _requests(rate=500.0)
    dev = FakeDevice()
    dev._reqs = {r.rid: r for r in reqs}
    sch = None

    def on_complete(res, active):
        if res.rid == 0:
            sch.cancel(9)

    sch = S.Scheduler(dev, mem_budget=10**9, max_slots=4, on_complete=on_complete)
    sch.cancel(2)
    res = sch.run(reqs, cancel_after={5: 3})
    by = {r.rid: r for r in res}
    assert len(res) == len(reqs)
    assert by[2].status == "cancelled" and by[2].steps == 0
    assert by[5].status == "cancelled" and by[5].steps == 3 and by[5].info["steps"] == 3
    assert by[9].status == "cancelled" and by[9].steps < reqs[9].steps
    for q in reqs:
        if q.rid not in (2, 5, 9):
            assert by[q.rid].status == "ok" and by[q.rid].info["steps"] == q.steps
    assert dev.live_bytes == 0 and not dev.members
    s = S.summarize(res)
    assert s["cancelled"] == 3 and s["completed"] == len(reqs) - 3 and s["failed"] == 0


def test_idle_device_waits_for_arrivals():
    reqs = _requests(count=5, rate=0.5)  # far apart: each served alone right away
    dev, sch, res = _serve(reqs)
    for r, q in zip(res, reqs):
        assert r.admitted == pytest.approx(q.arrival)
        single = q.steps * (dev.a + dev.b * 2 * q.n_per_beam)
        assert r.latency == pytest.approx(single, rel=1e-9)


def test_percentile_matches_numpy_linear():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 100):
        v = rng.exponential(size=n)
        for q in (0, 50, 90, 99, 100):
            assert S.percentile(v, q) == pytest.approx(np.percentile(v, q), rel=1e-12)
    assert math.isnan(S.percentile([], 50))


def test_fifo_one_at_a_time():
    reqs = [I.TwoStreamRequest(i, a, (8, 8, 8), (1, 1, 1), 0.2, 0.01, 10, i) for i, a in enumerate((0.0, 1.0, 1.5, 10.0))]
    res = S.fifo_one_at_a_time(reqs, {0: 2.0, 1: 1.0, 2: 3.0, 3: 1.0})
    assert [r.done for r in res] == [2.0, 3.0, 6.0, 11.0]
    assert [r.latency for r in res] == [2.0, 2.0, 4.5, 1.0]
    s = S.summarize(res, t_first=0.0)
    assert s["makespan_s"] == 11.0 and s["p50_s"] == 2.0
    assert s["updates_per_s"] == pytest.approx(sum(r.updates for r in reqs) / 11.0)


def test_serving_requests_stream():
    a = I.serving_requests(count=256)
    b = I.serving_requests(count=256)
    assert a == b
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    assert 0.8 < len(a) / arr[-1] < 1.2  # rate 1 per second
    assert {r.n for r in a} == set(I.SERVING_GRIDS)
    assert {r.ppc for r in a} == {8, 16, 32, 64}
    assert all(0.1 <= r.v_beam <= 0.5 and 200 <= r.steps <= 2000 for r in a)
    sizes = [2 * r.n_per_beam for r in a]
    assert min(sizes) >= 32768 * 16 and max(sizes) <= 65536 * 128
    assert len({r.seed for r in a}) == 256


def test_workspace_size_is_host_only_and_validates():
    from paper_1211_4575_amd import pp
    P = pp.make_params((32, 32, 32), d=(0.1,) * 3, dt=0.04, shape_order=3, field_order=6,
                       precision=pp.PP_PREC_FP32_SPLIT)
    b0 = pp.pp_workspace_size(P, 0, 2)
    b1 = pp.pp_workspace_size(P, 1000, 2)
    # two int32 of sort scratch per particle of the largest species, one int32 rank and one
    # int32 sort permutation entry per particle of each species
    assert b1 - b0 == 2 * 1000 * 4 + 2 * (2 * 1000 * 4)
    nc = 32 ** 3
    assert b0 >= (3 + 3 + 2 + 3) * 3 * nc * 8 // 3  # relaxation buffers, J2, rho pair, fixed-point J
    P64 = pp.make_params((32, 32, 32), shape_order=3, field_order=2)
    assert pp.pp_workspace_size(P64, 1000, 2) < b0
    with pytest.raises(pp.PPError):
        pp.pp_workspace_size(pp.make_params((8, 8, 8), dt=1.0), 10, 1)
