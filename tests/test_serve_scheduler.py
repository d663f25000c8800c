"""Scheduling logic of the serving loop, driven by a virtual clock and a
test-only executor that computes nothing (the real executor runs the library)."""
import numpy as np

from paper_2606_25595_amd.serve import Request, Server, request_stream


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Launches finish after `cost` virtual seconds per energy point of the batch."""

    def __init__(self, clock, n_slots=2, cost=0.01):
        self.clock, self.n_slots, self.cost = clock, n_slots, cost
        self.done_at = {}
        self.live_requests = set()
        self.launched = []

    def footprint(self, req, n):
        return n * req.b * req.n_b

    def request_bytes(self, req):
        return req.b * req.n_b

    def start_request(self, req):
        self.live_requests.add(req.rid)

    def finish_request(self, req):
        self.live_requests.remove(req.rid)

    def make_chunk(self, c):
        c.handle = ("chunk", c.req.rid, c.e0)

    def launch(self, slot, chunks):
        self.launched.append([(c.req.rid, c.e0) for c in chunks])
        self.done_at[slot] = self.clock() + self.cost * sum(c.e1 - c.e0 for c in chunks)

    def poll(self, slot):
        return self.clock() >= self.done_at[slot]

    def collect(self, c):
        c.handle = None


def drive(server, clock, arrivals, dt=0.001, t_max=1e4):
    queue = sorted(arrivals, key=lambda r: r.t_arrive)
    while (queue or not server.idle()) and clock.t < t_max:
        while queue and queue[0].t_arrive <= clock.t:
            server.submit(queue.pop(0))
        server.step()
        clock.t += dt


def test_all_requests_complete_and_budget_respected():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    arrivals = request_stream(rate=20.0, duration=2.0, seed=1, b_choices=[8, 16], nb_range=(2, 4), ne_range=(1, 20))
    budget = 4000
    srv = Server(ex, hbm_budget=budget, chunk_energies=4, clock=clock)
    drive(srv, clock, arrivals)
    assert all(r.t_done is not None for r in arrivals)
    assert srv.peak_used <= budget
    assert srv.used == 0 and not ex.live_requests
    rep = srv.report(clock.t)
    assert rep["completed"] == len(arrivals) and rep["p99_latency_s"] >= rep["p50_latency_s"] > 0


def test_continuous_batching_mixes_requests_and_overlaps():
    clock = VirtualClock()
    ex = FakeExecutor(clock, n_slots=2, cost=0.05)
    arrivals = [Request(rid=i, b=8, n_b=2, n_e=8, seed=i, t_arrive=0.02 * i) for i in range(6)]
    srv = Server(ex, hbm_budget=10 ** 6, chunk_energies=4, clock=clock)
    drive(srv, clock, arrivals)
    # some launch carries chunks of more than one request
    assert any(len({rid for rid, _ in l}) > 1 for l in ex.launched)
    # a request that arrived while another launch was running was launched before that one finished
    assert srv.launches < sum(-(-r.n_e // 4) for r in arrivals)
    assert all(r.t_done is not None for r in arrivals)


def test_rejection_when_queue_full_or_too_large():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    srv = Server(ex, hbm_budget=100, chunk_energies=4, max_pending=3, clock=clock)
    big = Request(rid=0, b=64, n_b=8, n_e=4, seed=0)            # one chunk can never fit
    assert not srv.submit(big) and big.rejected
    ok = Request(rid=1, b=2, n_b=2, n_e=8, seed=1)              # two chunks
    assert srv.submit(ok)
    more = Request(rid=2, b=2, n_b=2, n_e=8, seed=2)            # would exceed 3 pending chunks
    assert not srv.submit(more) and more.rejected


def test_poisson_stream_is_reproducible():
    a = request_stream(rate=200.0, duration=1.0, seed=0)
    b = request_stream(rate=200.0, duration=1.0, seed=0)
    assert [(r.b, r.n_b, r.n_e, r.precision, r.t_arrive) for r in a] == \
           [(r.b, r.n_b, r.n_e, r.precision, r.t_arrive) for r in b]
    assert 150 < len(a) < 250
    assert all(128 <= r.b <= 512 and 8 <= r.n_b <= 48 and 16 <= r.n_e <= 128 for r in a)
    assert np.all(np.diff([r.t_arrive for r in a]) > 0)


def test_on_done_called_once_per_completed_request_in_completion_order():
    clock = VirtualClock()
    ex = FakeExecutor(clock, n_slots=2, cost=0.02)
    arrivals = [Request(rid=i, b=8, n_b=2, n_e=4 + 3 * i, seed=i, t_arrive=0.01 * i) for i in range(5)]
    seen = []

    def on_done(r):
        assert r.t_done is not None and r.chunks_left == 0
        seen.append((r.rid, r.t_done))

    srv = Server(ex, hbm_budget=10 ** 6, chunk_energies=4, clock=clock, on_done=on_done)
    drive(srv, clock, arrivals)
    assert sorted(rid for rid, _ in seen) == list(range(5))
    assert [t for _, t in seen] == sorted(t for _, t in seen)
    rejected = Request(rid=9, b=64, n_b=8, n_e=4, seed=9)
    small = Server(FakeExecutor(clock), hbm_budget=100, chunk_energies=4, clock=clock, on_done=on_done)
    assert not small.submit(rejected)
    assert len(seen) == 5   # a rejected request never completes


def test_executor_footprint_compact_forms():
    """Admission bytes of the GPU executor's storage forms (no device needed): dense
    complex128 Sigma and outputs, b-vector Sigma, FPX off-diagonal outputs."""
    from paper_2606_25595_amd.serve import GpuExecutor, Request
    r = Request(rid=0, b=256, n_b=10, n_e=8, seed=1)
    bb = 256 * 256 * 16
    ex = object.__new__(GpuExecutor)
    ex.sigma_diag, ex.out_bits = False, 64
    assert ex.footprint(r, 3) == 3 * (2 * 10 + 5 * 10 - 3) * bb
    ex.sigma_diag, ex.out_bits = True, 32
    per = 2 * 10 * 256 * 16 + 2 * 10 * bb + 3 * 9 * (2 * 256 * 256 * 32 // 8)
    assert ex.footprint(r, 3) == 3 * per
    assert ex.footprint(r, 1) / (67 * bb) < 0.52                   # about half the dense bytes


def test_executor_rejects_bad_storage_forms():
    """Checked before any device work: an FPX width the library does not take, and FPX
    outputs with split chains."""
    import pytest
    from paper_2606_25595_amd.serve import GpuExecutor
    for kw in (dict(out_bits=20), dict(out_bits=8), dict(out_bits=60), dict(out_bits=32, split=True)):
        with pytest.raises(ValueError):
            GpuExecutor(**kw)


def _two_requests():
    big = Request(rid=0, b=64, n_b=10, n_e=8, seed=1, t_arrive=0.0)
    small = Request(rid=1, b=16, n_b=4, n_e=2, seed=2, t_arrive=0.001)
    return big, small


def test_sjf_admits_the_lighter_request_first():
    """With room for one request at a time, shortest-job-first runs the later, lighter
    request before the earlier heavy one; FIFO keeps arrival order."""
    for policy, first in (("sjf", 1), ("fifo", 0)):
        clock = VirtualClock()
        ex = FakeExecutor(clock, n_slots=1, cost=0.05)
        big, small = _two_requests()
        budget = max(ex.footprint(big, 8) + ex.request_bytes(big), ex.footprint(small, 2) + ex.request_bytes(small))
        srv = Server(ex, hbm_budget=budget, chunk_energies=8, clock=clock, policy=policy, max_wait=1e9)
        # both pending before the first scheduling round
        srv.submit(big)
        srv.submit(small)
        drive(srv, clock, [])
        assert big.t_done is not None and small.t_done is not None
        assert ex.launched[0][0][0] == first, (policy, ex.launched)


def test_sjf_ages_waiting_requests():
    """A request pending for max_wait is admitted first whatever its work."""
    clock = VirtualClock()
    ex = FakeExecutor(clock, n_slots=1, cost=0.05)
    big, small = _two_requests()
    budget = max(ex.footprint(big, 8) + ex.request_bytes(big), ex.footprint(small, 2) + ex.request_bytes(small))
    srv = Server(ex, hbm_budget=budget, chunk_energies=8, clock=clock, policy="sjf", max_wait=0.5)
    srv.submit(big)
    srv.submit(small)
    clock.t = 1.0          # the big request has waited 1 s > max_wait
    drive(srv, clock, [])
    assert ex.launched[0][0][0] == 0


def test_sjf_completes_every_request_within_budget():
    clock = VirtualClock()
    ex = FakeExecutor(clock, n_slots=2, cost=0.002)
    reqs = request_stream(rate=50.0, duration=2.0, seed=3, b_choices=[32, 64, 128], nb_range=(4, 12),
                          ne_range=(4, 40))
    budget = 4 * max(ex.footprint(r, 8) + ex.request_bytes(r) for r in reqs)
    srv = Server(ex, hbm_budget=budget, chunk_energies=8, clock=clock, policy="sjf", max_wait=0.5)
    drive(srv, clock, reqs)
    assert all(r.t_done is not None for r in reqs)
    assert srv.peak_used <= budget
