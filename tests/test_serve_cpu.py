"""Scheduling of the continuous-batching server, on the CPU with a fake
executor (the device side is replaced by a model of step progress)."""
import types

import pytest

from paper_2009_04619_amd.serve import Executor, Request, Server, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor(Executor):
    """Each request needs `steps`; launch(n) moves every admitted request by
    n steps and costs `sec_per_step` of simulated time."""

    def __init__(self, clock, sec_per_step=0.001, fail_on=None):
        self.clock = clock
        self.sps = sec_per_step
        self.left = {}
        self.started = []
        self.detached = []
        self.finished = []
        self.waited = []
        self.launches = 0
        self.fail_on = fail_on

    def bytes_for(self, r):
        return r.shot.nbytes

    def start(self, r):
        self.left[r.rid] = r.shot.steps
        self.started.append(r.rid)

    def launch(self, n):
        self.clock.t += n * self.sps
        for k in self.left:
            if k not in self.detached:
                self.left[k] = max(0, self.left[k] - n)
        self.launches += 1
        return self.launches

    def wait(self, token):
        self.waited.append(token)

    def remaining(self, r):
        return self.left[r.rid]

    def detach(self, r):
        assert self.left[r.rid] == 0
        self.detached.append(r.rid)

    def finish(self, r, keep_field):
        # read out only after the launch that completed it has been waited for
        assert r.rid in self.detached and self.waited and self.waited[-1] <= self.launches
        del self.left[r.rid]
        self.finished.append(r.rid)
        r.traces = "traces"


def req(rid, t, steps, nbytes):
    shot = types.SimpleNamespace(steps=steps, nbytes=nbytes, nx=10, ny=10, nz=10)
    return Request(rid=rid, arrival=t, shot=shot)


def test_admission_respects_budget_and_order():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=100, block_steps=10, clock=clk, sleep=clk.sleep)
    rs = [req(0, 0.0, 50, 60), req(1, 0.0, 20, 60), req(2, 0.0, 10, 30)]
    done = srv.run(rs)
    assert [r.rid for r in done] == [0, 1, 2]
    assert all(r.error is None for r in done)
    # 1 cannot start until 0 leaves (60 + 60 > 100); 2 must not overtake 1
    assert ex.started == [0, 1, 2]
    assert srv.peak_in_use <= 100
    admit = {e[1]: e[2] for e in srv.log if e[0] == "admit"}
    fin = {e[1]: e[2] for e in srv.log if e[0] == "finish"}
    assert admit[1] >= fin[0]


def test_requests_join_while_others_run():
    clk = FakeClock()
    ex = FakeExecutor(clk, sec_per_step=0.01)
    srv = Server(ex, budget_bytes=1000, block_steps=5, clock=clk, sleep=clk.sleep)
    rs = [req(0, 0.0, 100, 10), req(1, 0.2, 20, 10)]
    done = srv.run(rs)
    admit = {e[1]: e[2] for e in srv.log if e[0] == "admit"}
    fin = {e[1]: e[2] for e in srv.log if e[0] == "finish"}
    assert admit[1] < fin[0]               # overlapped with request 0
    assert fin[1] < fin[0]                 # short request finishes first
    assert done[1].latency == pytest.approx(fin[1] - 0.2)


def test_oversized_request_is_rejected_not_blocking():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=100, block_steps=10, clock=clk, sleep=clk.sleep)
    done = srv.run([req(0, 0.0, 10, 500), req(1, 0.0, 10, 50)])
    assert done[0].error and "budget" in done[0].error
    assert done[1].error is None
    s = summarize(done, 1.0)
    assert s["served"] == 1 and s["rejected"] == 1


def test_idle_server_sleeps_until_next_arrival():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=100, block_steps=10, clock=clk, sleep=clk.sleep)
    done = srv.run([req(0, 5.0, 10, 10)])
    assert done[0].admitted >= 5.0
    assert done[0].latency == pytest.approx(10 * 0.001, abs=1e-3)


def test_next_block_is_queued_before_the_previous_is_collected():
    """Read-out of the requests a block completes happens after the next
    block has been launched (one block in flight), and every launch is
    waited for exactly once."""
    clk = FakeClock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=1000, block_steps=10, clock=clk, sleep=clk.sleep)
    srv.run([req(0, 0.0, 10, 10), req(1, 0.0, 30, 10)])
    assert ex.finished == [0, 1]
    assert sorted(ex.waited) == list(range(1, ex.launches + 1))
    # request 0 completes with launch 1 and is read out after launch 2 was issued
    fin = {e[1]: e[2] for e in srv.log if e[0] == "finish"}
    assert fin[0] == pytest.approx(2 * 10 * 0.001)
