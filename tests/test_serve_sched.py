"""The continuous-batching scheduler on a simulated executor (virtual clock, fake HBM
budget, fixed per-request iteration needs): admission by footprint, slot reuse,
release of idle groups, latency accounting, no deadlock on requests that cannot fit."""
import time

import numpy as np
import pytest

from paper_2103_09686_amd import serve


class FakeGroup(serve.Group):
    def __init__(self, ex, key, capacity):
        self.ex, self.key, self.capacity = ex, key, capacity
        self.footprint = ex.footprint(key, capacity)
        self.need, self.done_iters = {}, {}
        ex.live += 1
        ex.max_live = max(ex.max_live, ex.live)

    def admit(self, slot, req):
        assert slot not in self.need, "slot handed out twice"
        self.need[slot] = req.payload
        self.done_iters[slot] = 0
        self.ex.max_active[self.key] = max(self.ex.max_active.get(self.key, 0), len(self.need))

    def step(self, iterations):
        out = []
        vox = 0
        for slot in list(self.need):
            self.done_iters[slot] += iterations
            vox += self.key[0]
            if self.done_iters[slot] >= self.need[slot]:
                out.append((slot, 0, 1e-5, self.need[slot]))
                del self.need[slot]
        self.ex.tick_cost = max(self.ex.tick_cost, 1e-4 + 1e-9 * vox * iterations)
        return out

    def cancel(self, slot):
        it = self.done_iters.pop(slot)
        del self.need[slot]
        return 1e-2, it

    def release(self):
        self.ex.live -= 1
        self.ex.released += 1


class FakeExecutor(serve.Executor):
    def __init__(self, per_slot_bytes=100, caps=None):
        self.t, self.tick_cost = 0.0, 0.0
        self.per_slot = per_slot_bytes
        self.caps = caps or {}
        self.live = self.max_live = self.released = 0
        self.max_active = {}

    def capacity(self, key):
        return self.caps.get(key, 4)

    def footprint(self, key, capacity):
        return self.per_slot * capacity * key[0]

    def make_group(self, key, capacity):
        return FakeGroup(self, key, capacity)

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def after_tick(self):
        self.t += self.tick_cost
        self.tick_cost = 0.0


def reqs(n, keys, seed=0, rate=100.0):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1 / rate)
        k = keys[rng.integers(len(keys))]
        out.append(serve.Request(rid=i, arrival=t, key=k, voxels=k[0], payload=int(rng.integers(3, 40))))
    return out


def test_all_requests_finish_with_their_iterations():
    ex = FakeExecutor()
    srv = serve.Server(ex, budget_bytes=10 ** 9, iters_per_tick=4, threads=2)
    rs = reqs(60, [(1,), (2,), (3,)])
    need = {r.rid: r.payload for r in rs}
    done = srv.run(rs)
    srv.close()
    assert sorted(r.rid for r in done) == list(range(60))
    for r in done:
        assert r.iters == need[r.rid] and r.status == 0
        assert r.t_done >= r.t_admit >= r.arrival
    s = serve.summary(done)
    assert s["p99_s"] >= s["p50_s"] > 0 and s["requests"] == 60


def test_slots_never_exceed_capacity_and_are_reused():
    ex = FakeExecutor(caps={(1,): 2})
    srv = serve.Server(ex, budget_bytes=10 ** 9, iters_per_tick=2, threads=1)
    rs = [serve.Request(rid=i, arrival=0.0, key=(1,), voxels=1, payload=10) for i in range(7)]
    done = srv.run(rs)
    srv.close()
    assert len(done) == 7 and ex.max_active[(1,)] == 2


def test_budget_limits_groups_and_idle_groups_are_released():
    # a group costs 100 * capacity * key[0] bytes: (1,) x4 = 400, (2,) x2 = 400; the
    # budget holds one of them at a time, so the classes take turns
    ex = FakeExecutor()
    srv = serve.Server(ex, budget_bytes=450, iters_per_tick=4, threads=2)
    rs = reqs(30, [(1,), (2,)], seed=3)
    done = srv.run(rs)
    srv.close()
    assert len(done) == 30 and all(r.status == 0 for r in done)
    assert srv.peak_bytes <= 450
    assert ex.max_live == 1 and ex.released >= 1


def test_group_shrinks_to_fit_budget():
    ex = FakeExecutor(caps={(5,): 8})
    srv = serve.Server(ex, budget_bytes=1000, iters_per_tick=4, threads=1)
    done = srv.run([serve.Request(rid=i, arrival=0.0, key=(5,), voxels=5, payload=5) for i in range(5)])
    srv.close()
    assert len(done) == 5 and srv.peak_bytes <= 1000   # capacity 8 -> 2 (1000 / 500)


def test_request_that_cannot_fit_fails_instead_of_hanging():
    ex = FakeExecutor()
    srv = serve.Server(ex, budget_bytes=50, iters_per_tick=4, threads=1)
    done = srv.run([serve.Request(rid=0, arrival=0.0, key=(1,), voxels=1, payload=5)])
    srv.close()
    assert len(done) == 1 and done[0].status == -2


def test_request_stream_and_level_rule():
    st = serve.request_stream(200, 20.0, seed=0)
    assert len(st) == 200
    gaps = np.diff([0.0] + [a for (a, *_ ) in st])
    assert abs(gaps.mean() - 1 / 20.0) < 0.02
    from paper_2103_09686_amd import dmcr
    key = serve.make_key((128, 128, 128), 3)
    assert key[1] == 2 and key[2] == 0 and key[3] == (16,)
    spec = dmcr.Spec(shape=key[0], n_channels=key[1], n_levels=key[2], max_disp=key[3])
    assert dmcr.dmcr_level_count(spec) == 3          # 128 -> 64 -> 32 = 2 (16 + 1) - 2
    for n, L in ((128, 2), (256, 3), (512, 4), (1024, 5)):
        k = serve.make_key((n, n), 2)
        assert dmcr.dmcr_level_count(dmcr.Spec(shape=k[0], n_levels=k[2], max_disp=k[3])) == L


# -- asynchronous groups (real clock: each group's advance sleeps in proportion to
# its field size, so groups of different sizes finish their advances at different times)
class TimedGroup(FakeGroup):
    def __init__(self, ex, key, capacity):
        super().__init__(ex, key, capacity)
        self.in_step = False

    def admit(self, slot, req):
        assert not self.in_step, "request admitted while the group is being advanced"
        super().admit(slot, req)

    def step(self, iterations):
        self.in_step = True
        time.sleep(2e-5 * self.key[0] * iterations)
        out = super().step(iterations)
        self.in_step = False
        return out


class TimedExecutor(FakeExecutor):
    def make_group(self, key, capacity):
        return TimedGroup(self, key, capacity)

    def now(self):
        return time.perf_counter()

    def wait_until(self, t):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(min(d, 0.005))


def test_asynchronous_groups_finish_every_request():
    ex = TimedExecutor(caps={(1,): 3, (20,): 2})
    srv = serve.Server(ex, budget_bytes=10 ** 9, iters_per_tick=4, threads=4, asynchronous=True)
    rs = reqs(40, [(1,), (20,)], seed=5, rate=400.0)
    need = {r.rid: r.payload for r in rs}
    done = srv.run(rs)
    srv.close()
    assert sorted(r.rid for r in done) == list(range(40))
    for r in done:
        assert r.iters == need[r.rid] and r.status == 0
        assert r.t_done >= r.t_admit >= r.arrival
    assert ex.max_active[(1,)] <= 3 and ex.max_active[(20,)] <= 2


def test_asynchronous_budget_and_unfit_requests():
    ex = TimedExecutor()
    srv = serve.Server(ex, budget_bytes=450, iters_per_tick=4, threads=2, asynchronous=True)
    rs = reqs(20, [(1,), (2,)], seed=3, rate=400.0)
    done = srv.run(rs)
    srv.close()
    assert len(done) == 20 and all(r.status == 0 for r in done) and srv.peak_bytes <= 450
    srv = serve.Server(TimedExecutor(), budget_bytes=50, iters_per_tick=4, threads=1, asynchronous=True)
    done = srv.run([serve.Request(rid=0, arrival=0.0, key=(1,), voxels=1, payload=5)])
    srv.close()
    assert len(done) == 1 and done[0].status == -2


@pytest.mark.parametrize("asynchronous", [False, True])
def test_cancel_and_timeout(asynchronous):
    """A cancelled request and one whose timeout passes are retired with CANCELLED and
    TIMED_OUT (queued or running), their slots are reused, and every other request
    still finishes with its own iterations."""
    ex = FakeExecutor(caps={(1,): 2}) if not asynchronous else None
    if asynchronous:
        ex = TimedExecutor(caps={(1,): 2})
    srv = serve.Server(ex, budget_bytes=10 ** 9, iters_per_tick=1, threads=1, asynchronous=asynchronous)
    rs = [serve.Request(rid=i, arrival=0.0, key=(1,), voxels=1, payload=6) for i in range(6)]
    rs[0].payload = 10 ** 6          # would run for ever: times out while running
    rs[0].timeout = 0.02 if asynchronous else 0.002
    rs[5].timeout = 0.0              # times out in the queue
    srv.cancel(3)                    # cancelled before it is admitted
    done = srv.run(rs)
    srv.close()
    by = {r.rid: r for r in done}
    assert sorted(by) == list(range(6))
    assert by[0].status == serve.TIMED_OUT and by[0].iters > 0
    assert by[5].status == serve.TIMED_OUT and by[5].iters == 0
    assert by[3].status == serve.CANCELLED
    for i in (1, 2, 4):
        assert by[i].status == 0 and by[i].iters == 6
    s = serve.summary(done)
    assert s["timed_out"] == 2 and s["cancelled"] == 1 and s["converged"] == 3
