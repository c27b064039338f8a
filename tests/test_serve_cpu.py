"""Serving loop on the CPU: scheduler policy with a fake backend and an
injected clock (admission by memory and slots, continuous admission,
timeouts, cancellation, backpressure, failure isolation)."""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_2606_26439_amd import serve as S


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def idle(self, dt):
        self.t += max(dt, 1e-4)


class FakeBackend(S.Backend):
    """Scores with the FP64 oracle; a batch takes `per_pair` seconds per pair
    of simulated device time, starting when launched."""

    def __init__(self, clock, pool, per_pair=1e-6, k=10, fail_rids=()):
        self.clock, self.pool, self.per_pair, self.k = clock, pool, per_pair, k
        self.fail_rids = set(fail_rids)
        self.launches = []
        self.max_inflight_seen = 0
        self._inflight = 0

    def launch(self, batch):
        if any(r.rid in self.fail_rids for r in batch.requests):
            raise RuntimeError("injected device failure")
        pairs = sum(len(r.cand_ids) for r in batch.requests)
        self._inflight += 1
        self.max_inflight_seen = max(self.max_inflight_seen, self._inflight)
        h = {"done_at": self.clock() + pairs * self.per_pair, "batch": batch}
        self.launches.append((self.clock(), batch))
        return h

    def poll(self, h):
        return self.clock() >= h["done_at"]

    def results(self, h):
        self._inflight -= 1
        out = []
        d, d_off = self.pool
        for r in h["batch"].requests:
            sc = oracle.maxsim(r.query, [0, len(r.query)], d, d_off,
                               [0, len(r.cand_ids)], r.cand_ids)
            ids, vals = oracle.topk(sc, self.k, r.cand_ids.astype(np.int64))
            out.append((ids, vals.astype(np.float32)))
        return out


@pytest.fixture(scope="module")
def pool():
    c = W.ragged_case(300, dim=64, nq=4)
    return c["d"], c["d_off"]


def make_requests(n, n_pool, seed=0, rate=1000.0, nq=(2, 6), cand=(20, 80), dim=64):
    g = W.rng(seed)
    arr = W.poisson_arrivals(n, rate, seed=seed + 3)
    out = []
    for i in range(n):
        q = W.unit_tokens(int(g.integers(nq[0], nq[1] + 1)), dim, g)
        ids = g.choice(n_pool, size=int(g.integers(cand[0], cand[1] + 1)), replace=False)
        out.append(S.Request(i, q, ids.astype(np.int32), arrival=float(arr[i])))
    return out


def run(reqs, pool, clock=None, **kw):
    clock = clock or SimClock()
    fb_kw = {k: kw.pop(k) for k in ("per_pair", "fail_rids") if k in kw}
    be = FakeBackend(clock, pool, **fb_kw)
    sched = S.Scheduler(dim=64, k=10, **kw)
    srv = S.Server(sched, be, clock=clock, idle=clock.idle)
    done = srv.run(reqs)
    return done, be, srv


def test_every_request_completes_with_oracle_results(pool):
    reqs = make_requests(40, 300)
    done, be, srv = run(reqs, pool)
    assert len(done) == 40 and all(r.status == "done" for r in done)
    d, d_off = pool
    for r in reqs[:5]:
        sc = oracle.maxsim(r.query, [0, len(r.query)], d, d_off, [0, len(r.cand_ids)], r.cand_ids)
        ids, _ = oracle.topk(sc, 10, r.cand_ids.astype(np.int64))
        assert r.top_ids.tolist() == ids.tolist()
        assert r.latency >= 0


def test_slots_bound_the_batches_in_flight(pool):
    reqs = make_requests(30, 300, rate=1e6)
    done, be, srv = run(reqs, pool, max_inflight=1, per_pair=1e-4)
    assert be.max_inflight_seen == 1
    assert all(r.status == "done" for r in done)


def test_memory_budget_limits_a_batch(pool):
    reqs = make_requests(12, 300, rate=1e6)
    one = S.request_bytes(6, 80, 64, 10)
    done, be, srv = run(reqs, pool, mem_budget=2 * one + 1, max_inflight=4, per_pair=1e-4)
    assert all(len(b.requests) <= 2 for _, b in be.launches)
    assert all(r.status == "done" for r in done)


def test_oversized_request_is_rejected(pool):
    reqs = make_requests(3, 300)
    reqs[1].cand_ids = np.arange(300, dtype=np.int32)
    small = S.request_bytes(6, 80, 64, 10)
    done, _, _ = run(reqs, pool, mem_budget=small)
    st = {r.rid: r.status for r in done}
    assert st[1] == "rejected" and st[0] == "done" and st[2] == "done"


def test_arrivals_join_while_a_batch_runs(pool):
    # two slots: the second batch launches before the first completes
    reqs = make_requests(2, 300)
    reqs[0].arrival, reqs[1].arrival = 0.0, 0.001
    done, be, srv = run(reqs, pool, max_inflight=2, per_pair=1e-3)
    (t0, b0), (t1, b1) = be.launches
    first_done = min(r.done_at for r in b0.requests)
    assert t1 < first_done
    assert [r.rid for r in b0.requests] == [0] and [r.rid for r in b1.requests] == [1]


def test_requests_queued_behind_a_busy_slot_are_batched_together(pool):
    reqs = make_requests(6, 300)
    for i, r in enumerate(reqs):
        r.arrival = 0.0 if i == 0 else 0.001 * i
    done, be, srv = run(reqs, pool, max_inflight=1, per_pair=1e-3)
    sizes = [len(b.requests) for _, b in be.launches]
    assert sizes[0] == 1 and sum(sizes) == 6 and max(sizes[1:]) > 1


def test_deadline_expires_in_the_queue(pool):
    reqs = make_requests(3, 300)
    for r in reqs:
        r.arrival = 0.0
    reqs[2].deadline = 0.005
    done, be, srv = run(reqs, pool, max_inflight=1, max_batch_requests=1, per_pair=1e-3)
    st = {r.rid: r.status for r in done}
    assert st[2] == "timeout" and st[0] == "done" and st[1] == "done"


def test_cancellation(pool):
    reqs = make_requests(3, 300)
    for r in reqs:
        r.arrival = 0.0
    clock = SimClock()
    be = FakeBackend(clock, pool, per_pair=1e-3)
    srv = S.Server(S.Scheduler(dim=64, k=10, max_inflight=1, max_batch_requests=1), be,
                   clock=clock, idle=clock.idle)
    done = srv.run(reqs, cancel_at={2: 0.001})
    st = {r.rid: r.status for r in done}
    assert st[2] == "cancelled" and st[0] == "done"


def test_backend_failure_fails_only_its_batch(pool):
    reqs = make_requests(8, 300, rate=50.0)
    done, be, srv = run(reqs, pool, fail_rids={3}, max_batch_requests=1)
    st = {r.rid: r.status for r in done}
    assert st[3] == "error" and "injected" in next(r.error for r in done if r.rid == 3)
    assert all(st[i] == "done" for i in st if i != 3)


def test_queue_full_backpressure(pool):
    reqs = make_requests(10, 300)
    for r in reqs:
        r.arrival = 0.0
    done, be, srv = run(reqs, pool, max_inflight=1, max_batch_requests=1, max_queue=3,
                        per_pair=1e-3)
    st = [r.status for r in done]
    assert st.count("rejected") >= 1 and st.count("done") >= 3


def test_latency_stats():
    rs = [S.Request(i, np.zeros((1, 4), np.float32), np.zeros(1, np.int32), arrival=0.0)
          for i in range(100)]
    for i, r in enumerate(rs):
        r.status, r.done_at = "done", (i + 1) * 1e-3
    st = S.latency_stats(rs)
    assert st["n"] == 100 and abs(st["p50_ms"] - 50.5) < 1e-6 and st["p99_ms"] > 99


def test_residual_requests_are_charged_for_their_table_columns():
    # a residual-mode request also holds up to 64 FP32 table entries per
    # centroid; exact and PQ requests do not
    sched = S.Scheduler(64, 10, mem_budget=1 << 30, residual_centroids=1000)
    q = np.zeros((6, 64), np.float32)
    ids = np.arange(80, dtype=np.int32)
    base = S.request_bytes(6, 80, 64, 10)
    assert sched.cost(S.Request(0, q, ids, mode="exact")) == base
    assert sched.cost(S.Request(1, q, ids, mode="pq")) == base
    assert sched.cost(S.Request(2, q, ids, mode="residual")) == base + 1000 * 64 * 4
    # a budget that fits the request but not its table rejects it
    tight = S.Scheduler(64, 10, mem_budget=base + 1000, residual_centroids=1000)
    r = S.Request(3, q, ids, mode="residual")
    assert not tight.submit(r) and r.status == "rejected"


def test_request_charge_covers_the_library_topk_workspace():
    # the memory admission charges at least the top-k workspace the library
    # itself asks for per segment (maxsim_topk_workspace_size)
    from paper_2606_26439_amd import _binding as B
    for k in (1, 10, 100, 1024):
        ws = B.topk_workspace_bytes(1, k)
        assert ws > 0
        assert S.request_bytes(1, 1, 64, k) >= ws + 8 * k
        assert S.Scheduler(64, k).cost(S.Request(0, np.zeros((1, 64), np.float32),
                                                 np.zeros(1, np.int32))) >= ws
    # n segments need n times one segment's workspace
    assert B.topk_workspace_bytes(7, 100) == 7 * B.topk_workspace_bytes(1, 100)


class SlotBackend(FakeBackend):
    """FakeBackend with GpuBackend's slot discipline: a fixed number of
    execution slots, taken at launch and given back by results() or
    release(); a launch without a free slot raises. `poll_fail` / `launch_fail`
    name request ids whose poll / launch raises (once each)."""

    def __init__(self, clock, pool, n_slots=1, poll_fail=(), launch_fail=(), **kw):
        super().__init__(clock, pool, **kw)
        self.free = n_slots
        self.poll_fail, self.launch_fail = set(poll_fail), set(launch_fail)
        self.released = 0

    def launch(self, batch):
        if self.free == 0:
            raise RuntimeError("no free execution slot")
        hit = self.launch_fail & {r.rid for r in batch.requests}
        if hit:
            self.launch_fail -= hit
            raise RuntimeError("injected launch failure")  # nothing taken
        self.free -= 1
        return super().launch(batch)

    def poll(self, h):
        hit = self.poll_fail & {r.rid for r in h["batch"].requests}
        if hit:
            self.poll_fail -= hit
            raise RuntimeError("injected poll failure")
        return super().poll(h)

    def results(self, h):
        try:
            return super().results(h)
        finally:
            self.free += 1

    def release(self, h):
        self._inflight -= 1
        self.free += 1
        self.released += 1


@pytest.mark.parametrize("n_slots", [1, 2])
def test_failed_poll_gives_its_slot_back(pool, n_slots):
    # a batch whose poll raises fails its own requests; its slot returns, so
    # every later batch still runs (with no release, all of them would fail
    # with "no free execution slot")
    reqs = make_requests(10, 300, rate=1e6)
    clock = SimClock()
    be = SlotBackend(clock, pool, n_slots=n_slots, poll_fail={2, 5}, per_pair=1e-4)
    srv = S.Server(S.Scheduler(dim=64, k=10, max_inflight=n_slots, max_batch_requests=1), be,
                   clock=clock, idle=clock.idle)
    done = srv.run(reqs)
    st = {r.rid: r.status for r in done}
    assert st[2] == "error" and st[5] == "error"
    assert all(st[i] == "done" for i in st if i not in (2, 5)), st
    assert be.released == 2 and be.free == n_slots


def test_failed_launch_leaves_no_slot_taken(pool):
    reqs = make_requests(6, 300, rate=1e6)
    clock = SimClock()
    be = SlotBackend(clock, pool, n_slots=1, launch_fail={1}, per_pair=1e-4)
    srv = S.Server(S.Scheduler(dim=64, k=10, max_inflight=1, max_batch_requests=1), be,
                   clock=clock, idle=clock.idle)
    done = srv.run(reqs)
    st = {r.rid: r.status for r in done}
    assert st[1] == "error" and all(st[i] == "done" for i in st if i != 1), st
    assert be.free == 1 and be.released == 0
