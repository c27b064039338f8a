"""Continuous-batching request loop over a device-resident document pool.

Requests (a query's token vectors plus a candidate id list) arrive at any
time. The scheduler admits queued requests into the next batch whenever an
execution slot is free and the batch's device memory fits the budget; a
batch is one multi-query call of the fused scorer with the per-request top-k
selected in its epilogue (or the fused PQ scorer, or the residual-compressed
scorer, followed by the per-request top-k), enqueued on its own HIP stream, so batches
formed while earlier ones are still on the GPU overlap with them. Every score
is produced by one wavefront with a fixed reduction order, so a request's
result does not depend on which batch carried it.

The scheduler is pure host logic; the device work sits behind a Backend with
launch / poll / results, so the admission, slot, timeout, cancellation and
failure paths run on the CPU with a fake backend and an injected clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    query: np.ndarray          # [Nq, d] float32 (converted on the device)
    cand_ids: np.ndarray       # [n_cand] int32 ids into the pool
    arrival: float = 0.0       # clock time of arrival
    mode: str = "exact"        # "exact" (fused MaxSim), "pq" (fused PQ) or
                               # "residual" (residual-compressed documents)
    deadline: Optional[float] = None
    # filled on completion
    status: str = "pending"    # pending | queued | running | done | timeout | cancelled | error | rejected
    error: str = ""
    done_at: Optional[float] = None
    top_ids: Optional[np.ndarray] = None
    top_scores: Optional[np.ndarray] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_at is None else self.done_at - self.arrival


def topk_workspace_per_request(k: int) -> int:
    """Bytes of top-k workspace one request's segment needs, as the library
    sizes it (maxsim_topk_workspace_size for one segment; a host call, no
    device needed)."""
    from . import _binding as B
    return B.topk_workspace_bytes(1, k)


def request_bytes(nq: int, n_cand: int, dim: int, k: int, elem: int = 2,
                  topk_ws: Optional[int] = None) -> int:
    """Device bytes a request occupies while in flight: query tokens (FP32
    staging + converted copy), candidate ids and scores, its query and
    candidate offsets, top-k outputs and its segment of the top-k workspace
    (the library's own figure unless `topk_ws` is given)."""
    if topk_ws is None:
        topk_ws = topk_workspace_per_request(k)
    return nq * dim * (4 + elem) + 8 * n_cand + 16 + 8 * k + topk_ws + 8


@dataclasses.dataclass
class Batch:
    bid: int
    requests: List[Request]
    mode: str
    nbytes: int
    handle: object = None
    launched_at: float = 0.0


class Scheduler:
    """Admission by free execution slots and a device-memory budget."""

    def __init__(self, dim: int, k: int = 100, max_inflight: int = 2,
                 mem_budget: int = 4 << 30, max_batch_requests: int = 64,
                 max_batch_pairs: int = 4_000_000, max_queue: int = 100_000,
                 residual_centroids: int = 0, batch_overhead: int = 0):
        self.dim, self.k = dim, k
        # device bytes a batch holds beyond what its requests are charged
        # (GpuBackend.batch_overhead: the fused top-k's per-workgroup parts)
        self.batch_overhead = batch_overhead
        self.topk_ws = topk_workspace_per_request(k)
        # a residual-mode request also holds its columns of the centroid-query
        # table: up to 64 (the query-token bound) FP32 entries per centroid
        self.residual_table_bytes = residual_centroids * 64 * 4
        self.max_inflight = max_inflight
        self.mem_budget = mem_budget
        self.max_batch_requests = max_batch_requests
        self.max_batch_pairs = max_batch_pairs
        self.max_queue = max_queue
        self.queue: collections.deque = collections.deque()
        self.inflight: List[Batch] = []
        self.mem_in_use = 0
        self._next_bid = 0

    def cost(self, r: Request) -> int:
        c = request_bytes(len(r.query), len(r.cand_ids), self.dim, self.k, topk_ws=self.topk_ws)
        if r.mode == "residual":
            c += self.residual_table_bytes
        return c

    def submit(self, r: Request) -> bool:
        """Queues a request; rejects one that can never fit or a full queue."""
        if (self.cost(r) + self.batch_overhead > self.mem_budget
                or len(r.cand_ids) > self.max_batch_pairs):
            r.status, r.error = "rejected", "request exceeds the device memory budget"
            return False
        if len(self.queue) >= self.max_queue:
            r.status, r.error = "rejected", "queue full"
            return False
        r.status = "queued"
        self.queue.append(r)
        return True

    def expire(self, now: float) -> List[Request]:
        """Removes queued requests whose deadline has passed."""
        out, keep = [], collections.deque()
        for r in self.queue:
            if r.deadline is not None and now > r.deadline:
                r.status, r.error, r.done_at = "timeout", "deadline passed while queued", now
                out.append(r)
            else:
                keep.append(r)
        self.queue = keep
        return out

    def cancel(self, rid: int, now: float) -> bool:
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                r.status, r.done_at = "cancelled", now
                return True
        return False

    def next_batch(self) -> Optional[Batch]:
        """Forms the next batch from the head of the queue (FIFO, one mode per
        batch) if a slot is free and at least one request fits the memory left."""
        if len(self.inflight) >= self.max_inflight or not self.queue:
            return None
        mode = self.queue[0].mode
        picked, nbytes, pairs = [], 0, 0
        free = self.mem_budget - self.mem_in_use - self.batch_overhead
        while self.queue and len(picked) < self.max_batch_requests:
            r = self.queue[0]
            if r.mode != mode:
                break
            c = self.cost(r)
            if nbytes + c > free or pairs + len(r.cand_ids) > self.max_batch_pairs:
                break
            picked.append(self.queue.popleft())
            nbytes += c
            pairs += len(r.cand_ids)
        if not picked:
            return None
        nbytes += self.batch_overhead
        b = Batch(self._next_bid, picked, mode, nbytes)
        self._next_bid += 1
        for r in picked:
            r.status = "running"
        self.mem_in_use += nbytes
        self.inflight.append(b)
        return b

    def finish(self, b: Batch):
        self.inflight.remove(b)
        self.mem_in_use -= b.nbytes


class Backend:
    """Device-side executor interface."""

    def launch(self, batch: Batch) -> object:
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def results(self, handle) -> List[tuple]:
        """Per request, (top ids int64 [k], top scores float32 [k])."""
        raise NotImplementedError

    def release(self, handle):
        """Gives back what a launched batch holds when it failed after its
        launch (its poll or results raised): the server calls this instead of
        results()."""


class GpuBackend(Backend):
    """Launches a batch on a stream of its own; completion is an event poll.
    Exact batches are one fused score + top-k call (the per-request top-k
    selected in the scorer's epilogue, no score array); PQ and residual
    batches are one scoring call and one top-k call.

    Each in-flight slot owns a stream, a pinned host staging buffer, a
    device input buffer, the converted query tokens, the fused call's
    workspace and its top-k rows (each grown on demand, then reused: they
    stay allocated while the backend lives, at most the largest batch's
    size per slot), so a batch costs one packed host-to-device copy, the
    conversion of its query tokens, the scoring (and top-k) launches and one
    device-to-host copy of the top-k rows, and no allocation once the slots
    have grown."""

    def __init__(self, pool_docs, pool_pq=None, k: int = 100, n_slots: int = 3,
                 device: str = "cuda", pool_res=None):
        import torch
        from . import _binding as B
        self.torch, self.B = torch, B
        self.docs, self.pq, self.k, self.device = pool_docs, pool_pq, k, device
        self.res = pool_res
        self.slots = [dict(stream=torch.cuda.Stream(device=device), busy=False, cap=0)
                      for _ in range(n_slots)]

    def batch_overhead(self, max_requests: int = 64, max_pairs: int = 4_000_000) -> int:
        """Device bytes an exact batch holds beyond its requests' charge: the
        fused score + top-k workspace of the largest batch the scheduler can
        form (as the library sizes it, for every query-length class), less
        the 4 bytes per (query, candidate) pair each request is already
        charged for its scores (the call's key spill takes their place).
        A host-side size query: the descriptors carry no device data."""
        import ctypes
        B = self.B
        dt = self.docs.dtype
        worst = 0
        for max_len in (16, 32, 64):
            qc = B.CSR(B.DTYPES[dt], self.docs.dim, max_requests, max_requests * max_len,
                       max_len, 0, 16, 16, 16 if dt == "fp8" else None)
            dc = self.docs.csr()
            cc = B.Cand(16, 16, max_pairs)
            n = int(B.lib().maxsim_score_topk_workspace_size(
                ctypes.byref(qc), ctypes.byref(dc), ctypes.byref(cc), self.k))
            if n == 0:
                raise RuntimeError("score_topk workspace size query failed: "
                                   + B.lib().maxsim_last_error().decode())
            worst = max(worst, n)
        return max(0, worst - 4 * max_pairs)

    def _slot(self):
        for sl in self.slots:
            if not sl["busy"]:
                return sl
        raise RuntimeError("no free execution slot (scheduler admitted too many batches)")

    def _ensure(self, sl, nbytes, n_req):
        torch = self.torch
        if sl["cap"] < nbytes:
            cap = max(nbytes, 2 * sl["cap"], 1 << 20)
            sl["host"] = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
            sl["dev"] = torch.empty(cap, dtype=torch.uint8, device=self.device)
            sl["cap"] = cap
        if sl.get("nreq", 0) < n_req:
            n = max(n_req, 2 * sl.get("nreq", 0), 16)
            sl["out_s"] = torch.empty((n, self.k), dtype=torch.float32, pin_memory=True)
            sl["out_i"] = torch.empty((n, self.k), dtype=torch.int32, pin_memory=True)
            sl["top_s"] = torch.empty((n, self.k), dtype=torch.float32, device=self.device)
            sl["top_i"] = torch.empty((n, self.k), dtype=torch.int32, device=self.device)
            sl["nreq"] = n

    def _grown(self, sl, key, shape, dtype):
        """A slot buffer of at least shape[0] rows (grown on demand), as a
        contiguous view of exactly `shape`."""
        torch = self.torch
        buf = sl.get(key)
        if buf is None or buf.shape[0] < shape[0] or buf.dtype != dtype:
            rows = max(shape[0], 2 * (buf.shape[0] if buf is not None else 0), 1)
            buf = torch.empty((rows,) + tuple(shape[1:]), dtype=dtype, device=self.device)
            sl[key] = buf
        return buf[:shape[0]]

    def launch(self, batch: Batch):
        reqs = batch.requests
        sl = self._slot()
        s = sl["stream"]
        nq = np.fromiter((len(r.query) for r in reqs), np.int64, len(reqs))
        nc = np.fromiter((len(r.cand_ids) for r in reqs), np.int64, len(reqs))
        dim = reqs[0].query.shape[1]
        tq, tc, n = int(nq.sum()), int(nc.sum()), len(reqs)
        # packed layout: q_off | c_off (int64) | query tokens (f32) | ids (i32)
        o_q, o_c = 0, 8 * (n + 1)
        o_tok = o_c + 8 * (n + 1)
        o_ids = o_tok + 4 * tq * dim
        nbytes = o_ids + 4 * tc
        self._ensure(sl, nbytes, n)
        h = sl["host"].numpy()
        q_off = h[o_q:o_c].view(np.int64)
        q_off[0] = 0
        np.cumsum(nq, out=q_off[1:])
        c_off = h[o_c:o_tok].view(np.int64)
        c_off[0] = 0
        np.cumsum(nc, out=c_off[1:])
        np.concatenate([r.query for r in reqs], out=h[o_tok:o_ids].view(np.float32).reshape(tq, dim))
        np.concatenate([r.cand_ids for r in reqs], out=h[o_ids:nbytes].view(np.int32))
        try:
            handle = self._enqueue(batch, sl, nq, tq, tc, n, dim, o_q, o_c, o_tok, o_ids, nbytes)
        except BaseException:
            # work may already be queued on the slot's stream (the copy out of
            # its pinned buffer): let it drain before the slot is reused
            try:
                s.synchronize()
            finally:
                sl["busy"] = False
            raise
        return handle

    def _enqueue(self, batch, sl, nq, tq, tc, n, dim, o_q, o_c, o_tok, o_ids, nbytes):
        torch, B = self.torch, self.B
        s, d = sl["stream"], sl["dev"]
        # the slot is taken from the first enqueued operation on
        sl["busy"] = True
        with torch.cuda.stream(s):
            d[:nbytes].copy_(sl["host"][:nbytes], non_blocking=True)
            qoff = d[o_q:o_c].view(torch.int64)
            coff = d[o_c:o_tok].view(torch.int64)
            q32 = d[o_tok:o_ids].view(torch.float32).view(tq, dim)
            ids = d[o_ids:nbytes].view(torch.int32)
            cand = B.Candidates(coff, ids)
            if batch.mode in ("pq", "residual"):
                qt = self._grown(sl, "qt16", (tq, dim), torch.float16)
                B.quantize(q32, "f16", stream=s, out=qt)
                Q = B.Tokens(qt, qoff, "f16", None, max_len=int(nq.max()))
                scores = self._grown(sl, "sc", (tc,), torch.float32)
                if batch.mode == "pq":
                    need = B.pq_workspace_bytes(Q, self.pq, cand)
                    ws = self._grown(sl, "ws", (max(need, 1),), torch.uint8)
                    B.pq_score(Q, self.pq, cand, out=scores, workspace=ws, stream=s)
                else:
                    need = B.residual_workspace_bytes(Q, self.res, cand)
                    ws = self._grown(sl, "ws", (max(need, 1),), torch.uint8)
                    B.residual_score(Q, self.res, cand, out=scores, workspace=ws, stream=s)
            else:
                dt = self.docs.dtype
                qt = self._grown(sl, "qt", (tq, dim), B.TORCH_DTYPES[dt])
                qs = self._grown(sl, "qs", (tq,), torch.float32) if dt == "fp8" else None
                B.quantize(q32, dt, stream=s, out=qt, scales=qs)
                Q = B.Tokens(qt, qoff, dt, qs, max_len=int(nq.max()))
                scores = None
                ws = self._grown(sl, "ws", (max(B.score_topk_workspace_bytes(Q, self.docs, self.k,
                                                                              cand), 1),),
                                 torch.uint8)
                ts, ti = B.score_topk(Q, self.docs, self.k, cand, workspace=ws,
                                      out=(sl["top_s"][:n], sl["top_i"][:n]), stream=s)
            if scores is not None:
                tws = self._grown(sl, "tkws", (max(B.topk_workspace_bytes(n, self.k), 1),),
                                  torch.uint8)
                ts, ti = B.topk(scores, coff, self.k, ids=ids, n_total=tc, workspace=tws,
                                stream=s, out=(sl["top_s"][:n], sl["top_i"][:n]))
            sl["out_s"][:n].copy_(ts, non_blocking=True)
            sl["out_i"][:n].copy_(ti, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        # the device temporaries stay referenced until the event has completed
        return (ev, sl, n, (qt, scores, ts, ti))

    def poll(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        ev, sl, n, _ = handle
        try:
            ev.synchronize()
            out_s, out_i = sl["out_s"].numpy(), sl["out_i"].numpy()
            return [(out_i[i].astype(np.int64), out_s[i].copy()) for i in range(n)]
        finally:
            sl["busy"] = False

    def release(self, handle):
        _, sl, _, _ = handle
        try:
            sl["stream"].synchronize()
        finally:
            sl["busy"] = False


class Server:
    """Drives the scheduler and a backend against a clock.

    run(requests) replays an open-loop arrival sequence (each request's
    `arrival` is its scheduled time) and returns when every request is
    finished; completed requests carry their latency (arrival -> results on
    the host)."""

    def __init__(self, scheduler: Scheduler, backend: Backend,
                 clock: Callable[[], float] = time.perf_counter,
                 idle: Callable[[float], None] = None):
        self.sched, self.backend, self.clock = scheduler, backend, clock
        self.idle = idle if idle is not None else (lambda dt: None)
        self.completed: List[Request] = []
        self.batches_launched = 0
        self.max_queue_depth = 0

    def _complete_batch(self, b: Batch, now: float):
        try:
            if isinstance(b.handle, _Failed):
                if b.handle.handle is not None:
                    # launched, then its poll raised: free what it holds
                    try:
                        self.backend.release(b.handle.handle)
                    except Exception:  # noqa: BLE001 -- the batch fails either way
                        pass
                raise b.handle.e
            res = self.backend.results(b.handle)
            for r, (ids, sc) in zip(b.requests, res):
                r.top_ids, r.top_scores, r.status, r.done_at = ids, sc, "done", now
        except Exception as e:  # noqa: BLE001 -- a failed batch fails its own requests only
            for r in b.requests:
                r.status, r.error, r.done_at = "error", f"{type(e).__name__}: {e}", now
        self.completed.extend(b.requests)
        self.sched.finish(b)

    def pump(self) -> bool:
        """One scheduling iteration. Returns True if anything progressed."""
        now = self.clock()
        progressed = False
        for r in self.sched.expire(now):
            self.completed.append(r)
            progressed = True
        for b in list(self.sched.inflight):
            if isinstance(b.handle, _Failed):
                ready = True
            else:
                try:
                    ready = self.backend.poll(b.handle)
                except Exception as e:  # noqa: BLE001
                    ready = True
                    b.handle = _Failed(e, b.handle)
            if ready:
                self._complete_batch(b, self.clock())
                progressed = True
        while True:
            b = self.sched.next_batch()
            if b is None:
                break
            b.launched_at = self.clock()
            try:
                b.handle = self.backend.launch(b)
            except Exception as e:  # noqa: BLE001
                b.handle = _Failed(e)
            self.batches_launched += 1
            progressed = True
        self.max_queue_depth = max(self.max_queue_depth, len(self.sched.queue))
        return progressed

    def run(self, requests: List[Request], cancel_at: Dict[int, float] = None) -> List[Request]:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        cancels = sorted((t, rid) for rid, t in (cancel_at or {}).items())
        total = len(pending)
        self.completed = []
        while len(self.completed) < total:
            now = self.clock()
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                if not self.sched.submit(r):
                    r.done_at = now
                    self.completed.append(r)
            while cancels and cancels[0][0] <= now:
                _, rid = cancels.pop(0)
                if self.sched.cancel(rid, now):
                    self.completed.extend(r for r in requests if r.rid == rid)
            if not self.pump():
                nxt = pending[0].arrival if pending else None
                self.idle(0.0 if nxt is None else max(0.0, nxt - self.clock()))
        return self.completed


class _Failed:
    """Handle of a batch whose launch or poll raised; `handle` is the
    backend's handle when the launch itself had succeeded."""

    def __init__(self, e, handle=None):
        self.e, self.handle = e, handle


def latency_stats(reqs: List[Request]) -> dict:
    lat = np.array([r.latency for r in reqs if r.status == "done"], np.float64)
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
