"""Request loop for P(k) + bispectrum jobs on one GPU (continuous batching).

Requests carry a field already on the device (for masked surveys the data
d = w * delta and the window w) and ask for the binned power spectrum and
bispectrum on their own grid and binning.  The server

* keeps one device-resident plan per (grid, box, edges): bin tables and
  the FP64 triangle counts are computed once and reused by every request
  with that geometry;
* admits requests in arrival order while a slot is free and the HBM the
  job needs (its workspace and outputs) fits the budget; that memory is a
  range of one device allocation of the whole budget, taken first-fit and
  given back when the batch retires, so serving makes no device
  allocation per request (a caching allocator fed a stream of mixed sizes
  fragments, and when it runs short it frees its cache, which waits for
  all work in flight); queued requests
  with the same plan as the one being admitted join it in one batched
  launch sequence (up to 8 jobs share the launches);
* runs every admitted batch on its own slot stream, so work of different
  requests overlaps on the device, and retires it when its completion
  event has fired, freeing the slot and the memory;
* with simulations attached, gives B the linear term of the numerator
  (Monte Carlo average, Sec. IV.C) before normalising (such requests
  batch only with each other, and their batch computes P alone: B comes
  from the linear-term call);
* normalises masked requests by the window moments (P / <w^2>,
  B / <w^3>: the conventional windowed estimators of Sec. III.D.2 and
  Sec. IV.D.2), and, when the request brings random fields, also returns
  the unwindowed power spectrum with the Monte Carlo Fisher matrix of
  Sec. III.C.2 (pb3_masked_power, on a full-grid power-only plan);
* records arrival, admission and completion times per request.

Each job's result depends only on its own inputs: the kernels and their
reduction orders do not depend on what else is in flight, so a result in
the mix equals the result computed alone, bit for bit.  The loop is
single-threaded: call :meth:`Server.poll` (or :meth:`Server.run_until_idle`)
to make progress.  Every device computation goes through the C ABI of
``libpb3.so``; this module only schedules.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import Batch, Plan, Pb3Error, _lib

__all__ = ["Request", "Completed", "Server"]

_MAX_JOBS_PER_LAUNCH = 8


@dataclass
class Request:
    """One estimator job.  ``data`` is an N^3 float32 CUDA tensor; ``window``
    (same shape, or None for an unmasked box) is the mask that multiplied it.
    ``edges`` are bin edges in units of k_f.  ``arrival`` is a
    ``time.perf_counter`` stamp (defaults to submission time); ``ready`` an
    optional CUDA event after which the inputs are valid; ``deadline`` an
    optional perf_counter stamp after which a request that is still queued
    expires."""

    rid: int
    grid: int
    box: float
    edges: np.ndarray
    data: object
    window: object = None
    precision: str = "mixed"
    arrival: float | None = None
    ready: object = None
    deadline: float | None = None
    grfs: list | None = None  # white unit-variance N^3 CUDA fields for the Monte Carlo Fisher matrix
    sims: list | None = None  # N^3 CUDA fields with about the data's covariance: B gets the linear term


@dataclass
class Completed:
    rid: int
    status: str  # "ok", "rejected", "cancelled", "expired", "error"
    pk: np.ndarray | None = None
    bk: np.ndarray | None = None
    moments: np.ndarray | None = None  # (<w^2>, <w^3>) for masked requests
    pk_unwindowed: np.ndarray | None = None  # F^-1 p with the Monte Carlo Fisher matrix
    fisher: np.ndarray | None = None
    arrival: float = 0.0
    admitted: float = 0.0
    done: float = 0.0
    batch_size: int = 0
    message: str = ""
    mc_ms: float = 0.0  # device time of the Monte Carlo masked power spectrum (random fields), if any

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def wait(self) -> float:
        return self.admitted - self.arrival

    @property
    def service(self) -> float:
        return self.done - self.admitted


@dataclass
class _Running:
    reqs: list
    slot: int
    batch: object
    workspace: object
    pks: list
    bks: list
    scratch: list
    unw: list
    event: object
    nbytes: int
    admitted: float
    pool_key: tuple
    mc_events: list = field(default_factory=list)  # per request: (start, end) events of the MC call, or None
    block: int = -1  # offset of the batch's range in the arena


class _Arena:
    """First-fit ranges of one device allocation (256-byte aligned)."""

    ALIGN = 256

    def __init__(self, torch, nbytes: int):
        self.buf = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")
        self.free = [(0, self.buf.numel())]  # (offset, size), sorted, coalesced

    @classmethod
    def up(cls, n: int) -> int:
        return (max(int(n), 1) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    def take(self, n: int):
        n = self.up(n)
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    del self.free[i]
                else:
                    self.free[i] = (o + n, sz - n)
                return o
        return None

    def give(self, off: int, n: int):
        n = self.up(n)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, sz in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + sz)
            else:
                merged.append((o, sz))
        self.free = merged

    def view(self, off: int, n: int, dtype=None, shape=None):
        t = self.buf[off:off + int(n)]
        if dtype is not None:
            t = t.view(dtype)
        return t if shape is None else t.view(shape)


@dataclass
class _Stats:
    admitted: int = 0
    launches: int = 0
    max_in_flight: int = 0
    max_queue: int = 0
    bytes_peak: int = 0
    batch_sizes: list = field(default_factory=list)


class Server:
    """Continuous-batching request loop (see the module docstring).

    hbm_budget: bytes of device memory the server may hold for running
    jobs (workspaces, outputs, scratch); max_slots: batches in flight at
    once, each on its own stream.
    """

    def __init__(self, hbm_budget: int, max_slots: int = 4, merge_same_plan: bool = True):
        import torch

        _lib.load()
        self.torch = torch
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.merge = merge_same_plan
        self.streams = [torch.cuda.Stream() for _ in range(self.max_slots)]
        self.free_slots = list(range(self.max_slots))
        self.queue: deque = deque()
        self.running: list[_Running] = []
        self.done: dict[int, Completed] = {}
        self.plans: dict = {}
        self.full_plans: dict = {}  # full-grid power-only plans for the Monte Carlo Fisher matrix
        self.pool: dict = {}  # (plan key, jobs) -> idle Batch objects (no workspace held)
        self.arena: _Arena | None = None  # the budget, allocated at the first admission
        self.bytes_in_use = 0
        self.stats = _Stats()

    # ------------------------------------------------------------ plans
    def plan_for(self, grid: int, box: float, edges) -> Plan:
        key = (int(grid), float(box), tuple(np.asarray(edges, dtype=np.float64).tolist()))
        p = self.plans.get(key)
        if p is None:
            p = Plan(grid, box, edges, ext_workspace=True)
            self.plans[key] = p
        return p

    def full_plan_for(self, grid: int, box: float, edges) -> Plan:
        key = (int(grid), float(box), tuple(np.asarray(edges, dtype=np.float64).tolist()))
        p = self.full_plans.get(key)
        if p is None:
            p = Plan(grid, box, edges, full_grid=True, power_only=True, ext_workspace=True)
            self.full_plans[key] = p
        return p

    @staticmethod
    def _plan_key(req: Request):
        return (int(req.grid), float(req.box), tuple(np.asarray(req.edges, dtype=np.float64).tolist()))

    def _layout(self, plan: Plan, group: list):
        """Ranges (offset, bytes) within a batch's block of everything the
        batch holds while it runs: the jobs' workspaces, outputs and window
        scratch, and one Monte Carlo and one linear-term workspace, which
        the jobs use in turn on the slot stream.  Returns (ranges, bytes)."""
        up = _Arena.up
        lay, off = {}, 0

        def take(key, n):
            nonlocal off
            lay[key] = (off, int(n))
            off += up(n)

        nb, nt = plan.n_bins, plan.n_triplets
        take("ws", len(group) * int(plan.workspace_bytes))
        mws = lws = 0
        for j, r in enumerate(group):
            take(("pk", j), 8 * nb)
            take(("bk", j), 8 * nt)
            if r.window is not None:
                take(("sc", j), 8 * _lib.WINDOW_SCRATCH)
            if r.grfs:
                take(("pu", j), 8 * nb)
                take(("F", j), 8 * nb * nb)
                mws = max(mws, int(self.full_plan_for(r.grid, r.box, r.edges).masked_workspace_bytes))
            if r.sims:
                lws = max(lws, int(plan.linear_workspace_bytes(len(r.sims))))
        if mws:
            take("mws", mws)
        if lws:
            take("lws", lws)
        return lay, off

    def job_bytes(self, plan: Plan, masked: bool, full: Plan | None = None) -> int:
        """HBM one job holds while it runs (its workspace, outputs, the
        window scratch and, with a full-grid plan for random fields, the
        Monte Carlo workspace and outputs), in 256-byte aligned ranges."""
        up = _Arena.up
        nb = plan.n_bins
        n = up(plan.workspace_bytes) + up(8 * nb) + up(8 * plan.n_triplets)
        n += up(8 * _lib.WINDOW_SCRATCH) if masked else 0
        if full is not None:
            n += up(8 * nb) + up(8 * nb * nb) + up(full.masked_workspace_bytes)
        return n

    def _req_bytes(self, plan: Plan, r: Request) -> int:
        return self._layout(plan, [r])[1]

    # ----------------------------------------------------------- submit
    def submit(self, req: Request):
        if req.arrival is None:
            req.arrival = time.perf_counter()
        n = req.grid
        if tuple(req.data.shape) != (n, n, n):
            raise ValueError("data shape does not match the grid")
        if req.window is not None and tuple(req.window.shape) != (n, n, n):
            raise ValueError("window shape does not match the grid")
        if req.grfs and req.window is None:
            raise ValueError("random fields are for masked requests (a window is needed)")
        for f in req.sims or []:
            if tuple(f.shape) != (n, n, n):
                raise ValueError("simulation shape does not match the grid")
        self.queue.append(req)
        self.stats.max_queue = max(self.stats.max_queue, len(self.queue))

    def cancel(self, rid: int) -> bool:
        """Remove a still-queued request; running ones finish."""
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                self.done[rid] = Completed(rid, "cancelled", arrival=r.arrival, done=time.perf_counter())
                return True
        return False

    # ------------------------------------------------------------- loop
    def poll(self) -> int:
        """Retire finished batches, expire and admit queued requests;
        returns the number of requests retired."""
        n = self._retire()
        self._expire()
        self._admit()
        return n

    def run_until_idle(self, sleep: float = 5e-5):
        while self.queue or self.running:
            if self.poll() == 0 and self.running:
                time.sleep(sleep)

    @property
    def idle(self) -> bool:
        return not self.queue and not self.running

    def _expire(self):
        now = time.perf_counter()
        for r in list(self.queue):
            if r.deadline is not None and now > r.deadline:
                self.queue.remove(r)
                self.done[r.rid] = Completed(r.rid, "expired", arrival=r.arrival, done=now)

    def _admit(self):
        torch = self.torch
        while self.queue and self.free_slots:
            head = self.queue[0]
            try:
                plan = self.plan_for(head.grid, head.box, head.edges)
            except Pb3Error as e:
                self.queue.popleft()
                self.done[head.rid] = Completed(head.rid, "error", arrival=head.arrival,
                                                done=time.perf_counter(), message=str(e))
                continue
            try:
                need_one = self._req_bytes(plan, head)
            except Pb3Error as e:
                self.queue.popleft()
                self.done[head.rid] = Completed(head.rid, "error", arrival=head.arrival,
                                                done=time.perf_counter(), message=str(e))
                continue
            if need_one > self.budget:
                self.queue.popleft()
                self.done[head.rid] = Completed(head.rid, "rejected", arrival=head.arrival,
                                                done=time.perf_counter(),
                                                message=f"needs {need_one} bytes, budget {self.budget}")
                continue
            if self.bytes_in_use + need_one > self.budget:
                break  # wait for memory (arrival order is kept)
            if self.arena is None:
                self.arena = _Arena(torch, self.budget)
            # the head plus queued requests of the same plan and precision
            group = [head]
            used = need_one
            if self.merge:
                key = self._plan_key(head)
                for r in list(self.queue)[1:]:
                    if len(group) >= _MAX_JOBS_PER_LAUNCH:
                        break
                    if self._plan_key(r) == key and r.precision == head.precision and bool(r.sims) == bool(head.sims):
                        more = self._layout(plan, group + [r])[1]
                        if self.bytes_in_use + more > self.budget:
                            break
                        group.append(r)
                        used = more
            block = self.arena.take(used)
            while block is None and len(group) > 1:  # free bytes enough, but not in one range
                group.pop()
                used = self._layout(plan, group)[1]
                block = self.arena.take(used)
            if block is None:
                break  # wait until retiring batches give ranges back
            for r in group:
                self.queue.remove(r)
            self._launch(plan, group, used, block)

    def _launch(self, plan: Plan, group: list, nbytes: int, block: int):
        torch = self.torch
        slot = self.free_slots.pop(0)
        stream = self.streams[slot]
        now = time.perf_counter()
        pkey = (self._plan_key(group[0]), len(group))
        idle = self.pool.get(pkey)
        batch = idle.pop() if idle else Batch([plan] * len(group), ext_workspace=True)
        lay, total = self._layout(plan, group)
        assert total == nbytes and batch.workspace_bytes <= lay["ws"][1]

        def view(key, dtype=None, shape=None):
            o, n = lay[key]
            return self.arena.view(block + o, n, dtype, shape)

        f64 = torch.float64
        nb = plan.n_bins
        with torch.cuda.stream(stream):
            for r in group:
                if r.ready is not None:
                    stream.wait_event(r.ready)
            ws = view("ws")
            batch.bind_workspace(ws)
            pks = [view(("pk", j), f64) for j in range(len(group))]
            bks = [view(("bk", j), f64) for j in range(len(group))]
            with_sims = bool(group[0].sims)  # a group is all with or all without simulations
            batch.run([r.data for r in group], group[0].precision, pk_outs=pks, bk_outs=None if with_sims else bks,
                      bispectrum=not with_sims, stream=stream)
            scratch, unw, mc_ev = [], [], []
            for j, (r, pk, bk) in enumerate(zip(group, pks, bks)):
                mc = None
                if r.sims:
                    # B with the linear term (the batch computed P only)
                    plan.bispectrum_linear(r.data, r.sims, r.precision, out=bk, workspace=view("lws"), stream=stream)
                ev_mc = None
                if r.grfs:
                    # before the window normalisation, which rescales pk in place
                    full = self.full_plan_for(r.grid, r.box, r.edges)
                    ev_mc = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    ev_mc[0].record(stream)
                    mc = full.masked_power(r.data, r.window, r.grfs, pk_out=view(("pu", j), f64),
                                           fisher_out=view(("F", j), f64, (nb, nb)), workspace=view("mws"),
                                           stream=stream)
                    ev_mc[1].record(stream)
                unw.append(mc)
                mc_ev.append(ev_mc)
                if r.window is not None:
                    sc = view(("sc", j), f64)
                    plan.window_normalize(r.window, pk, bk, scratch=sc, stream=stream)
                    scratch.append(sc)
                else:
                    scratch.append(None)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.running.append(_Running(group, slot, batch, ws, pks, bks, scratch, unw, ev, nbytes, now, pkey, mc_ev,
                                     block))
        self.bytes_in_use += nbytes
        st = self.stats
        st.admitted += len(group)
        st.launches += batch.launches(True, not group[0].sims)
        st.batch_sizes.append(len(group))
        st.max_in_flight = max(st.max_in_flight, len(self.running))
        st.bytes_peak = max(st.bytes_peak, self.bytes_in_use)

    def _retire(self) -> int:
        n = 0
        for run in list(self.running):
            if not run.event.query():
                continue
            now = time.perf_counter()
            for r, pk, bk, sc, mc, me in zip(run.reqs, run.pks, run.bks, run.scratch, run.unw, run.mc_events):
                self.done[r.rid] = Completed(
                    r.rid, "ok", pk=pk.cpu().numpy(), bk=bk.cpu().numpy(),
                    moments=None if sc is None else sc[:2].cpu().numpy(),
                    pk_unwindowed=None if mc is None else mc[0].cpu().numpy(),
                    fisher=None if mc is None else mc[1].cpu().numpy(),
                    arrival=r.arrival, admitted=run.admitted, done=now, batch_size=len(run.reqs),
                    mc_ms=0.0 if me is None else float(me[0].elapsed_time(me[1])))
                n += 1
            self.running.remove(run)
            self.free_slots.append(run.slot)
            self.arena.give(run.block, run.nbytes)
            self.bytes_in_use -= run.nbytes
            self.pool.setdefault(run.pool_key, []).append(run.batch)
        return n

    def reset_stats(self):
        """Forget completed requests and counters (plans, pooled batches and
        cached memory stay)."""
        self.done.clear()
        self.stats = _Stats()

    # ---------------------------------------------------------- reports
    def summary(self, rids=None) -> dict:
        res = [c for c in self.done.values() if c.status == "ok" and (rids is None or c.rid in rids)]
        if not res:
            return {"completed": 0}
        lat = np.array([c.latency for c in res]) * 1e3
        wait = np.array([c.wait for c in res]) * 1e3
        svc = np.array([c.service for c in res]) * 1e3
        t0 = min(c.arrival for c in res)
        t1 = max(c.done for c in res)
        return {
            "completed": len(res),
            "rejected": sum(1 for c in self.done.values() if c.status == "rejected"),
            "throughput_per_s": len(res) / max(t1 - t0, 1e-9),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "admission_wait_ms": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
            "service_ms": {"p50": float(np.percentile(svc, 50)), "p99": float(np.percentile(svc, 99)),
                           "max": float(svc.max())},
            "max_in_flight_batches": self.stats.max_in_flight,
            "max_queue": self.stats.max_queue,
            "mean_batch_size": float(np.mean(self.stats.batch_sizes)) if self.stats.batch_sizes else 0.0,
            # device time of the Monte Carlo masked power spectrum per request, and its share of the
            # requests' total service time (admission to completion)
            "mc_ms": {"p50": float(np.percentile([c.mc_ms for c in res], 50)),
                      "p99": float(np.percentile([c.mc_ms for c in res], 99))},
            "mc_share_of_service": float(sum(c.mc_ms for c in res) / max(1e-9, 1e3 * sum(c.service for c in res))),
            "peak_bytes": self.stats.bytes_peak,
            "plans": len(self.plans),
        }
