"""Continuous-batching server for transient non-negative diffusion solves.

A request is a P1 problem (mesh, tensor, source) and a number of
backward-Euler steps (Sec. 2.2.2, eq. Eq:non-negative with lower bound 0),
each step a non-negative QP warm-started from the previous one.  The server:

* admits arrived requests first-in first-out while their device memory fits
  the HBM budget (estimated from the mesh, replaced by nn_matrix_bytes once
  assembled); a request larger than the whole budget is rejected;
* assembles admitted requests on worker threads, each with its own library
  context and stream, so assembly overlaps the solves already running;
* keeps K, M/dt + K, f, c and the active set of every resident request on the
  device for all of its steps;
* runs ticks: one batched call (nn_step_transient_batch) advances every
  resident request by one step; requests that arrive or finish assembling
  join at the next tick, finished requests leave and free their memory;
* routes requests by size to lanes that tick independently on their own
  streams, so small requests are not held by a large one's step; the upper
  lanes step each of their requests with the single-problem solver;
* cancels a request at its `cancel_at` time or on `Server.cancel(rid)` from
  any thread: a waiting request leaves the queue, an admitted one is dropped
  after its assembly or between ticks, its memory is freed and its budget
  returned; the steps it finished stay in its result.

Because a batch member's arithmetic does not depend on the other members, a
request's result is bitwise the same whether it is served alone or in any mix.

The inner CG tolerance defaults to TRON1's 0.1: a request's first step from
c = 0 is mass-dominated (M/dt >> K), its free set grows outward from the
source one ring of nodes per outer iteration, and a looser inner solve makes
each iteration reach less far (one 117k-DOF request took 1,544 outer
iterations at 0.5 against 92 at 0.1).
The Python here only sequences calls; every step runs in the HIP library.
"""
import collections
import concurrent.futures as cf
import dataclasses
import math
import threading
import time
from typing import List, Optional

import numpy as np

from . import nnqp

NN_EBUDGET = nnqp.NN_EBUDGET
CANCELLED = -1   # Result.status of a request cancelled before its last step


@dataclasses.dataclass
class Request:
    rid: int
    problem: object          # workloads.Problem
    steps: int
    arrival: float           # seconds after the stream starts
    cancel_at: float = math.inf   # seconds after the stream starts: the client cancels


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    steps: int
    arrival: float
    admitted: float = math.nan
    started: float = math.nan     # first tick that included the request
    finished: float = math.nan
    status: int = 0
    step_stats: list = dataclasses.field(default_factory=list)
    c: object = None              # final state (device tensor) when kept

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class Report:
    results: List[Result]
    makespan: float
    ticks: int
    mean_batch: float
    deferred: int                 # requests that waited for memory before admission
    peak_bytes: int
    budget: int
    lane_ticks: list = dataclasses.field(default_factory=list)   # ticks run by each lane
    final_bytes: int = 0          # budget still held when the stream ended (0: all returned)

    def summary(self) -> dict:
        done = [r for r in self.results if r.status == 0]
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        dof_steps = sum(r.n * r.steps for r in done)
        return {"requests": len(self.results), "completed": len(done),
                "rejected": sum(r.status == NN_EBUDGET for r in self.results),
                "cancelled": sum(r.status == CANCELLED for r in self.results),
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_latency_s": float(lat.mean()), "max_latency_s": float(lat.max()),
                "makespan_s": self.makespan, "dof_steps_per_s": dof_steps / self.makespan,
                "requests_per_s": len(done) / self.makespan, "ticks": self.ticks,
                "mean_resident_per_tick": self.mean_batch, "admission_waits": self.deferred,
                "peak_resident_bytes": self.peak_bytes, "hbm_budget_bytes": self.budget,
                "lane_ticks": list(self.lane_ticks)}


def batch_workspace_bytes(n: int, dim: int, precision: int) -> int:
    """Device bytes a batched call allocates for one member for the length of
    the call: the member's rows in the concatenated work vectors (gradient,
    two search products, mask, start value, load, diagonal, row lengths and
    six CG vectors; whole 64-row slices) and its entries in the concatenated
    block-diagonal matrix (int32 columns, int16 offsets and float64 values;
    float32 values too in mixed precision), counted at the longest row of
    a structured P1 pattern (7 in 2D, 15 in 3D) for every row of a slice."""
    rows = 64 * ((n + 63) // 64)
    nsell = (7 if dim == 2 else 15) * rows
    if precision == nnqp.NN_MIXED:
        return int(77.0 * rows + 18.0 * nsell)
    return int(101.0 * rows + 14.0 * nsell)


def estimate_bytes(problem, precision: int, solo: bool = False) -> int:
    """Device bytes of a request before assembly: free DOF from the Dirichlet
    mask, nonzeros per row of a structured P1 mesh (7 in 2D, 15 in 3D).
    solo: stepped by the single-problem solver, which adds the paired copies
    (int16 offsets and values) and its own work vectors; otherwise stepped by
    batched calls, whose per-call workspace is counted."""
    n = int((np.asarray(problem.dirichlet) == 0).sum())
    per_row = 7 if problem.dim == 2 else 15
    nnz = n * per_row
    b = 8.0 * n + 16.0 * nnz + 4.0 * n          # CSR, sliced-ELL (padding ignored)
    b += 24.0 * nnz + 16.0 * n                  # capacity and M/dt + K values, diagonals
    b += 89.0 * n                               # solver work vectors
    if precision == nnqp.NN_MIXED:
        b += 4.0 * nnz + 40.0 * n
    if solo:
        b += (1.1 * (10.0 if precision == nnqp.NN_FP64 else 6.0)) * nnz + 40.0 * n
    else:
        b += batch_workspace_bytes(n, problem.dim, precision)
    return int(b + 17.0 * n)                    # f, c, active set


# statuses that belong to one request's step (the request fails, the server
# goes on); any other status is a failure of the call itself
_REQUEST_STATUSES = (nnqp.NN_EMAXIT, nnqp.NN_ENONFINITE, nnqp.NN_ENOTSPD)


def _step_one(ctx, K, dt, F, c, act, opts) -> dict:
    """One backward-Euler step by the single-problem solver.  A status of the
    request's own problem (iteration cap, non-finite value, curvature) is
    reported like a batch member's; any other failure (memory, HIP, invalid
    argument) is raised, and the server stops."""
    try:
        _, _, st = ctx.step_transient(K, dt, F, c, opts=opts, active=act, allow_maxit=True)
        return st
    except nnqp.NnError as e:
        if e.status not in _REQUEST_STATUSES:
            raise
        return {"status": e.status, "kkt_rel": math.inf, "cg_its": 0}


class _Lane:
    """One batching lane: its own context and stream, queue and resident set."""

    def __init__(self, idx, ctx, stream, solo=False):
        self.idx = idx
        self.solo = solo
        self.ctx = ctx
        self.stream = stream
        self.pending = collections.deque()
        self.waiting = collections.deque()
        self.assembling = {}
        self.resident = []
        self.ticks = 0
        self.batch_sum = 0


class Server:
    """Continuous batching of transient requests.

    Requests are routed by size (free DOF estimated from the Dirichlet mask)
    to `len(lane_bounds) + 1` lanes.  Each lane runs its own tick loop on its
    own context and stream, so the small requests of one lane step while a
    large request of another lane is still inside its step (without lanes a
    tick lasts as long as its slowest member); all lanes share one HBM
    budget and admit first-in first-out within the lane.
    """

    def __init__(self, device: int = 0, hbm_budget: Optional[int] = None,
                 precision: int = nnqp.NN_FP64, dt: float = 1e-3, tol: float = 1e-8,
                 inner_rtol: float = 0.1, assemble_workers: int = 2, keep_states: bool = False,
                 bounds=(0.0, math.inf), lane_bounds=(30000, 300000), solo_lanes=2,
                 allocator=None, subspace: int = 0):
        import torch
        self.torch = torch
        self.device = device
        self.precision = precision
        self.dt = dt
        # bounds c_min <= c <= c_max of every step (Sec. 2.2.2, eq. Eq:non-negative)
        self.opts = nnqp.default_opts(tol=tol, inner_rtol=inner_rtol, precision=precision,
                                      lower=float(bounds[0]), upper=float(bounds[1]),
                                      subspace=int(subspace))
        free, total = torch.cuda.mem_get_info(device)
        self.budget = int(hbm_budget) if hbm_budget else int(0.75 * free)
        self.workers = assemble_workers
        self.keep_states = keep_states
        self.lane_bounds = tuple(sorted(lane_bounds))
        # the top `solo_lanes` lanes step each request with the single-problem
        # solver (nn_step_transient) instead of one batched call: for the
        # largest requests it is about twice as fast per step (paired layout,
        # Cauchy ladder), and those requests set the tail latency; the many
        # small requests of the bottom lane gain from sharing launches
        self.solo_from = len(self.lane_bounds) + 1 - max(0, int(solo_lanes))
        # device memory of every context the server makes (lanes and assembly
        # workers): None for hipMalloc, else as nnqp.Context's `allocator`
        self.allocator = allocator
        self._tls = threading.local()
        self._cancel = set()
        self._cancel_lock = threading.Lock()

    def cancel(self, rid: int) -> None:
        """Cancel request `rid` (any thread, also while `run` is serving)."""
        with self._cancel_lock:
            self._cancel.add(rid)

    def _cancelled(self, req: Request, now: float) -> bool:
        if now >= req.cancel_at:
            return True
        with self._cancel_lock:
            return req.rid in self._cancel

    # worker-thread assembly on the thread's own context and stream
    def _assemble(self, req: Request):
        torch = self.torch
        if getattr(self._tls, "ctx", None) is None:
            stream = torch.cuda.Stream(self.device)
            self._tls.ctx = nnqp.Context(self.device, stream=stream, allocator=self.allocator)
        wctx = self._tls.ctx
        with torch.cuda.stream(wctx.stream):
            K, F, _ = wctx.assemble(req.problem, with_mass=True)
        wctx.stream.synchronize()
        return K, F

    def _lane_of(self, req: Request) -> int:
        n = int((np.asarray(req.problem.dirichlet) == 0).sum())
        return sum(1 for b in self.lane_bounds if n >= b)

    def is_solo(self, req: Request) -> bool:
        """Whether the request is stepped by the single-problem solver."""
        return self._lane_of(req) >= self.solo_from

    def run(self, requests: List[Request]) -> Report:
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        results = {r.rid: Result(r.rid, 0, r.steps, r.arrival) for r in reqs}
        lanes = []
        for k in range(len(self.lane_bounds) + 1):
            stream = torch.cuda.Stream(self.device)
            lanes.append(_Lane(k, nnqp.Context(self.device, stream=stream,
                                               allocator=self.allocator),
                               stream, solo=k >= self.solo_from))
        for r in reqs:
            lanes[self._lane_of(r)].pending.append(r)
        shared = {"used": 0, "peak": 0}
        lock = threading.Lock()
        waited = set()
        pool = cf.ThreadPoolExecutor(max_workers=self.workers)
        t0 = time.perf_counter()
        errors = []
        abort = threading.Event()   # a failed lane stops the others (they may wait on its memory)

        def lane_loop(L: _Lane):
            try:
                with torch.cuda.stream(L.stream):
                    self._lane_loop(L, results, shared, lock, waited, pool, t0, abort)
            except BaseException as e:   # surfaced after the lanes join
                errors.append(e)
                abort.set()

        threads = [threading.Thread(target=lane_loop, args=(L,)) for L in lanes]
        try:
            for t in threads:
                t.start()
            for t in threads:
                t.join()
        finally:
            pool.shutdown(wait=True)
        if errors:
            raise errors[0]
        torch.cuda.synchronize()
        makespan = time.perf_counter() - t0
        ticks = sum(L.ticks for L in lanes)
        batch_sum = sum(L.batch_sum for L in lanes)
        return Report([results[r.rid] for r in reqs], makespan, ticks,
                      batch_sum / max(ticks, 1), len(waited), shared["peak"], self.budget,
                      [L.ticks for L in lanes], shared["used"])

    def _lane_loop(self, L: _Lane, results, shared, lock, waited, pool, t0, abort):
        torch = self.torch

        def drop(req):
            res = results[req.rid]
            res.status = CANCELLED
            res.finished = time.perf_counter() - t0

        while (L.pending or L.waiting or L.assembling or L.resident) and not abort.is_set():
            now = time.perf_counter() - t0
            while L.pending and L.pending[0].arrival <= now:
                L.waiting.append(L.pending.popleft())
            # cancellations: queued requests leave, resident ones free their memory
            for q in (L.pending, L.waiting):
                for req in [r for r in q if self._cancelled(r, now)]:
                    q.remove(req)
                    drop(req)
            gone = [s for s in L.resident if self._cancelled(s["req"], now)]
            for s in gone:
                drop(s["req"])
                s["K"].free()
                with lock:
                    shared["used"] -= s["bytes"]
            if gone:
                L.resident = [s for s in L.resident if not any(s is g for g in gone)]
            # admission: first in, first out within the lane, while the estimate fits
            while L.waiting:
                req = L.waiting[0]
                est = estimate_bytes(req.problem, self.precision, solo=L.solo)
                if est > self.budget:
                    L.waiting.popleft()
                    res = results[req.rid]
                    res.status = NN_EBUDGET
                    res.finished = time.perf_counter() - t0
                    continue
                with lock:
                    if shared["used"] + est > self.budget:
                        waited.add(req.rid)
                        break
                    shared["used"] += est
                    shared["peak"] = max(shared["peak"], shared["used"])
                L.waiting.popleft()
                results[req.rid].admitted = time.perf_counter() - t0
                L.assembling[pool.submit(self._assemble, req)] = (req, est)
            # assembled requests become resident
            for fut in [f for f in L.assembling if f.done()]:
                req, est = L.assembling.pop(fut)
                K, F = fut.result()
                if self._cancelled(req, time.perf_counter() - t0):
                    drop(req)
                    K.free()
                    with lock:
                        shared["used"] -= est
                    continue
                nb = K.bytes(self.precision) + 17 * K.n
                if L.solo:   # the paired copies and work vectors its steps will add
                    nb = max(nb, est)
                else:        # the workspace of the batched calls that step it
                    nb += batch_workspace_bytes(K.n, req.problem.dim, self.precision)
                with lock:
                    shared["used"] += nb - est
                    shared["peak"] = max(shared["peak"], shared["used"])
                c = torch.zeros(max(K.n, 1), dtype=torch.float64, device=L.ctx.device)
                act = torch.empty(max(K.n, 1), dtype=torch.uint8, device=L.ctx.device)
                results[req.rid].n = K.n
                L.resident.append({"req": req, "K": K, "F": F, "c": c, "act": act, "bytes": nb,
                                   "done": 0})
            if L.resident:
                tnow = time.perf_counter() - t0
                for s in L.resident:
                    r = results[s["req"].rid]
                    if math.isnan(r.started):
                        r.started = tnow
                if L.solo:
                    stats = [_step_one(L.ctx, s["K"], self.dt, s["F"], s["c"], s["act"], self.opts)
                             for s in L.resident]
                else:
                    _, _, stats, rc = L.ctx.step_transient_batch(
                        [s["K"] for s in L.resident], self.dt, [s["F"] for s in L.resident],
                        [s["c"] for s in L.resident], opts=self.opts,
                        actives=[s["act"] for s in L.resident], allow_fail=True)
                    # members failing on their own problems are reported per
                    # request; a failure of the call itself stepped no member
                    if rc not in (nnqp.NN_OK,) + _REQUEST_STATUSES:
                        raise nnqp.NnError(rc, "nn_step_transient_batch: "
                                           + L.ctx.last_error())
                L.ticks += 1
                L.batch_sum += len(L.resident)
                tend = time.perf_counter() - t0
                keep = []
                for s, stt in zip(L.resident, stats):
                    r = results[s["req"].rid]
                    r.step_stats.append(stt)
                    s["done"] += 1
                    if stt["status"] != 0 and r.status == 0:
                        r.status = stt["status"]
                    if s["done"] >= s["req"].steps or stt["status"] not in (0,):
                        r.finished = tend
                        if self.keep_states:
                            r.c = s["c"][:s["K"].n].clone()
                        s["K"].free()
                        with lock:
                            shared["used"] -= s["bytes"]
                    else:
                        keep.append(s)
                L.resident = keep
            elif L.assembling:
                cf.wait(list(L.assembling), timeout=0.05, return_when=cf.FIRST_COMPLETED)
            elif L.pending and not L.waiting:
                time.sleep(max(0.0, min(0.05, L.pending[0].arrival - (time.perf_counter() - t0))))
            elif L.waiting:
                time.sleep(0.002)   # waiting for memory that another lane will free


def solve_alone(req: Request, precision: int = nnqp.NN_FP64, dt: float = 1e-3, tol: float = 1e-8,
                inner_rtol: float = 0.1, ctx=None, bounds=(0.0, math.inf), single: bool = False):
    """The same request run by itself (a batch of one per step, or the
    single-problem solver with `single`): final c and per-step stats."""
    import torch
    ctx = ctx or nnqp.Context(0)
    opts = nnqp.default_opts(tol=tol, inner_rtol=inner_rtol, precision=precision,
                             lower=float(bounds[0]), upper=float(bounds[1]))
    K, F, _ = ctx.assemble(req.problem, with_mass=True)
    c = torch.zeros(max(K.n, 1), dtype=torch.float64, device=ctx.device)
    stats = []
    for _ in range(req.steps):
        if single:
            _, _, st = ctx.step_transient(K, dt, F, c, opts=opts)
            stats.append(st)
        else:
            _, _, st, _ = ctx.step_transient_batch([K], dt, [F], [c], opts=opts)
            stats.append(st[0])
    out = c[:K.n].clone()
    K.free()
    return out, stats
