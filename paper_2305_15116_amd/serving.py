"""Serving loop: many solve requests on one GPU, with continuous batching.

A request is a Poisson problem on its own macro mesh (dimension, cells,
level, seeded right-hand side, tolerance).  The server admits requests by
their HBM footprint, prepares them (mesh set-up on the host, vectors on the
device) on a preparation thread, and solves them on a worker thread:

* batched: every admitted request joins one batch (batch_* in the C ABI);
  each step runs one outer iteration of the mixed-precision solver (CG
  preconditioned by an FP32 V-cycle, by default) for all members with shared
  launches, and finished members leave while new ones join at the next step
  (continuous batching);
* plain: one request at a time, in arrival order, with the all-FP64
  vcycle_solve (CG preconditioned by an FP64 V-cycle, by default).

Every computation runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import _binding as B


def storage_dofs(dim: int, n_cells: int, level: int) -> int:
    """Storage DoFs of a mesh of n_cells macros at `level` (each macro's closed index space)."""
    n = 1 << level
    per = (n + 1) * (n + 2) // 2 if dim == 2 else (n + 1) * (n + 2) * (n + 3) // 6
    return n_cells * per


def footprint_bytes(dim: int, n_cells: int, level: int, mode: int) -> int:
    """Device bytes one request holds while it is served: b and x (FP64), the
    solver workspace of `mode` (mesh_workspace_bytes' layout) and the mesh
    metadata, with a small margin."""
    s = [storage_dofs(dim, n_cells, l) for l in range(level + 1)]
    vec = 16 * s[level]
    ws = 24 * s[level] + 24 * sum(s[:level]) if mode % 2 == 0 else 8 * s[level] + 12 * sum(s)
    if mode >= 2:
        ws += (16 if mode == 2 else 24) * s[level]
    n = 1 << level
    rows = n_cells * ((n + 1) if dim == 2 else (n + 1) * (n + 2) // 2)
    part = 16 * (s[level] // 64 + rows + 64)
    meta = 24 * s[level] // 64 + 16 * rows + 4096 * n_cells * (level + 1)
    return int(1.02 * (vec + ws + part + meta)) + (1 << 20)


@dataclass
class Request:
    rid: int
    dim: int
    coords: np.ndarray
    cells: np.ndarray
    level: int
    rhs_seed: int
    tol: float
    t_arrival: float
    footprint: int
    future: cf.Future = field(default_factory=cf.Future)
    t_admit: float = 0.0
    mesh: object = None
    b: object = None
    x: object = None
    ws: object = None


class Server:
    """Solve server for one GPU.

    budget_bytes: device memory the server may hold for requests; a request
    whose footprint alone exceeds it is rejected (its future raises MFError
    with MF_ENOMEM).  batched: continuous batching with the mixed solver
    (default), else plain one-at-a-time FIFO with the all-FP64 solver.
    Requests are admitted in arrival order and prepared (mesh set-up, device
    vectors) by `preparers` threads, so both servers solve them in the order
    their preparation ends.
    submit() returns a Future of (x, info): x the solution (torch, storage
    layout), info a dict with status, iters, rel_res and the arrival, admission
    and completion times (time.perf_counter()).
    """

    def __init__(self, budget_bytes: int, batched: bool = True, max_batch: int = 64, max_iter: int = 100,
                 keep_solutions: bool = True, mode: int | None = None, lanes: int | None = None,
                 split_dofs: int = 4_000_000, preparers: int = 3):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.batched = batched
        # solver mode (vcycle_solve): mixed-precision CG for the batched server,
        # all-FP64 CG for the plain one
        self.mode = (3 if batched else 2) if mode is None else mode
        self.max_batch = max_batch
        self.max_iter = max_iter
        self.keep = keep_solutions
        self.used = 0
        self.rejected = 0   # footprint above the budget
        self.failed = 0     # could not be prepared (device memory)
        self.completed = 0
        self.busy_s = 0.0
        # batched: requests below split_dofs storage DoFs and the larger ones
        # step in separate batches on separate streams (lanes), so that a
        # small request's iterations are not gated by a large member's
        self.lanes = (2 if batched else 1) if lanes is None else max(1, lanes)
        self.split_dofs = split_dofs
        self._pending: collections.deque[Request] = collections.deque()
        self._ready = [collections.deque() for _ in range(self.lanes)]
        self.lane_busy_s = [0.0] * self.lanes
        self._inflight = 0  # prepared or being solved
        self._cv = threading.Condition()
        self._stop = False
        self._error: BaseException | None = None
        self._dev = torch.cuda.current_device()
        self._next = 0
        self._live: dict[int, Request] = {}  # submitted, not finished
        # mesh set-up on the host takes as long as a solve or longer (3D level 8:
        # about 35 ms against a 20 ms mixed CG solve), so several threads
        # prepare requests; ctypes releases the GIL during the library calls
        self._prep = [threading.Thread(target=self._prep_loop, name=f"mf-prep{k}", daemon=True)
                      for k in range(max(1, preparers))]
        self._work = [threading.Thread(target=self._work_loop, args=(k,), name=f"mf-work{k}", daemon=True)
                      for k in range(self.lanes)]
        for t in self._prep:
            t.start()
        for t in self._work:
            t.start()

    # ------------------------------------------------------------ client side
    def submit(self, dim, coords, cells, level, rhs_seed, tol=1e-8, t_arrival=None) -> cf.Future:
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        fp = footprint_bytes(dim, cells.shape[0], level, self.mode)
        with self._cv:
            rid = self._next
            self._next += 1
        r = Request(rid, dim, np.ascontiguousarray(coords, dtype=np.float64), cells, level, rhs_seed, tol,
                    time.perf_counter() if t_arrival is None else t_arrival, fp)
        if fp > self.budget:
            with self._cv:
                self.rejected += 1
            r.future.set_exception(B.MFError(B.MF_ENOMEM, f"request needs {fp} B of device memory, "
                                                          f"budget is {self.budget} B"))
            return r.future
        with self._cv:
            if self._error is not None:
                r.future.set_exception(RuntimeError(f"server failed: {self._error!r}"))
                return r.future
            self._live[r.rid] = r
            self._pending.append(r)
            self._cv.notify_all()
        return r.future

    def close(self, wait: bool = True):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        if wait:
            for t in self._prep:
                t.join()
            for t in self._work:
                t.join()
        if self._error is not None:
            raise self._error

    # ------------------------------------------------------------ preparation
    def _prep_loop(self):
        torch = self.torch
        torch.cuda.set_device(self._dev)
        stream = torch.cuda.Stream()
        try:
            while True:
                with self._cv:
                    while not self._stop and not (self._pending and self._admissible(self._pending[0])):
                        self._cv.wait(0.05)
                    if self._stop and not self._pending:
                        return
                    if not self._pending or not self._admissible(self._pending[0]):
                        continue
                    r = self._pending.popleft()
                    self.used += r.footprint
                    self._inflight += 1
                r.t_admit = time.perf_counter()
                err = None
                for attempt in range(2):
                    try:
                        s = self._prepare(r, stream)
                        err = None
                        break
                    except (B.MFError, torch.OutOfMemoryError, RuntimeError) as e:
                        # device memory beyond the accounting (allocator caching,
                        # fragmentation): release the cache and retry once
                        err = e
                        r.b = r.x = r.ws = None
                        if r.mesh is not None:
                            r.mesh.close()
                            r.mesh = None
                        torch.cuda.empty_cache()
                if err is not None:
                    self._drop(r, err)
                    continue
                lane = 0 if (self.lanes == 1 or s < self.split_dofs) else self.lanes - 1
                with self._cv:
                    self._ready[lane].append(r)
                    self._cv.notify_all()
        except BaseException as e:  # surfaced by close()
            self._fail(e)

    def _prepare(self, r: Request, stream) -> int:
        """Mesh set-up on the host, vectors on the device; returns storage DoFs."""
        torch = self.torch
        r.mesh = B.create_macro_mesh(r.coords, r.cells, r.level)
        s, _ = B.mesh_num_dofs(r.mesh, r.level)
        with torch.cuda.stream(stream):
            r.b = torch.empty(s, dtype=torch.float64, device="cuda")
            r.x = torch.zeros(s, dtype=torch.float64, device="cuda")
            r.ws = torch.empty(B.mesh_workspace_bytes(r.mesh, r.level, self.mode), dtype=torch.uint8,
                               device="cuda")
            B.mesh_fill_random(r.mesh, r.level, r.rhs_seed, r.b, stream)
            B.mesh_set_dirichlet(r.mesh, r.level, None, r.b, stream)
        stream.synchronize()
        return s

    def _drop(self, r: Request, e: BaseException):
        """A request that could not be prepared fails alone (counted in `failed`)."""
        with self._cv:
            self.used -= r.footprint
            self._inflight -= 1
            self.failed += 1
            self._live.pop(r.rid, None)
            self._cv.notify_all()
        if isinstance(e, B.MFError):
            r.future.set_exception(e)
        else:
            r.future.set_exception(B.MFError(B.MF_ENOMEM, f"preparing the request failed: {e!r}"))

    def _fail(self, e: BaseException):
        """A thread died: every unfinished request fails with the error."""
        import sys
        print(f"serving: thread failed: {e!r}", file=sys.stderr, flush=True)
        with self._cv:
            if self._error is None:
                self._error = e
            self._stop = True
            live = list(self._live.values())
            self._live.clear()
            self._pending.clear()
            for q in self._ready:
                q.clear()
            self._cv.notify_all()
        for r in live:
            if not r.future.done():
                r.future.set_exception(RuntimeError(f"server failed: {e!r}"))

    def _admissible(self, r: Request) -> bool:
        return self.used + r.footprint <= self.budget and self._inflight < self.max_batch

    # ------------------------------------------------------------ solving
    def _finish(self, r: Request, status: int, iters: int, rel: float):
        t = time.perf_counter()
        info = {"status": status, "iters": iters, "rel_res": rel, "t_arrival": r.t_arrival, "t_admit": r.t_admit,
                "t_done": t, "latency": t - r.t_arrival, "rid": r.rid}
        x = r.x if self.keep else None
        r.b = r.ws = r.x = None
        if r.mesh is not None:
            r.mesh.close()
            r.mesh = None
        with self._cv:
            self.used -= r.footprint
            self._inflight -= 1
            self.completed += 1
            self._live.pop(r.rid, None)
            self._cv.notify_all()
        r.future.set_result((x, info))

    def _work_loop(self, lane: int):
        torch = self.torch
        torch.cuda.set_device(self._dev)
        stream = torch.cuda.Stream()
        try:
            if self.batched:
                self._batched_loop(stream, lane)
            else:
                self._plain_loop(stream, lane)
        except BaseException as e:
            self._fail(e)

    def _done_all(self) -> bool:
        return (self._stop and not self._pending and self._inflight == 0) or self._error is not None

    def _take_ready(self, lane: int, block: bool):
        with self._cv:
            while block and not self._ready[lane] and not self._done_all():
                self._cv.wait(0.05)
            out = list(self._ready[lane])
            self._ready[lane].clear()
            return out

    def _plain_loop(self, stream, lane: int):
        while True:
            rs = self._take_ready(lane, block=True)
            if not rs:
                with self._cv:
                    if self._done_all():
                        return
                continue
            for r in rs:
                t0 = time.perf_counter()
                rc, it, rel, _ = B.vcycle_solve(r.mesh, r.level, r.b, r.x, r.ws, mode=self.mode, rtol=r.tol,
                                                max_iter=self.max_iter, stream=stream)
                dt = time.perf_counter() - t0
                self.busy_s += dt
                self.lane_busy_s[lane] += dt
                self._finish(r, rc, it, rel)

    def _batched_loop(self, stream, lane: int):
        batch = B.batch_create(self.max_batch, mode=self.mode, max_iter=self.max_iter)
        members: dict[int, Request] = {}
        try:
            while True:
                rs = self._take_ready(lane, block=not members)
                for r in rs:
                    B.batch_add(batch, r.mesh, r.level, r.b, r.x, r.ws, r.tol, r.rid)
                    members[r.rid] = r
                if not members:
                    with self._cv:
                        if self._done_all():
                            return
                    continue
                t0 = time.perf_counter()
                done = B.batch_step(batch, stream)
                dt = time.perf_counter() - t0
                self.busy_s += dt
                self.lane_busy_s[lane] += dt
                for tag, st, it, rel, _ in done:
                    self._finish(members.pop(tag), st, it, rel)
        finally:
            batch.close()


def latency_stats(infos, t0: float, t1: float) -> dict:
    """p50 / p99 / mean latency (ms) and throughput of completed requests."""
    lat = np.array([i["latency"] for i in infos]) * 1e3
    if lat.size == 0:
        return {"completed": 0}
    return {"completed": int(lat.size), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "solves_per_s": lat.size / (t1 - t0)}
