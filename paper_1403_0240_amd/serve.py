"""Continuous-batching segmentation server on one GPU.

Requests (one image each, with initial labels and method parameters) are
admitted into the free slots of a batch as soon as a slot and HBM room are
free, run to convergence together with whatever else is resident, and retire
on their own: the slot is reused at once, and the label field goes back to
the host (one asynchronous copy into page-locked staging memory, landed in the
request's array by a helper thread) while the pools run on; the request's
memory is released when its labels have landed.  Requests with different kernel geometry
(ndim, E, eps) live in separate batches, one HIP stream each, so their work
overlaps on the device.

Every iteration runs in the library's batched kernels; this module only
decides which context sits in which slot and when.  A request's result does
not depend on what else is resident: a batch slot follows its context's own
stand-alone trajectory bit for bit, and a tick never takes a job past its
iteration cap, so each job stops exactly where `run(ctx, max_iters, tol, mode)`
on its own would.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import gc
import time

import numpy as np
import torch

from . import sobrc as S


@dataclasses.dataclass
class Request:
    rid: int
    work: object                 # workloads.Workload
    arrival: float               # seconds since the server's clock started
    admitted: float = -1.0
    done: float = -1.0
    iterations: int = 0
    labels: np.ndarray | None = None  # uint16, the image's shape
    switch_iter: int = -1
    error: str | None = None     # set when the request failed (its labels are those it stopped at)
    footprint: int = 0
    capacity: int | None = None  # particle capacity (None: default_capacity of the image)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Job:
    def __init__(self, req: Request, ctx, img, cap):
        self.req, self.ctx, self.img, self.cap = req, ctx, img, cap


class _Pool:
    """One batch (one kernel geometry) with its slots, stream and the
    committed iterations of each resident job."""

    def __init__(self, n_slots: int):
        self.batch = S.Batch(n_slots)
        self.stream = torch.cuda.Stream()
        self.jobs: list[_Job | None] = [None] * n_slots
        self.iters = np.zeros(n_slots, np.int64)
        self.ready: list[_Job] = []  # initialised, waiting for the pool to be idle

    def free_slots(self) -> int:
        return sum(j is None for j in self.jobs)

    def live(self):
        return [(k, j) for k, j in enumerate(self.jobs) if j is not None]


def footprint(w, capacity: int, tile: int = 0) -> int:
    """Device bytes a request holds while resident: its context workspace
    plus the image."""
    return S.workspace_size(S.workload_params(w, capacity, tile)) + w.image.nbytes


def default_capacity(w) -> int:
    return max(4096, w.labels.size // 4)


class Server:
    """Continuous batching over per-geometry pools.

    hbm_budget: device bytes the resident requests may hold together;
    slots: slots per pool; tol: flip tolerance (stop when flips < tol * N);
    max_iters: per-request iteration cap; tick: iterations enqueued per pool
    between host looks; tiles: cell shape per image dimension (sobrc.TILE_*;
    results do not depend on it)."""

    def __init__(self, hbm_budget: int = 8 << 30, slots: int = 64, tol: float = 1e-3,
                 max_iters: int = 500, tick: int = 4, mode: int = S.MODE_AUTO, tiles=None):
        self.tiles = dict(tiles or {})
        self.budget, self.slots, self.tol = hbm_budget, slots, tol
        self.max_iters, self.tick, self.mode = max_iters, tick, mode
        self.pools: dict[tuple, _Pool] = {}
        self.waiting: collections.deque[Request] = collections.deque()
        self.finished: list[Request] = []
        self.used = 0
        self.t0 = time.perf_counter()
        self.admit_stream = torch.cuda.Stream()
        # retired jobs whose labels are on their way to the host:
        # (request, job, staging buffer, future of (labels, landing time))
        self.landing: list[tuple] = []
        self.staging: dict[int, list] = collections.defaultdict(list)  # power-of-two sizes
        self.lander = concurrent.futures.ThreadPoolExecutor(max_workers=2)

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        if getattr(req.work, "topo", 0) or getattr(req.work, "psf_sigma", 0.0) > 0.0:
            # such contexts are not batched: run them with sobrc.run on their own
            raise ValueError(f"request {req.rid}: topological control and the deconvolving model "
                             f"are not served in batches")
        if req.capacity is None:
            req.capacity = default_capacity(req.work)
        req.footprint = footprint(req.work, req.capacity, self._tile(req.work))
        if req.footprint > self.budget:
            raise ValueError(f"request {req.rid} needs {req.footprint} bytes > budget {self.budget}")
        self.waiting.append(req)

    def _tile(self, w) -> int:
        return self.tiles.get(w.ndim, getattr(w, "tile", 0))

    # ------------------------------------------------------------ admission
    def _pool_of(self, w) -> _Pool:
        key = (w.ndim, float(w.E), float(w.eps), self._tile(w))
        if key not in self.pools:
            self.pools[key] = _Pool(self.slots)
        return self.pools[key]

    def _prepare(self):
        """FIFO: initialise the head request's context while its pool has a
        slot not yet promised and the budget has room (a head that does not
        fit waits; nothing overtakes it).  Runs on the admission stream, so
        it overlaps the pools' work in flight."""
        while self.waiting:
            req = self.waiting[0]
            pool = self._pool_of(req.work)
            if pool.free_slots() - len(pool.ready) <= 0 or self.used + req.footprint > self.budget:
                return
            self.waiting.popleft()
            w = req.work
            cap = req.capacity
            with torch.cuda.stream(self.admit_stream):
                ctx, img, lab = S.from_workload(w, max_particles=cap, tile=self._tile(w))
                S.init_labels(ctx, img, lab, stream=self.admit_stream)
                del lab
            pool.ready.append(_Job(req, ctx, img, cap))
            self.used += req.footprint

    def _place(self):
        """Move initialised contexts into free slots; called only while no
        pool has work in flight (slot tables are read by running kernels)."""
        for pool in self.pools.values():
            while pool.ready:
                k = next(i for i, j in enumerate(pool.jobs) if j is None)
                job = pool.ready.pop(0)
                pool.batch.set(k, job.ctx, stream=pool.stream)
                pool.jobs[k] = job
                pool.iters[k] = 0
                job.req.admitted = self.now()

    # ---------------------------------------------------------------- ticks
    def _land(self, ev, stage):
        """Helper thread: wait for the label copy, then move it out of the
        staging buffer (both release the GIL)."""
        ev.synchronize()
        return stage.numpy().copy(), self.now()

    def _retire(self, pool: _Pool, k: int, error: str | None = None):
        job = pool.jobs[k]
        req = job.req
        pool.batch.set(k, None, stream=pool.stream)
        req.switch_iter = S.gradient_switch(job.ctx, stream=pool.stream)
        req.iterations = int(pool.iters[k])
        req.error = error
        pool.jobs[k] = None
        shape = tuple(job.ctx.shape)
        n = int(np.prod(shape))
        free = self.staging[1 << (n - 1).bit_length()]
        buf = free.pop() if free else torch.empty(1 << (n - 1).bit_length(), dtype=torch.uint16,
                                                  pin_memory=True)
        stage = buf[:n].view(shape)
        S.get_labels_u16(job.ctx, stage, stream=pool.stream)
        ev = torch.cuda.Event()
        ev.record(pool.stream)
        self.landing.append((req, job, buf, self.lander.submit(self._land, ev, stage)))

    def _landed(self, wait: bool = False):
        """Finish the retired jobs whose labels have reached the host (with
        wait, all of them): release their contexts, memory and staging."""
        keep = []
        for item in self.landing:
            req, job, buf, fut = item
            if not (wait or fut.done()):
                keep.append(item)
                continue
            req.labels, req.done = fut.result()
            self.staging[buf.numel()].append(buf)
            self.used -= req.footprint
            job.ctx.close()
            self.finished.append(req)
        self.landing = keep

    def step(self) -> bool:
        """One tick: enqueue iterations on every busy pool (one stream each),
        admit waiting requests meanwhile, then collect and retire stopped
        jobs.  Returns whether anything is resident afterwards."""
        busy = []
        for pool in self.pools.values():
            live = pool.live()
            if not live:
                continue
            # never past a resident job's cap, so every stop is exact
            left = min(self.max_iters - int(pool.iters[k]) for k, _ in live)
            pool.batch.launch(max(1, min(self.tick, left)), self.tol, self.mode, stream=pool.stream)
            busy.append(pool)
        self._prepare()
        for pool in busy:
            # a slot's own failure (e.g. its particle set outgrew its
            # capacity) ends that request only
            it, state = pool.batch.collect(stream=pool.stream, slot_errors=True)
            for k, job in pool.live():
                pool.iters[k] = it[k]
                if state[k] < 0:
                    self._retire(pool, k, error=f"sobrc error {int(state[k])} after {int(it[k])} iterations")
                elif state[k] or it[k] >= self.max_iters:
                    self._retire(pool, k)
        # every pool is idle: place what was prepared, then fill freed slots
        self._landed()
        self._place()
        self._prepare()
        self._place()
        live = any(p.live() for p in self.pools.values())
        if not live and self.landing:
            # nothing runs: the next admission waits for memory that landing frees
            self._landed(wait=True)
            self._prepare()
            self._place()
            live = any(p.live() for p in self.pools.values())
        return live

    def serve(self, stream_of_requests, realtime: bool = True):
        """Run a list of (arrival seconds, Workload) or (arrival seconds,
        Workload, particle capacity) to completion.  With realtime, each
        request is submitted when the clock reaches its arrival time;
        otherwise all arrive at time 0 (saturation).

        While it runs, the objects the process already holds are frozen out
        of the garbage collector: a full collection over them (torch's
        modules and the like) pauses the loop for tens of milliseconds,
        which would land on whichever request is retiring."""
        pending = collections.deque(
            Request(k, item[1], float(item[0]) if realtime else 0.0,
                    capacity=item[2] if len(item) > 2 else None)
            for k, item in enumerate(stream_of_requests))
        gc.freeze()
        try:
            self.t0 = time.perf_counter()
            while pending or self.waiting or self.landing or any(p.live() for p in self.pools.values()):
                while pending and pending[0].arrival <= self.now():
                    self.submit(pending.popleft())
                if not self.step() and not self.waiting and pending:
                    time.sleep(max(0.0, min(pending[0].arrival - self.now(), 0.05)))
            self._landed(wait=True)
        finally:
            gc.unfreeze()
        return self.finished

    def close(self):
        self._landed(wait=True)
        self.lander.shutdown()
        self.staging.clear()
        for pool in self.pools.values():
            for k, job in pool.live():
                pool.batch.set(k, None, stream=pool.stream)
                job.ctx.close()
            for job in pool.ready:
                job.ctx.close()
            pool.batch.close()
        self.pools.clear()


def latency_stats(reqs) -> dict:
    lat = np.array([r.latency for r in reqs])
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "images_per_s": len(reqs) / span if span > 0 else float("inf"),
            "span_s": span}
