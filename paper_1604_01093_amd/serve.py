"""Serving loop for pose-alignment solves (host-side scheduling around libbf).

Requests are whole solves of the energy of paper Sec. 4.3-4.4: intra-chunk
solves (a handful of frames, Sec. 4.1) and global keyframe solves (tens to
hundreds of keyframes, Sec. 4.2).  Their frames, correspondences and poses
stay in device memory from submission to completion.  Two lanes run on the GPU
at the same time, each with its own libbf context and HIP stream:

* the batch lane takes every waiting small request (at most `small_max_frames`
  frames, same intrinsics) whenever it is free and solves them together in one
  bf_gauss_newton_batch call -- continuous batching: requests that arrive while
  a batch runs join the next one;
* the large lane solves the other requests one at a time with bf_gauss_newton.

Admission is by device-memory footprint: a request (or a batch) starts only
when the estimated workspace of everything in flight stays within
`max_inflight_bytes`; otherwise its lane waits until running work finishes.

A request can be cancelled (`Server.cancel`): while it waits it leaves its queue
at once; once admitted into a running batch or solve the GPU call is not
interrupted (it is one launch sequence over all members), the other members
complete as usual and the cancelled one completes with a `Cancelled` error and
no result.

Warm start (paper Sec. 4.4: each solve starts from the result of the last one):
a request that names a problem (`key`) leaves its result poses resident under
that key; a later request with the same key and `warm_start=True` starts from
them instead of its own initial poses, for as many leading frames as the stored
result has (a grown problem, one with new frames appended, keeps its own initial
poses for the new frames).  The stored result is the one of the last request of
that key completed when the warm request starts running; if none has completed,
the request starts from its own initial poses (`Request.warm_frames` says how many
frames were warm-started).

Every computation of a solve runs in libbf's kernels; this module only
queues, groups, concatenates device tensors and records times.
"""
from __future__ import annotations

import collections
import threading
import time

import torch

from . import bf


def footprint_bytes(num_frames, width, height, num_corrs, num_pairs=None, directions=1):
    """Estimated device bytes of one solve: the inputs (depth and intensity, the
    correspondences' frame indices and points) and the context's workspace --
    prepared frames, pair search flags, pair records (one per pair job: `directions`
    per pair, up to four partial records each when the dense launch splits jobs into
    tiles), edge blocks, correspondence indexing and sorting -- with the workspace
    taken a quarter larger (its buffers grow by a quarter more than asked) plus 1 MiB
    for the small fixed buffers.  The pair count is bounded by F (F - 1) / 2 when it
    is not known."""
    F, HW = int(num_frames), int(width) * int(height)
    P = int(num_pairs) if num_pairs is not None else F * (F - 1) // 2
    M = int(num_corrs)
    inputs = F * HW * 8 + M * 32
    frames = F * HW * 20
    pair_search = F * F + 24 * (F + 1)
    records = P * (4 * 256 * int(directions) + 16)
    edges = (P + F) * (1024 + 144 + 64)
    corr = M * 96
    work = frames + pair_search + records + edges + corr + 64 * F * 16
    return inputs + work + work // 4 + (1 << 20)


class Cancelled(RuntimeError):
    """The request was cancelled before its result was delivered."""


class Request:
    """One solve: a DeviceProblem, its initial poses (device) and parameters."""

    _next_id = 0

    def __init__(self, problem: "bf.DeviceProblem", init_poses: torch.Tensor, params, tag=None, key=None,
                 warm_start=False):
        self.id = Request._next_id
        Request._next_id += 1
        self.problem = problem
        self.init_poses = init_poses
        self.params = params
        self.tag = tag
        self.key = key
        self.warm_start = bool(warm_start) and key is not None
        self.warm_frames = 0
        self.num_frames = problem.num_frames
        intr = problem.intr
        self.intr_key = (intr.fx, intr.fy, intr.cx, intr.cy, intr.width, intr.height)
        self.footprint = footprint_bytes(self.num_frames, intr.width, intr.height, problem.num_corrs,
                                         directions=2 if getattr(params, "bidirectional", 0) else 1)
        self.t_arrival = None
        self.t_start = None
        self.t_done = None
        self.poses = None
        self.energy = None
        self.error = None
        self.batch_size = 0
        self.lane = None
        self.ready_event = None
        self.cancelled = False
        self.done = threading.Event()

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


class Server:
    """Two GPU lanes with continuous batching of small requests and admission by
    device-memory footprint."""

    def __init__(self, max_inflight_bytes=64 << 30, small_max_frames=65, max_batch=512):
        self.max_inflight = int(max_inflight_bytes)
        self.small_max_frames = small_max_frames
        self.max_batch = max_batch
        self.cv = threading.Condition()
        self.inflight = 0
        self.small = collections.deque()
        self.large = collections.deque()
        self.stop = False
        self.lanes = []
        self.batches = []  # (number of requests, seconds) of every batch-lane call
        self.resident = {}  # key -> result poses (device) of the last completed request of that key
        for name, fn in (("batch", self._batch_lane), ("large", self._large_lane)):
            stream = torch.cuda.Stream()
            ctx = bf.Context(stream=stream)
            th = threading.Thread(target=fn, args=(ctx, stream), name=f"bf-{name}", daemon=True)
            self.lanes.append((th, ctx, stream))
        for th, _, _ in self.lanes:
            th.start()

    # ---------------------------------------------------------------- submission
    def submit(self, req: Request, t_arrival=None):
        req.t_arrival = time.perf_counter() if t_arrival is None else t_arrival
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())  # the request's tensors are ready after this point
        req.ready_event = ev
        if req.footprint > self.max_inflight:
            req.error = bf.BFError(bf.BF_ERR_OUT_OF_MEMORY, "request exceeds the device-memory budget")
            req.t_done = time.perf_counter()
            req.done.set()
            return req
        with self.cv:
            (self.small if req.num_frames <= self.small_max_frames else self.large).append(req)
            self.cv.notify_all()
        return req

    def cancel(self, req: Request):
        """Cancel a submitted request.  Returns "queued" if it was removed before
        running, "running" if it was admitted already (it then completes with a
        Cancelled error when its GPU call returns, its result discarded), or "done"
        if it had completed."""
        with self.cv:
            if req.done.is_set():
                return "done"
            req.cancelled = True
            for q in (self.small, self.large):
                if req in q:
                    q.remove(req)
                    req.error = Cancelled(f"request {req.id} cancelled while queued")
                    req.t_done = time.perf_counter()
                    req.done.set()
                    self.cv.notify_all()
                    return "queued"
            return "running"

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for th, ctx, _ in self.lanes:
            th.join()
            ctx.close()

    # ---------------------------------------------------------------- lanes
    def _admit(self, queue, take_many):
        """Under the lock: pop the requests to run next from `queue` (FIFO), within
        the memory budget; empty list when nothing can start yet."""
        if not queue:
            return []
        first = queue[0]
        if self.inflight + first.footprint > self.max_inflight:
            return []
        out = [queue.popleft()]
        total = first.footprint
        if take_many:
            keep = collections.deque()
            while queue and len(out) < self.max_batch:
                r = queue.popleft()
                if (r.intr_key == first.intr_key and r.params is first.params
                        and self.inflight + total + r.footprint <= self.max_inflight):
                    out.append(r)
                    total += r.footprint
                else:
                    keep.append(r)
            keep.extend(queue)
            queue.clear()
            queue.extend(keep)
        self.inflight += total
        return out

    def _release(self, reqs):
        with self.cv:
            self.inflight -= sum(r.footprint for r in reqs)
            self.cv.notify_all()

    def _next(self, queue, take_many):
        with self.cv:
            while True:
                got = self._admit(queue, take_many)
                if got or self.stop:
                    return got
                self.cv.wait(0.05)

    def _finish(self, reqs, lane, t_start, err=None):
        t = time.perf_counter()
        with self.cv:
            for r in reqs:
                r.t_start = t_start
                r.t_done = t
                r.lane = lane
                r.batch_size = len(reqs)
                r.error = err
                if r.cancelled and err is None:
                    r.error = Cancelled(f"request {r.id} cancelled while running")
                    r.poses = r.energy = None
                if r.key is not None and r.error is None:
                    self.resident[r.key] = r.poses
                r.done.set()

    def _initial_poses(self, r):
        """The poses a request starts from (on the current stream): its own, or with
        warm start the leading frames from the resident result of its key."""
        if not r.warm_start:
            return r.init_poses
        with self.cv:
            prev = self.resident.get(r.key)
        if prev is None:
            return r.init_poses
        n = min(prev.shape[0], r.num_frames)
        init = r.init_poses.clone()
        init[:n].copy_(prev[:n])
        r.warm_frames = n
        return init

    def forget(self, key):
        """Drop the resident result of `key` (its device memory is freed when no
        request holds it)."""
        with self.cv:
            self.resident.pop(key, None)

    def _batch_lane(self, ctx, stream):
        while True:
            reqs = self._next(self.small, True)
            if not reqs:
                return
            t0 = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    for r in reqs:
                        stream.wait_event(r.ready_event)
                    inits = [self._initial_poses(r) for r in reqs]
                    if len(reqs) == 1:
                        r = reqs[0]
                        res = bf.bf_gauss_newton(ctx, r.problem, inits[0], r.params)
                        r.poses, r.energy = res["poses"], res["energy"]
                    else:
                        dp, offs, init = concat_device(reqs, inits)
                        res = bf.bf_gauss_newton_batch(ctx, dp, offs, init, reqs[0].params)
                        for b, r in enumerate(reqs):
                            r.poses = res["poses"][offs[b]:offs[b + 1]].clone()
                            r.energy = res["energy"][b]
                    stream.synchronize()
                self.batches.append((len(reqs), time.perf_counter() - t0))
                self._finish(reqs, "batch", t0)
            except bf.BFError as e:
                self._finish(reqs, "batch", t0, e)
            finally:
                self._release(reqs)

    def _large_lane(self, ctx, stream):
        while True:
            reqs = self._next(self.large, False)
            if not reqs:
                return
            r = reqs[0]
            t0 = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    stream.wait_event(r.ready_event)
                    res = bf.bf_gauss_newton(ctx, r.problem, self._initial_poses(r), r.params)
                    r.poses, r.energy = res["poses"], res["energy"]
                    stream.synchronize()
                self._finish(reqs, "large", t0)
            except bf.BFError as e:
                self._finish(reqs, "large", t0, e)
            finally:
                self._release(reqs)


def concat_device(reqs, inits=None):
    """One DeviceProblem over the requests' frames (device copies on the current
    stream), their frame offsets and initial poses (`inits`, else the requests'
    own)."""
    offs = [0]
    for r in reqs:
        offs.append(offs[-1] + r.num_frames)
    P = [r.problem for r in reqs]
    depth = torch.cat([p.depth for p in P])
    inten = torch.cat([p.intensity for p in P])
    init = torch.cat(inits if inits is not None else [r.init_poses for r in reqs])
    with_c = [p for p in P if p.num_corrs > 0]
    if with_c:
        ci = torch.cat([p.keep[0] + o for p, o in zip(P, offs) if p.num_corrs > 0])
        cj = torch.cat([p.keep[1] + o for p, o in zip(P, offs) if p.num_corrs > 0])
        pi = torch.cat([p.keep[2] for p in with_c])
        pj = torch.cat([p.keep[3] for p in with_c])
        dp = bf.DeviceProblem(depth, inten, reqs[0].intr_key, ci, cj, pi, pj)
    else:
        dp = bf.DeviceProblem(depth, inten, reqs[0].intr_key)
    return dp, offs, init


def run_one_at_a_time(reqs, arrivals, ctx):
    """Baseline: one plain bf_gauss_newton per request, in arrival order, on one
    stream, each starting no earlier than its arrival."""
    t0 = time.perf_counter()
    for r, a in zip(reqs, arrivals):
        r.t_arrival = t0 + a
        now = time.perf_counter()
        if now < r.t_arrival:
            time.sleep(r.t_arrival - now)
        ts = time.perf_counter()
        res = bf.bf_gauss_newton(ctx, r.problem, r.init_poses, r.params)
        r.poses, r.energy = res["poses"], res["energy"]
        r.t_start, r.t_done, r.lane, r.batch_size = ts, time.perf_counter(), "plain", 1
        r.done.set()
    return time.perf_counter() - t0


def run_stream(server, reqs, arrivals):
    """Submit each request at its arrival time (seconds from now) and wait for all."""
    t0 = time.perf_counter()
    for r, a in zip(reqs, arrivals):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        server.submit(r, t_arrival=t0 + a)
    for r in reqs:
        r.done.wait()
    return time.perf_counter() - t0


def latency_stats(reqs, wall):
    import numpy as np
    lat = np.array([r.latency for r in reqs if r.error is None]) * 1e3
    return {"solves_per_s": round(len(lat) / wall, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "max_ms": round(float(lat.max()), 3),
            "errors": sum(r.error is not None for r in reqs), "requests": len(reqs)}
