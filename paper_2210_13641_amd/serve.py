"""Render-request loop with continuous batching, interleaved with training.

The mapping thread keeps training while it renders for visualisation
(Sec. 3.3).  Requests (pose, intrinsics, image size) arrive at any time.
Each is admitted when its output buffers -- and, for the first request bound
to a parameter snapshot, that snapshot -- fit the memory budget, bound to
the parameter snapshot current at admission, and cut into 64-pixel tiles.
The budget defaults to the device memory free when the server starts, less
a reserve for the training step; a request that could never fit is
rejected (NSL_E_BUDGET) and the loop goes on.  Every
launch of nsl_render_batch packs tiles from all admitted requests, so a
request that arrives while others are rendering joins the next launch
instead of waiting for them to finish.  Because each tile reads its own
request's snapshot and rays are independent, a request's pixels are the
same whether it is rendered alone or in the mix.

Training steps run on their own stream; a snapshot is a copy of the live
parameters plus their MFMA operands, taken on the training stream after a
step and made visible to the render stream through an event.

Latency is measured from the request's scheduled arrival to a timing event
recorded on the render stream after the launch that holds its last tile;
it splits into queueing (arrival to admission, host clock) and service
(admission to completion).
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import nsl

OUT_BYTES_PER_PIXEL = 6 * 4       # rgb, depth, var, opacity (float32)


def tile_run(slot, first_pixel, n_tiles, n_pixels):
    """nsl_render_tile records [n_tiles, 3] (int32) of consecutive 64-pixel
    tiles of one request starting at first_pixel."""
    start = first_pixel + nsl.RENDER_TILE * np.arange(n_tiles, dtype=np.int64)
    out = np.empty((n_tiles, 3), np.int32)
    out[:, 0] = slot
    out[:, 1] = start
    out[:, 2] = np.minimum(nsl.RENDER_TILE, n_pixels - start)
    return out


@dataclasses.dataclass
class Snapshot:
    params: torch.Tensor
    prepared: torch.Tensor
    ready: torch.cuda.Event
    refs: int = 0
    version: int = 0

    @property
    def nbytes(self):
        return self.params.numel() * 4 + self.prepared.numel()


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # host seconds, relative to the server's clock origin
    pose: object
    intr: object
    H: int
    W: int
    snap: Snapshot = None
    out: list = None
    next_pixel: int = 0
    done_event: torch.cuda.Event = None
    latency: float = None
    admitted: float = None    # host seconds of admission
    error: int = 0            # nsl status: E_BUDGET when the request can never fit
    slot: int = -1

    @property
    def n_pixels(self):
        return self.H * self.W


def free_memory_budget(device, reserve_bytes):
    """Device memory free now, less a reserve (the training step's
    workspace and whatever else the caller will still allocate)."""
    free, _ = torch.cuda.mem_get_info(device)
    return max(0, int(free) - int(reserve_bytes))


class RenderServer:
    def __init__(self, field: nsl.Field, cfg: nsl.RenderConfig, device, budget_bytes=None, reserve_bytes=0,
                 tiles_per_launch=2048, max_inflight=2, keep_snapshots=False):
        """budget_bytes: memory the server may hold for outputs and request
        snapshots (None: free device memory at start, less reserve_bytes)."""
        self.field, self.cfg, self.device = field, cfg, device
        self.keep_snapshots = keep_snapshots
        self.launch_sizes = []                    # (requests, tiles) per launch
        self.budget = free_memory_budget(device, reserve_bytes) if budget_bytes is None else int(budget_bytes)
        self.used = 0
        self.peak_used = 0
        self.rejected = []
        self.held = []                            # admitted requests whose memory is not yet released
        self.admission_log = []                   # per admission: (requests held, snapshot versions held)
        self.tiles_per_launch = tiles_per_launch
        self.max_inflight = max_inflight
        self.stream = torch.cuda.Stream(device)
        self.pending = collections.deque()       # arrived, not admitted
        self.active = []                          # admitted, tiles left
        self.waiting = []                         # all tiles launched, not finished
        self.finished = []
        self.inflight = collections.deque()
        self.snap = None
        self.version = 0
        self.origin_event = torch.cuda.Event(enable_timing=True)
        self.origin_event.record(self.stream)
        torch.cuda.synchronize(device)
        self.origin = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.origin

    # -- snapshots -----------------------------------------------------------
    def publish(self, params, train_stream):
        """New snapshot of the live parameters, taken on the training stream
        after the work queued on it so far."""
        with torch.cuda.stream(train_stream):
            p = params.detach().clone()
            prep = nsl.prepare(self.field, p)
            ev = torch.cuda.Event()
            ev.record(train_stream)
        self.version += 1
        self.snap = Snapshot(p, prep, ev, 0, self.version)

    def _release(self, snap):
        snap.refs -= 1
        if snap.refs == 0:                        # its last request finished
            self.used -= snap.nbytes

    # -- requests -----------------------------------------------------------
    def submit(self, rid, arrival, pose, intr, H, W):
        self.pending.append(Request(rid, arrival, pose, intr, H, W))

    def _admit(self, now):
        while self.pending and self.pending[0].arrival <= now:
            r = self.pending[0]
            out_bytes = r.n_pixels * OUT_BYTES_PER_PIXEL
            snap_bytes = self.snap.nbytes if self.snap.refs == 0 else 0   # charged to its first request
            if out_bytes + self.snap.nbytes > self.budget:                # can never fit
                self.pending.popleft()
                r.error = nsl.E_BUDGET
                self.rejected.append(r)
                continue
            if self.used + out_bytes + snap_bytes > self.budget:
                break                              # wait for memory to free up
            self.pending.popleft()
            self.used += out_bytes + snap_bytes
            self.peak_used = max(self.peak_used, self.used)
            r.admitted = now
            n = r.n_pixels
            dev = self.device
            with torch.cuda.stream(self.stream):
                r.out = [torch.empty(n, 3, device=dev), torch.empty(n, device=dev), torch.empty(n, device=dev),
                         torch.empty(n, device=dev)]
            r.snap = self.snap
            r.snap.refs += 1
            self.held.append(r)
            self.admission_log.append((len(self.held), len({h.snap.version for h in self.held})))
            self.stream.wait_event(r.snap.ready)
            self.active.append(r)

    def _launch(self):
        if not self.active:
            return
        # Each active request gets a contiguous run of its next tiles; the
        # launch budget is shared evenly (round robin over requests).
        reqs, runs = [], []
        budget = self.tiles_per_launch
        left = [r for r in self.active if r.next_pixel < r.n_pixels]
        while budget > 0 and left:
            share = max(1, budget // len(left))
            nxt = []
            for r in left:
                if budget == 0:
                    nxt.append(r)
                    continue
                remaining = -(-(r.n_pixels - r.next_pixel) // nsl.RENDER_TILE)
                k = min(share, remaining, budget)
                if r.slot < 0:
                    r.slot = len(reqs)
                    reqs.append(nsl.render_request(r.snap.params, r.snap.prepared, r.pose, r.intr, r.H, r.W,
                                                   *r.out))
                runs.append((r.slot, r.next_pixel, k, r.n_pixels))
                r.next_pixel = min(r.n_pixels, r.next_pixel + k * nsl.RENDER_TILE)
                budget -= k
                if r.next_pixel < r.n_pixels:
                    nxt.append(r)
            left = nxt
        tiles = np.concatenate([tile_run(*x) for x in runs])
        with torch.cuda.stream(self.stream):
            rq = nsl.records_to_device(reqs, nsl.RenderRequest, self.device)
            tl = nsl.bytes_to_device(tiles.tobytes(), self.device)
            nsl.render_batch(self.field, rq, len(reqs), tl, len(tiles), self.cfg)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(self.stream)
        self.inflight.append((ev, rq, tl))
        self.launch_sizes.append((len(reqs), len(tiles)))
        still = []
        for r in self.active:
            r.slot = -1
            if r.next_pixel >= r.n_pixels:
                r.done_event = ev
                self.waiting.append(r)
            else:
                still.append(r)
        self.active = still

    def _poll(self, block=False):
        """Retire finished launches (with block, wait for the oldest one)."""
        if block and self.inflight:
            self.inflight.popleft()[0].synchronize()
        while self.inflight and self.inflight[0][0].query():
            self.inflight.popleft()
        keep = []
        for r in self.waiting:
            if r.done_event.query():
                done = self.origin_event.elapsed_time(r.done_event) / 1e3
                r.latency = done - r.arrival
                self.used -= r.n_pixels * OUT_BYTES_PER_PIXEL
                self.held.remove(r)
                self._release(r.snap)
                if not self.keep_snapshots:
                    r.snap = None
                    r.out = None
                self.finished.append(r)
            else:
                keep.append(r)
        self.waiting = keep

    def pump(self):
        """One scheduling round: admit, launch, collect."""
        now = self.now()
        self._admit(now)
        while len(self.inflight) >= self.max_inflight:
            self._poll(block=True)
        self._launch()
        self._poll()

    def drain(self):
        while self.pending or self.active or self.waiting or self.inflight:
            if self.pending and not self.active and not self.waiting:
                wait = self.pending[0].arrival - self.now()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
            self.pump()
            self._poll(block=not self.active and not self.pending)


def serve(field, cfg, device, requests, params, train_fn=None, train_period=5e-3, budget_bytes=None,
          reserve_bytes=0, tiles_per_launch=2048, warmup=0, keep_snapshots=False):
    """Run the loop over `requests` (dicts with arrival, pose [12], intr [4],
    H, W).  train_fn() queues one training step on the current stream (the
    loop makes its training stream current); it is called every
    train_period seconds of host time.  The memory budget is budget_bytes,
    or the free device memory at start less reserve_bytes.  Returns the
    server, the finished requests (with latency) and run statistics;
    rejected requests are in srv.rejected."""
    train_stream = torch.cuda.Stream(device)
    srv = RenderServer(field, cfg, device, budget_bytes, reserve_bytes, tiles_per_launch,
                       keep_snapshots=keep_snapshots)
    srv.publish(params, train_stream)
    for i, q in enumerate(requests):
        srv.submit(i, q["arrival"], q["pose"], q["intr"], q["H"], q["W"])
    steps = 0
    next_train = 0.0
    t_start = srv.now()
    while srv.pending or srv.active or srv.waiting or srv.inflight:
        now = srv.now()
        if train_fn is not None and now >= next_train:
            with torch.cuda.stream(train_stream):
                train_fn()
            steps += 1
            next_train += train_period
            srv.publish(params, train_stream)
        srv.pump()
        if not srv.active and srv.pending:
            wait = srv.pending[0].arrival - srv.now()      # read the clock once
            if wait > 0:
                time.sleep(min(wait, 2e-4))
    torch.cuda.synchronize(device)
    wall = srv.now() - t_start
    done = sorted(srv.finished, key=lambda r: r.rid)
    measured = [r for r in done if r.rid >= warmup]
    lat = sorted(r.latency for r in measured)
    pix = sum(r.n_pixels for r in measured)
    span = (max(r.arrival + r.latency for r in measured) - min(r.arrival for r in measured)) if measured else 0.0

    def pct(p):
        return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))] if lat else None

    def pcts(xs):
        xs = sorted(xs)
        if not xs:
            return None
        at = lambda p: xs[min(len(xs) - 1, int(round(p / 100.0 * (len(xs) - 1))))]
        return {"p50_ms": 1e3 * at(50), "p99_ms": 1e3 * at(99), "n": len(xs)}

    by_size = {}
    for r in measured:
        by_size.setdefault(f"{r.W}x{r.H}", []).append(r.latency)
    stats = dict(requests=len(measured), p50_ms=1e3 * pct(50) if lat else None,
                 p99_ms=1e3 * pct(99) if lat else None, rays_per_s=pix / span if span > 0 else None,
                 train_steps=steps, wall_s=wall, launches=len(srv.launch_sizes),
                 max_requests_per_launch=max((a for a, _ in srv.launch_sizes), default=0),
                 queueing=pcts([r.admitted - r.arrival for r in measured]),
                 service=pcts([r.arrival + r.latency - r.admitted for r in measured]),
                 latency_by_size={k: pcts(v) for k, v in sorted(by_size.items())},
                 budget_bytes=srv.budget, peak_used_bytes=srv.peak_used, rejected=len(srv.rejected))
    return srv, done, stats
