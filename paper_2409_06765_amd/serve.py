"""Continuous-batching render server over a resident Gaussian scene.

Requests (pose, intrinsics, width, height) arrive over time.  Each step the
scheduler admits waiting requests in arrival order while a slot is free
(at most ``max_batch`` views, capped by the library's camera limit) and while
their estimated device memory fits the budget; it then renders the admitted
views of different resolutions together: one projection, one binning pass
and one compositing launch over the tiles of all of them.  Work overlaps on
the device: the next step's projection and binning run on a second stream
while the current step composites, so requests that arrive while others are
on the GPU are admitted as soon as slots and memory free up.

The memory of a request is its per-view state (projected arrays, packed
records, binning workspace: about ``bytes_per_gaussian`` per Gaussian), its
image buffers (24 B per pixel) and its intersection lists (about 20 B per
intersection, the count estimated from the observed intersections per pixel
and corrected once the batch's real count is known).  A request larger than
the whole budget is rejected.

``Server`` is backend-agnostic: ``GpuBackend`` runs the HIP path, and the
tests drive the same scheduler with a CPU backend.
"""
import collections
import dataclasses
import time

import numpy as np

MAX_CAMERAS = 64


@dataclasses.dataclass
class Ticket:
    req: object
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    image: object = None
    error: str = None


@dataclasses.dataclass
class ServeStats:
    n_done: int
    n_rejected: int
    wall_s: float
    views_per_s: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    steps: int
    max_inflight_bytes: int


class Server:
    """Scheduler.  ``backend`` provides:
      bytes_for(req, m_per_px) -> int       estimated device bytes of one request
      prepare(reqs) -> handle                start projection + binning (may wait for M)
      finish(handle) -> None                 start compositing (asynchronous)
      poll(handle) -> bool                   True once the images are ready
      collect(handle) -> list of images      images in request order
      now() -> float                         the clock (seconds)
      idle(until) -> None                    wait for an arrival or for device work
    """

    def __init__(self, backend, max_batch=16, mem_budget=8 << 30, overlap=True):
        self.b = backend
        self.max_batch = max(1, min(int(max_batch), MAX_CAMERAS))
        self.budget = int(mem_budget)
        self.overlap = overlap
        self.m_per_px = 4.0            # intersections per pixel, refined as batches complete

    def _admit(self, waiting, rejected, avail):
        """Takes waiting requests in arrival order while slots and ``avail``
        bytes last; a request that could never fit the whole budget is
        rejected, one that only has to wait for memory stays queued."""
        batch, used = [], 0
        while waiting and len(batch) < self.max_batch:
            t = waiting[0]
            need = self.b.bytes_for(t.req, self.m_per_px)
            if need > self.budget:
                waiting.popleft()
                t.error = f"needs {need} bytes, budget {self.budget}"
                rejected.append(t)
                continue
            if used + need > avail:
                break
            batch.append(waiting.popleft())
            used += need
        return batch, used

    def run(self, trace):
        """Serve ``trace`` (objects with ``arrival`` in seconds from the start);
        returns (tickets in request order, ServeStats)."""
        tickets = [Ticket(r, r.arrival) for r in trace]
        order = sorted(range(len(tickets)), key=lambda i: tickets[i].arrival)
        waiting = collections.deque()
        rejected = []
        t0 = self.b.now()
        nxt = 0
        inflight = None          # (handle, batch, bytes) compositing on the device
        staged = None            # (handle, batch, bytes) projected and binned, not yet composited
        steps, batch_sizes, peak = 0, [], 0

        def arrivals(now):
            nonlocal nxt
            while nxt < len(order) and tickets[order[nxt]].arrival <= now - t0:
                waiting.append(tickets[order[nxt]])
                nxt += 1

        while nxt < len(order) or waiting or inflight or staged:
            now = self.b.now()
            arrivals(now)
            # retire the batch on the device
            if inflight is not None and self.b.poll(inflight[0]):
                h, batch, _ = inflight
                imgs = self.b.collect(h)
                fin = self.b.now() - t0
                for t, im in zip(batch, imgs):
                    t.image, t.finished = im, fin
                m = getattr(h, "M", None)
                px = sum(t.req.W * t.req.H for t in batch)
                if m is not None and px > 0:
                    self.m_per_px = 0.7 * self.m_per_px + 0.3 * (m / px)
                inflight = None
            # start compositing the staged batch
            if inflight is None and staged is not None:
                self.b.finish(staged[0])
                inflight, staged = staged, None
            # stage the next batch (overlaps the compositing in flight)
            if staged is None and waiting and (self.overlap or inflight is None):
                avail = self.budget - (inflight[2] if inflight else 0)
                batch, used = self._admit(waiting, rejected, avail)
                if batch:
                    adm = self.b.now() - t0
                    for t in batch:
                        t.admitted = adm
                    h = self.b.prepare([t.req for t in batch])
                    staged = (h, batch, used)
                    steps += 1
                    batch_sizes.append(len(batch))
                    peak = max(peak, used + (inflight[2] if inflight else 0))
                    continue
            if inflight is None and staged is None:
                if waiting:
                    continue
                if nxt < len(order):
                    self.b.idle(t0 + tickets[order[nxt]].arrival)
                continue
            if inflight is not None:
                self.b.idle(None)

        wall = self.b.now() - t0
        done = [t for t in tickets if t.image is not None]
        lat = np.array([1e3 * (t.finished - t.arrival) for t in done]) if done else np.zeros(1)
        stats = ServeStats(n_done=len(done), n_rejected=len(rejected), wall_s=wall,
                           views_per_s=len(done) / wall if wall > 0 else 0.0,
                           p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                           mean_batch=float(np.mean(batch_sizes)) if batch_sizes else 0.0, steps=steps,
                           max_inflight_bytes=int(peak))
        return tickets, stats


class GpuBackend:
    """HIP backend: the scene stays resident; a batch is rendered as C views of
    different sizes in one projection, one binning pass and one compositing
    launch.  Projection and binning run on ``stage_stream``, compositing on
    ``raster_stream``."""

    BYTES_PER_GAUSSIAN = 40 + 48 + 92    # projected arrays + packed record + binning workspace

    def __init__(self, scene, params, device="cuda:0"):
        import torch
        from . import rasterize as R
        self.torch, self.R = torch, R
        self.dev = device
        self.scene = scene
        self.p = params
        self.N = int(scene["means"].shape[0])
        self.stage_stream = torch.cuda.Stream(device=device)
        self.raster_stream = torch.cuda.Stream(device=device)

    def now(self):
        return time.perf_counter()

    def idle(self, until):
        if until is None:
            time.sleep(0)
            return
        dt = until - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.002))

    def bytes_for(self, req, m_per_px):
        px = req.W * req.H
        return int(self.BYTES_PER_GAUSSIAN * self.N + 24 * px + 20 * m_per_px * px + (1 << 20))

    def prepare(self, reqs):
        torch, R = self.torch, self.R

        class H:
            pass
        h = H()
        h.W = [int(r.W) for r in reqs]
        h.H = [int(r.H) for r in reqs]
        with torch.cuda.stream(self.stage_stream):
            vm = torch.from_numpy(np.stack([r.viewmat for r in reqs]).astype(np.float32)).to(self.dev, non_blocking=False)
            Ks = torch.from_numpy(np.stack([r.K for r in reqs]).astype(np.float32)).to(self.dev, non_blocking=False)
            s = self.scene
            h.proj = R.project(self.p, s["means"], s["quats"], s["scales"], s["opacities"], s["sh"], vm, Ks, h.W, h.H,
                               stream=self.stage_stream)
            h.isect = R.intersect(self.p, h.proj, h.W, h.H, stream=self.stage_stream)
            h.ready = torch.cuda.Event()
            h.ready.record(self.stage_stream)
        return h

    def finish(self, h):
        torch, R = self.torch, self.R
        # the count is long on the host by now; lists that overflowed their capacity are rebuilt on the
        # staging stream, which the compositing then waits for
        if h.isect.check():
            h.ready = torch.cuda.Event()
            h.ready.record(self.stage_stream)
        h.M = h.isect["M"]
        self.raster_stream.wait_event(h.ready)
        with torch.cuda.stream(self.raster_stream):
            h.fwd = R.rasterize_forward(self.p, h.proj, self.scene["opacities"], h.isect, h.W, h.H,
                                        stream=self.raster_stream)
            h.done = torch.cuda.Event()
            h.done.record(self.raster_stream)

    def poll(self, h):
        return h.done.query()

    def collect(self, h):
        h.done.synchronize()
        out, off = [], 0
        for w, hh in zip(h.W, h.H):
            out.append(h.fwd["image"][off:off + w * hh].view(hh, w, 3))
            off += w * hh
        return out


def serve_one_at_a_time(backend, trace):
    """The reference policy: one view per launch, no batching, no overlap."""
    return Server(backend, max_batch=1, overlap=False).run(trace)
