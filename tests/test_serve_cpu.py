"""The continuous-batching scheduler, driven on the CPU by a backend that
renders with the oracle and advances a simulated clock (no GPU)."""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes
from paper_2409_06765_amd.serve import MAX_CAMERAS, Server, serve_one_at_a_time

O32 = Oracle(np.float32)


class SimBackend:
    """Renders with the oracle; a batch of views costs `fixed + per_px * pixels`
    simulated seconds; the clock only moves when the scheduler waits."""

    def __init__(self, scene, P, fixed=0.004, per_px=2e-8, bytes_per_view=1 << 20, m_per_px_true=3.0):
        self.scene, self.P = scene, P
        self.fixed, self.per_px = fixed, per_px
        self.t = 0.0
        self.bytes_per_view = bytes_per_view
        self.m_true = m_per_px_true
        self.busy_until = 0.0
        self.log = []

    def now(self):
        return self.t

    def idle(self, until):
        if until is None:
            self.t = max(self.t, self.busy_until)
        else:
            self.t = max(self.t, until)

    def bytes_for(self, req, m_per_px):
        return int(self.bytes_per_view + 20 * m_per_px * req.W * req.H)

    def prepare(self, reqs):
        class H:
            pass
        h = H()
        h.reqs = reqs
        h.M = int(self.m_true * sum(r.W * r.H for r in reqs))
        self.log.append(len(reqs))
        return h

    def finish(self, h):
        px = sum(r.W * r.H for r in h.reqs)
        start = max(self.t, self.busy_until)
        self.busy_until = start + self.fixed + self.per_px * px
        h.done_at = self.busy_until
        cams = scenes.cameras([r.viewmat for r in h.reqs], [r.K for r in h.reqs], [r.W for r in h.reqs],
                              [r.H for r in h.reqs])
        _, _, ras = O32.forward(self.P, self.scene, cams)
        h.images, off = [], 0
        for r in h.reqs:
            h.images.append(ras["image"][off:off + r.W * r.H].reshape(r.H, r.W, 3))
            off += r.W * r.H

    def poll(self, h):
        return self.t >= h.done_at

    def collect(self, h):
        return h.images


def _small_trace(n=24, rate=400.0, seed=3):
    res = [(32, 32), (48, 40), (64, 48), (40, 64)]
    tr = scenes.serving_trace(rate, n_requests=n, seed=seed, resolutions=res)
    for r in tr:     # a small focal so the tiny scene fills these small views
        r.K = scenes.intrinsics(1.0 * r.W, r.W, r.H).astype(np.float32)
        r.viewmat = scenes.look_at(4.0 * r.viewmat[:3, :3].T @ np.array([0, 0, -1.0])).astype(np.float32)
    return tr


@pytest.fixture(scope="module")
def scene():
    return scenes.scene_tiny(200, sh_degree=1, seed=8, log_scale_mean=-2.5)


def test_every_request_served_and_each_image_equals_its_render_alone(scene):
    P = OracleParams(sh_degree=1)
    be = SimBackend(scene, P)
    trace = _small_trace()
    tickets, st = Server(be, max_batch=6, mem_budget=64 << 20).run(trace)
    assert st.n_done == len(trace) and st.n_rejected == 0
    assert max(be.log) > 1, "requests that arrive together must be batched"
    for t in tickets:
        r = t.req
        cams = scenes.cameras([r.viewmat], [r.K], [r.W], [r.H])
        _, _, ras = O32.forward(P, scene, cams)
        np.testing.assert_array_equal(t.image, ras["image"].reshape(r.H, r.W, 3))
        assert t.arrival <= t.admitted <= t.finished


def test_batches_respect_slots_memory_and_arrival_order(scene):
    P = OracleParams(sh_degree=1)
    be = SimBackend(scene, P, bytes_per_view=10 << 20)
    trace = _small_trace(n=30, rate=5000.0)
    budget = 45 << 20      # about four views at a time
    tickets, st = Server(be, max_batch=8, mem_budget=budget).run(trace)
    assert st.n_done == 30
    assert max(be.log) <= 4 and st.max_inflight_bytes <= budget
    adm = [t.admitted for t in sorted(tickets, key=lambda t: t.arrival)]
    assert all(a <= b for a, b in zip(adm, adm[1:])), "admission must follow arrival order"


def test_request_larger_than_the_budget_is_rejected_others_served(scene):
    P = OracleParams(sh_degree=1)
    be = SimBackend(scene, P, bytes_per_view=1 << 20)
    trace = _small_trace(n=10)
    trace[3].W, trace[3].H = 4000, 4000           # would need ~1.3 GB of lists
    tickets, st = Server(be, max_batch=4, mem_budget=64 << 20).run(trace)
    assert st.n_rejected == 1 and st.n_done == 9
    assert tickets[3].image is None and "budget" in tickets[3].error


def test_batching_beats_one_view_per_launch_under_load(scene):
    P = OracleParams(sh_degree=1)
    trace = _small_trace(n=40, rate=2000.0)
    _, batched = Server(SimBackend(scene, P), max_batch=16, mem_budget=256 << 20).run(trace)
    _, single = serve_one_at_a_time(SimBackend(scene, P), trace)
    assert batched.n_done == single.n_done == 40
    assert batched.p99_ms < single.p99_ms
    assert batched.views_per_s > single.views_per_s


def test_slot_cap_is_the_library_camera_limit(scene):
    assert Server(SimBackend(scene, OracleParams()), max_batch=1000).max_batch == MAX_CAMERAS
