"""A forward + backward view captured once as a HIP graph and replayed.

For a fixed scene and fixed image sizes the whole step (projection, binning
into a list buffer of fixed capacity, dispatch order, forward compositing,
backward compositing, projection backward) is the same sequence of about 40
launches every time.  Capturing it once removes the per-launch host cost
(Python marshalling and the launch calls), which is what bounds the time of
small scenes.  The step is a ``pipeline.ViewPipeline``, whose buffers are all
allocated before the capture; the cameras are its static slots, which
``replay`` fills first.

The intersection count stays on the device: a replay whose lists would
exceed the capacity builds them truncated (in bounds), so ``count()`` /
``fits()`` compare the device count with the capacity and the caller
captures again with more room when a view does not fit.  Nothing inside
the graph clears memory with a memset: the gradient buffers are zeroed by
the library's fill kernel.
"""
import torch

from . import rasterize as R
from .pipeline import ViewPipeline


class CapturedStep:
    """scene: means, quats, scales, opacities (activated) and sh (SH
    coefficients, or colours with sh_degree -1) as device tensors, which
    the graph reads at every replay (keep them alive; update them in place).
    W, H: per-camera sizes of the C views of one replay.  v_image: the
    upstream image gradient [P, 3], read at every replay.  capacity: list
    buffer entries (default: 1.25 x the count of ``warm_cams`` plus 1024)."""

    def __init__(self, p, scene, W, H, v_image, warm_cams, capacity=None):
        self.p = p
        self.W, self.H = [int(w) for w in W], [int(h) for h in H]
        d = scene["means"].device
        self.v_image = v_image
        if capacity is None:
            sc = scene
            proj = R.project(p, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"],
                             warm_cams[0], warm_cams[1], self.W, self.H)
            M = R.intersect(p, proj, self.W, self.H)["M"]         # eager: waits for the count
            capacity = int(M * 1.25) + 1024
        self.capacity = int(capacity)
        self.pipe = ViewPipeline(p, scene, self.W, self.H, self.capacity)
        self.pipe.set_cameras(*warm_cams)
        # one eager run of the exact captured sequence (first launches), on the capture's side stream
        side = torch.cuda.Stream(device=d)
        side.wait_stream(torch.cuda.current_stream(d))
        with torch.cuda.stream(side):
            self.pipe.step(self.v_image)
        torch.cuda.current_stream(d).wait_stream(side)
        torch.cuda.synchronize(d)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.pipe.step(self.v_image)
        pp = self.pipe
        self.out = dict(proj=pp.proj, isect=dict(total_dev=pp.totals, ids=pp.ids, ranges=pp.ranges),
                        fwd=dict(image=pp.image, alpha=pp.alpha, final_T=pp.final_T, last_ids=pp.last_ids),
                        g2=pp.g2, g3=pp.g3)

    def replay(self, viewmats, Ks):
        """Render and differentiate the views whose cameras are given
        ([C,4,4], [C,3,3] device tensors); returns the output buffers, which
        the next replay overwrites."""
        self.pipe.vm.copy_(viewmats)
        self.pipe.Ks.copy_(Ks)
        self.graph.replay()
        return self.out

    def count(self):
        """Intersections of the last replay (waits for it)."""
        return self.pipe.counts()[0]

    def fits(self):
        return self.count() <= self.capacity
