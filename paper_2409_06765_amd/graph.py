"""A forward + backward view captured once as a HIP graph and replayed.

For a fixed scene and fixed image sizes the whole step (projection, binning
into a list buffer of fixed capacity, dispatch order, forward compositing,
backward compositing, projection backward) is the same sequence of about 40
launches every time.  Capturing it once removes the per-launch host cost
(Python marshalling and the launch calls), which is what bounds the time of
small scenes.  The cameras are a static slot that ``replay`` fills first.

The intersection count stays on the device: a replay whose lists would
exceed the capacity builds them truncated (in bounds), so ``count()`` /
``fits()`` compare the device count with the capacity and the caller
captures again with more room when a view does not fit.  Nothing inside
the graph clears memory with a memset: the backward zeroes its gradient
buffers with its own kernel.
"""
import torch

from . import rasterize as R


class CapturedStep:
    """scene: means, quats, scales, opacities (activated) and sh (SH
    coefficients, or colours with sh_degree -1) as device tensors, which
    the graph reads at every replay (keep them alive; update them in place).
    W, H: per-camera sizes of the C views of one replay.  v_image: the
    upstream image gradient [P, 3], read at every replay.  capacity: list
    buffer entries (default: 1.25 x the count of ``warm_cams`` plus 1024)."""

    def __init__(self, p, scene, W, H, v_image, warm_cams, capacity=None):
        self.p = p
        self.scene = scene
        self.W, self.H = [int(w) for w in W], [int(h) for h in H]
        C = len(self.W)
        d = scene["means"].device
        self.v_image = v_image
        self.vm = torch.empty((C, 4, 4), device=d, dtype=torch.float32)
        self.Ks = torch.empty((C, 3, 3), device=d, dtype=torch.float32)
        self.vm.copy_(warm_cams[0])
        self.Ks.copy_(warm_cams[1])
        if capacity is None:
            proj = self._project()
            M = R.intersect(p, proj, self.W, self.H)["M"]         # eager: waits for the count
            capacity = int(M * 1.25) + 1024
        self.capacity = int(capacity)
        # one eager run of the exact captured sequence (first launches, allocator warm-up)
        side = torch.cuda.Stream(device=d)
        side.wait_stream(torch.cuda.current_stream(d))
        with torch.cuda.stream(side):
            self._step()
        torch.cuda.current_stream(d).wait_stream(side)
        torch.cuda.synchronize(d)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = self._step()

    def _project(self):
        sc = self.scene
        return R.project(self.p, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], self.vm,
                         self.Ks, self.W, self.H)

    def _step(self):
        sc, p, W, H = self.scene, self.p, self.W, self.H
        proj = self._project()
        isect = R.intersect(p, proj, W, H, capacity=self.capacity, defer=True)
        fwd = R.rasterize_forward(p, proj, sc["opacities"], isect, W, H)
        g2 = R.rasterize_backward(p, proj, sc["opacities"], isect, W, H, fwd, self.v_image, overwrite=True)
        g3 = R.project_backward(p, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], self.vm,
                                self.Ks, W, H, proj, g2)
        return dict(proj=proj, isect=isect, fwd=fwd, g2=g2, g3=g3)

    def replay(self, viewmats, Ks):
        """Render and differentiate the views whose cameras are given
        ([C,4,4], [C,3,3] device tensors); returns the output buffers, which
        the next replay overwrites."""
        self.vm.copy_(viewmats)
        self.Ks.copy_(Ks)
        self.graph.replay()
        return self.out

    def count(self):
        """Intersections of the last replay (waits for it)."""
        return int(self.out["isect"]["total_dev"].item())

    def fits(self):
        return self.count() <= self.capacity
