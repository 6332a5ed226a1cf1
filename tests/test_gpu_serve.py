"""Serving on the GPU: every request's image is the same alone and in the
mix of batched views of uneven sizes (the forward has no atomics, so equal
means bit-identical)."""
import numpy as np
import pytest
import torch

from paper_2409_06765_amd import scenes

pytestmark = pytest.mark.gpu


def test_served_images_equal_their_renders_alone():
    from _gpu import scene_to_dev, params
    from paper_2409_06765_amd import rasterize as R
    from paper_2409_06765_amd.serve import GpuBackend, Server
    print("[gpu-serve] 40 requests against a 20k-Gaussian scene", flush=True)
    sc = scenes.scene_clusters1m_sh3_1080p(n=20_000)
    d = scene_to_dev(sc)
    p = params(sh_degree=3)
    trace = scenes.serving_trace(3000.0, n_requests=40, seed=5,
                                 resolutions=[(64, 64), (128, 96), (200, 120), (256, 256)])
    be = GpuBackend(d, p)
    tickets, st = Server(be, max_batch=8, mem_budget=2 << 30).run(trace)
    assert st.n_done == 40 and st.mean_batch > 1.0
    for t in tickets:
        r = t.req
        vm = torch.from_numpy(r.viewmat[None]).cuda()
        K = torch.from_numpy(r.K[None]).cuda()
        proj = R.project(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, K, [r.W], [r.H])
        isect = R.intersect(p, proj, [r.W], [r.H])
        fwd = R.rasterize_forward(p, proj, d["opacities"], isect, [r.W], [r.H])
        alone = fwd["image"].view(r.H, r.W, 3).cpu().numpy()
        np.testing.assert_array_equal(t.image.cpu().numpy(), alone)
