"""The captured forward + backward step (paper_2409_06765_amd/graph.py).

Replays of one captured graph for different views, with eager work and
synchronisations between them, against the eager step for the same view:
forward outputs bit for bit (same lists, same order), gradients to float
atomics' rounding; a capacity that is too small is detected (the count on
the device exceeds it) and the truncated lists stay in bounds.
"""
import numpy as np
import pytest
import torch

from paper_2409_06765_amd import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-graph] {msg}", flush=True)


def _setup(deg=3, n=3000, seed=5):
    from _gpu import to_dev
    sc = scenes.scene_tiny(n, sh_degree=deg, seed=seed, log_scale_mean=-2.6)
    cams = scenes.cams_tiny(W=96, H=72, f=80.0, n_cams=3, seed=seed)
    d = {k: to_dev(v) for k, v in sc.items() if isinstance(v, np.ndarray)}
    vm, Ks = to_dev(cams["viewmats"]), to_dev(cams["Ks"])
    v_image = to_dev(np.random.default_rng(seed).normal(size=(96 * 72, 3)).astype(np.float32))
    return d, vm, Ks, v_image


def _eager(p, d, vm, Ks, v_image, v):
    from paper_2409_06765_amd import rasterize as R
    W, H = [96], [72]
    proj = R.project(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm[v:v + 1], Ks[v:v + 1], W, H)
    isect = R.intersect(p, proj, W, H)
    fwd = R.rasterize_forward(p, proj, d["opacities"], isect, W, H)
    if isect.check():
        fwd = R.rasterize_forward(p, proj, d["opacities"], isect, W, H)
    g2 = R.rasterize_backward(p, proj, d["opacities"], isect, W, H, fwd, v_image)
    g3 = R.project_backward(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm[v:v + 1],
                            Ks[v:v + 1], W, H, proj, g2)
    torch.cuda.synchronize()
    return dict(fwd={k: fwd[k].cpu().numpy() for k in ("image", "alpha", "final_T", "last_ids")},
                g3={k: g3[k].cpu().numpy() for k in ("v_means", "v_quats", "v_scales", "v_opacities", "v_sh")},
                M=isect["M"])


def _close(got, ref, name):
    scale = max(np.abs(ref).max(), 1e-30)
    assert np.abs(got - ref).max() <= 1e-5 * scale, name


def test_replays_match_the_eager_step():
    from paper_2409_06765_amd import rasterize as R
    from paper_2409_06765_amd.graph import CapturedStep
    p = R.make_params(sh_degree=3)
    d, vm, Ks, v_image = _setup()
    ref = [_eager(p, d, vm, Ks, v_image, v) for v in range(3)]
    cs = CapturedStep(p, d, [96], [72], v_image, (vm[0:1], Ks[0:1]))
    _say(f"captured: capacity {cs.capacity}, counts {[r['M'] for r in ref]}")
    for i, v in enumerate([0, 1, 2, 0, 2, 1]):
        out = cs.replay(vm[v:v + 1], Ks[v:v + 1])
        torch.cuda.synchronize()
        assert cs.fits() and cs.count() == ref[v]["M"]
        for k in ("image", "alpha", "final_T", "last_ids"):
            np.testing.assert_array_equal(out["fwd"][k].cpu().numpy(), ref[v]["fwd"][k], err_msg=f"{i}:{k}")
        for k in ref[v]["g3"]:
            _close(out["g3"][k].cpu().numpy(), ref[v]["g3"][k], f"{i}:{k}")
        # the program's own eager work between replays
        _eager(p, d, vm, Ks, v_image, (v + 1) % 3)
        torch.cuda.synchronize()


def test_a_small_capacity_is_detected():
    from paper_2409_06765_amd import rasterize as R
    from paper_2409_06765_amd.graph import CapturedStep
    p = R.make_params(sh_degree=3)
    d, vm, Ks, v_image = _setup(seed=6)
    cs = CapturedStep(p, d, [96], [72], v_image, (vm[0:1], Ks[0:1]), capacity=1024)
    cs.replay(vm[0:1], Ks[0:1])
    torch.cuda.synchronize()
    _say(f"count {cs.count()} capacity {cs.capacity}")
    assert cs.count() > 1024 and not cs.fits()
    ref = _eager(p, d, vm, Ks, v_image, 0)
    assert cs.count() == ref["M"]
