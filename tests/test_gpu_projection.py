"""Projection backward term by term: one upstream gradient at a time (2D
means, conics, colours through the SH direction, opacities with the
anti-aliasing compensation) on Gaussians near the camera, inside and outside
the Jacobian clamp, with strong higher SH bands; the pose (view-matrix)
gradient with them.  The GPU result is judged
against the float64 oracle fed the same upstream gradients, allowing a few
times the float32 oracle's own distance from it."""
import numpy as np
import pytest
import torch

from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes
from _util import wide_cone_scene

pytestmark = pytest.mark.gpu
O32 = Oracle(np.float32)
O64 = Oracle(np.float64)


@pytest.mark.parametrize("which", ["v_means2d", "v_conics", "v_colors", "v_opacities", "all"])
@pytest.mark.parametrize("aa", [False, True])
def test_projection_backward_one_term_at_a_time(which, aa):
    from _gpu import assert_as_accurate_as_f32, np_, params, scene_to_dev, to_dev
    from paper_2409_06765_amd import rasterize as R
    print(f"[gpu-projection] {which} aa={aa}", flush=True)
    sc = wide_cone_scene(400, seed=5)
    cams = scenes.cams_tiny(W=120, H=90, f=80.0)
    P = OracleParams(sh_degree=3, antialiased=int(aa))
    p = params(sh_degree=3, antialiased=aa)
    args = (sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], cams["viewmats"], cams["Ks"],
            cams["W"], cams["H"])
    proj = O32.project(P, *args)
    vis = proj["radii"] > 0
    u = proj["means2d"][vis]
    lim = 1.3 * np.array([60.0, 45.0])
    outside = np.abs(u - np.array([60.0, 45.0])) > lim
    assert outside[:, 0].sum() >= 10 and outside[:, 1].sum() >= 10, "scene must exercise the clamp"
    g = np.random.default_rng(6)
    C, N = proj["radii"].shape
    up = dict(v_means2d=g.normal(0, 1, (C, N, 2)), v_conics=g.normal(0, 30, (C, N, 3)),
              v_colors=g.normal(0, 1, (C, N, 3)), v_opacities=g.normal(0, 1, (C, N)))
    for k in up:
        if which not in (k, "all"):
            up[k][:] = 0
        up[k] = (up[k] * vis.reshape(C, N, *([1] * (up[k].ndim - 2)))).astype(np.float32)
    ref32 = O32.project_bwd(P, *args, up["v_means2d"], up["v_conics"], up["v_colors"], up["v_opacities"],
                            viewmat_grad=True)
    ref64 = O64.project_bwd(P, *args, up["v_means2d"], up["v_conics"], up["v_colors"], up["v_opacities"],
                            viewmat_grad=True)
    d = scene_to_dev(sc)
    vm, Ks = to_dev(cams["viewmats"]), to_dev(cams["Ks"])
    W, H = [int(w) for w in cams["W"]], [int(h) for h in cams["H"]]
    gproj = R.project(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, Ks, W, H)
    np.testing.assert_array_equal(np_(gproj["radii"]), proj["radii"])
    g2 = {k: to_dev(v) for k, v in up.items()}
    g3 = R.project_backward(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, Ks, W, H, gproj, g2,
                            viewmat_grad=True)
    torch.cuda.synchronize()
    for k in ("v_means", "v_quats", "v_scales", "v_opacities", "v_sh", "v_viewmats"):
        assert_as_accurate_as_f32(np_(g3[k]), ref32[k], ref64[k], f"{which}:{k}")
