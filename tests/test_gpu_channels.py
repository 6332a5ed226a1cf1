"""N-D feature channels and depth rendering on the GPU against the oracle.

Feature counts D = 1 .. 32 (shared [N,D] and per-camera [C,N,D]), RGB plus
accumulated or expected depth, and depth alone, through the C ABI: images
within 1e-4 times the channel's magnitude (at least 1) outside the pixels the
oracle flags as near a threshold, last_ids bit-exact there; gradients (2D
means, conics, opacities, features, depths) within 1e-3 relative
(tests/_gpu.assert_grad_close); and the whole chain through rasterization()
with expected depth against the oracle's projection backward.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes

pytestmark = pytest.mark.gpu

O32 = Oracle(np.float32)


def _say(msg):
    print(f"[gpu-channels] {msg}", flush=True)


@pytest.fixture(scope="module")
def base():
    from _gpu import gpu_forward, params
    sc = scenes.scene_tiny(600, seed=71, log_scale_mean=-2.4)
    cams = scenes.cams_tiny(W=83, H=61, f=60.0, n_cams=2, seed=71)
    P = OracleParams()
    p = params()
    st = gpu_forward(p, sc, cams)
    proj, isect, ras = O32.forward(P, sc, cams)
    return sc, cams, P, st, proj, isect, ras


# (D, shared, depth mode)
CASES = [(1, True, "none"), (2, False, "none"), (4, True, "none"), (5, False, "none"), (16, True, "none"),
         (32, False, "none"), (3, False, "accumulated"), (3, False, "expected"), (0, True, "accumulated"),
         (0, True, "expected"), (5, True, "expected"), (31, False, "accumulated")]


def _features(proj, D, shared, seed):
    C, N = proj["radii"].shape
    g = np.random.default_rng(seed)
    if D == 3 and not shared:
        return None                                    # the projected colours
    shape = (N, D) if shared else (C, N, D)
    return g.uniform(-1.0, 2.0, shape).astype(np.float32)


@pytest.mark.parametrize("D,shared,depth", CASES, ids=[f"D{d}{'s' if s else 'c'}-{m}" for d, s, m in CASES])
def test_channels_forward_and_backward(base, D, shared, depth):
    from _gpu import assert_grad_close, np_, params, to_dev
    from paper_2409_06765_amd import rasterize as R
    sc, cams, P, st, proj, isect, ras = base
    _say(f"D={D} shared={shared} depth={depth}")
    feats = _features(proj, D, shared, seed=D + 100 * shared)
    p = params(render_depth=depth)
    fdev = None if feats is None else to_dev(feats)
    if D == 0:
        fdev = to_dev(np.zeros((proj["radii"].shape[1], 0), np.float32))
    bg = None
    if D > 0:
        bg = np.random.default_rng(D).uniform(0.0, 1.0, (len(cams["W"]), D)).astype(np.float32)
    fwd = R.rasterize_forward(p, st["proj"], st["d"]["opacities"], st["isect"], st["W"], st["H"],
                              None if bg is None else to_dev(bg), features=fdev)
    ofeat = feats if D > 0 else np.zeros((proj["radii"].shape[1], 0), np.float32)
    ref = O32.channels_fwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"],
                           features=ofeat, depth=depth, background=bg)
    img = np_(fwd["image"])
    Dt = D + (depth != "none")
    assert img.shape == (ras["final_T"].shape[0], Dt) and ref["image"].shape == img.shape
    ok = ras["flags"] == 0
    scale = np.maximum(np.abs(ref["image"][ok]).max(axis=0), 1.0)
    err = (np.abs(img - ref["image"])[ok] / scale).max()
    assert err <= 1e-4, err
    np.testing.assert_array_equal(np_(fwd["last_ids"])[ok], ras["last_ids"][ok])

    g = np.random.default_rng(7 + D)
    v_image = g.normal(size=img.shape).astype(np.float32)
    v_alpha = g.normal(size=ras["final_T"].shape).astype(np.float32)
    v_image[~ok] = 0
    v_alpha[~ok] = 0
    g2 = R.rasterize_backward(p, st["proj"], st["d"]["opacities"], st["isect"], st["W"], st["H"], fwd,
                              to_dev(v_image), to_dev(v_alpha), None if bg is None else to_dev(bg),
                              features=fdev)
    o2 = O32.channels_bwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"], ref,
                          v_image, v_alpha, features=ofeat, depth=depth, background=bg, abs_sums=True)
    keys = ["v_means2d", "v_conics", "v_opacities"] + (["v_colors"] if D > 0 else []) + \
        (["v_depths"] if depth != "none" else [])
    for k in keys:
        abs_ref = o2.get("abs_" + k)
        if k == "v_colors" and shared:
            abs_ref = None                     # summed over cameras: the per-camera magnitudes add
        assert_grad_close(np_(g2[k]), o2[k], f"D{D}:{depth}:{k}", abs_ref=abs_ref)
    if D == 0:
        assert g2["v_colors"] is None or g2["v_colors"].numel() == 0


def test_expected_depth_through_rasterization_matches_oracle_chain():
    """rasterization(render_mode="RGB+ED") with SH degree 1: image and alpha
    against the oracle, and the gradients of the Gaussians' parameters
    (including the depth channel's way through t_z) against the oracle's
    projection backward fed by its compositing backward."""
    import torch
    from _gpu import assert_chain_close, np_, oracle_project_bwd, to_dev
    from paper_2409_06765_amd.rasterize import rasterization
    sc = scenes.scene_tiny(300, sh_degree=1, seed=77, log_scale_mean=-2.4)
    cams = scenes.cams_tiny(W=72, H=56, f=55.0, n_cams=2, seed=77)
    P = OracleParams(sh_degree=1)
    proj, isect, ras = O32.forward(P, sc, cams)
    args = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"])
    ref = O32.channels_fwd(*args, depth="expected")
    t = {k: to_dev(sc[k]).requires_grad_(True) for k in ("means", "quats", "scales", "opacities", "sh")}
    img, alpha, meta = rasterization(t["means"], t["quats"], t["scales"], t["opacities"], t["sh"],
                                     to_dev(cams["viewmats"]), to_dev(cams["Ks"]), 72, 56, sh_degree=1,
                                     render_mode="RGB+ED")
    assert tuple(img.shape) == (2, 56, 72, 4)
    ok = ras["flags"] == 0
    gi = np_(img).reshape(-1, 4)
    scale = np.maximum(np.abs(ref["image"][ok]).max(axis=0), 1.0)
    assert (np.abs(gi - ref["image"])[ok] / scale).max() <= 1e-4
    g = np.random.default_rng(78)
    v_image = g.normal(size=ref["image"].shape).astype(np.float32)
    v_image[~ok] = 0
    loss = (img * to_dev(v_image).view(img.shape)).sum()
    loss.backward()
    torch.cuda.synchronize()
    # the chain (compositing gradients from meta, then the projection backward with the depth channel's way
    # through t_z) against the float64 oracle chain
    O64 = Oracle(np.float64)
    ref64 = O64.channels_fwd(*args, depth="expected")
    o2x = O64.channels_bwd(*args, ref64, v_image, depth="expected")
    g2 = {k: np_(v) for k, v in meta["grads2d"].items() if v is not None}
    g3 = {ko: np_(t[k].grad) for k, ko in (("means", "v_means"), ("quats", "v_quats"), ("scales", "v_scales"),
                                            ("opacities", "v_opacities"), ("sh", "v_sh"))}
    pb32, pb64 = oracle_project_bwd(O32, P, sc, cams), oracle_project_bwd(O64, P, sc, cams)
    assert_chain_close(g3, g2, o2x, pb64(o2x), pb32, pb64, "RGB+ED")


def test_channel_count_limits_are_rejected():
    from _gpu import params, to_dev
    from paper_2409_06765_amd import _lib as L
    from paper_2409_06765_amd import rasterize as R
    sc = scenes.scene_tiny(50, seed=3)
    cams = scenes.cams_tiny(W=32, H=32, f=30.0)
    from _gpu import gpu_forward
    st = gpu_forward(params(), sc, cams)
    N = st["proj"]["radii"].shape[1]
    for D, depth in ((33, "none"), (32, "accumulated"), (0, "none")):
        with pytest.raises(L.GsrError):
            R.rasterize_forward(params(render_depth=depth), st["proj"], st["d"]["opacities"], st["isect"],
                                st["W"], st["H"], features=to_dev(np.zeros((N, D), np.float32)))
