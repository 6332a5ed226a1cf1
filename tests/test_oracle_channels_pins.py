"""Pins of the oracle's N-D feature and depth channels (no GPU).

N-dimensional features composite every channel with the same alpha and T;
depth rendering (Depth rendering appendix) composites z as a channel,
accumulated (sum z alpha T) or expected (divided by sum alpha T).  Pinned by
channel independence, linearity of the backward in the upstream gradient,
closed forms for one and two Gaussians, the telescoping identity
sum alpha T = 1 - final T, and central differences of the rendered loss.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes
from _util import one_gaussian_scene, simple_cam, stack_scenes

O64 = Oracle(np.float64)
O32 = Oracle(np.float32)


def _scene(n=160, seed=31, n_cams=2, W=48, H=40):
    sc = scenes.scene_tiny(n, seed=seed, log_scale_mean=-2.2)
    cams = scenes.cams_tiny(W=W, H=H, f=50.0, n_cams=n_cams, seed=seed)
    return sc, cams


def _fwd(o, P, sc, cams):
    return o.forward(P, sc, cams)


@pytest.mark.parametrize("o", [O32, O64], ids=["f32", "f64"])
def test_channels_are_independent_and_extend_rgb(o):
    """Channel d of a D = 5 render equals a D = 1 render of that channel
    alone, bit for bit; the projected colours as the first three channels
    reproduce the RGB render; the colour gradient of each channel is that of
    its D = 1 backward."""
    P = OracleParams()
    sc, cams = _scene()
    proj, isect, ras = _fwd(o, P, sc, cams)
    C, N = proj["radii"].shape
    g = np.random.default_rng(3)
    extra = g.uniform(-1.0, 2.0, (C, N, 2)).astype(np.float32)
    feats = np.concatenate([proj["colors"], extra], axis=-1)
    args = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"])
    f5 = o.channels_fwd(*args, features=feats)
    np.testing.assert_array_equal(f5["image"][:, :3], ras["image"])
    np.testing.assert_array_equal(f5["final_T"], ras["final_T"])
    npix = f5["image"].shape[0]
    v = g.normal(size=(npix, 5))
    g5 = o.channels_bwd(*args, f5, v, features=feats)
    geo = {k: np.zeros_like(g5[k], dtype=np.float64) for k in ("v_means2d", "v_conics", "v_opacities")}
    for d in range(5):
        f1 = o.channels_fwd(*args, features=np.ascontiguousarray(feats[..., d:d + 1]))
        np.testing.assert_array_equal(f1["image"][:, 0], f5["image"][:, d])
        g1 = o.channels_bwd(*args, f1, v[:, d:d + 1], features=np.ascontiguousarray(feats[..., d:d + 1]))
        np.testing.assert_array_equal(g1["v_colors"][..., 0], g5["v_colors"][..., d])
        for k in geo:
            geo[k] += g1[k]
    # the geometry gradients are linear in the upstream gradient: the five
    # single-channel backwards sum to the five-channel one
    tol = 1e-11 if o is O64 else 2e-4
    for k, s in geo.items():
        scale = np.abs(g5[k]).max()
        assert np.abs(s - g5[k]).max() <= tol * scale, k


def test_shared_features_equal_their_per_camera_copies():
    P = OracleParams()
    sc, cams = _scene(n_cams=3)
    proj, isect, ras = _fwd(O64, P, sc, cams)
    C, N = proj["radii"].shape
    g = np.random.default_rng(5)
    f_shared = g.uniform(0.0, 1.0, (N, 4))
    f_cam = np.broadcast_to(f_shared, (C, N, 4)).copy()
    args = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"])
    a = O64.channels_fwd(*args, features=f_shared, depth="accumulated")
    b = O64.channels_fwd(*args, features=f_cam, depth="accumulated")
    np.testing.assert_array_equal(a["image"], b["image"])
    v = g.normal(size=a["image"].shape)
    ga = O64.channels_bwd(*args, a, v, features=f_shared, depth="accumulated")
    gb = O64.channels_bwd(*args, b, v, features=f_cam, depth="accumulated")
    assert ga["v_colors"].shape == (N, 4) and gb["v_colors"].shape == (C, N, 4)
    np.testing.assert_allclose(ga["v_colors"], gb["v_colors"].sum(axis=0), rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(ga["v_depths"], gb["v_depths"])


def _pixel_centre_cam(W=32, H=32, f=40.0, x0=16, y0=16):
    return simple_cam(W, H, f, cx=x0 + 0.5, cy=y0 + 0.5)


def test_depth_closed_forms_two_gaussians():
    """Two Gaussians on the pixel centre at z1 < z2: accumulated depth
    z1 a1 + z2 a2 (1 - a1), expected depth that over a1 + a2 (1 - a1); zero
    where nothing is composited."""
    P = OracleParams()
    s1 = one_gaussian_scene((0.0, 0.0, 2.0), scale=(0.05,) * 3, opacity=0.6)
    s2 = one_gaussian_scene((0.0, 0.0, 3.0), scale=(0.05,) * 3, opacity=0.7)
    sc = stack_scenes(s2, s1)
    cam = _pixel_centre_cam()
    proj, isect, ras = O64.forward(P, sc, cam)
    args = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cam["W"], cam["H"])
    z2, z1 = proj["depths"][0]
    assert (z1, z2) == (2.0, 3.0)
    a1, a2 = float(np.float32(0.6)), float(np.float32(0.7))
    p = 16 * 32 + 16
    acc = O64.channels_fwd(*args, features=np.zeros((2, 0)), depth="accumulated")
    exp = O64.channels_fwd(*args, features=np.zeros((2, 0)), depth="expected")
    A = z1 * a1 + z2 * a2 * (1 - a1)
    np.testing.assert_allclose(acc["image"][p, 0], A, rtol=1e-12)
    np.testing.assert_allclose(exp["image"][p, 0], A / (a1 + a2 * (1 - a1)), rtol=1e-12)
    far = 0                                               # corner pixel: nothing composited
    assert acc["image"][far, 0] == 0.0 and exp["image"][far, 0] == 0.0 and exp["weight"][far] == 0.0
    # one Gaussian: expected depth is its depth wherever it is composited
    one = O64.forward(P, s1, cam)
    e1 = O64.channels_fwd(P, one[0], s1["opacities"], one[1]["ranges"], one[1]["ids"], cam["W"], cam["H"],
                          features=np.zeros((1, 0)), depth="expected")
    lit = one[2]["last_ids"] >= 0
    assert lit.sum() > 4
    np.testing.assert_allclose(e1["image"][lit, 0], 2.0, rtol=1e-13)
    # with colours: the feature channels are unchanged, depth comes last
    rgbd = O64.channels_fwd(*args, depth="expected")
    np.testing.assert_array_equal(rgbd["image"][:, :3], ras["image"])
    np.testing.assert_array_equal(rgbd["image"][:, 3], exp["image"][:, 0])
    # the background fills the feature channels only: depth has none
    bg = O64.channels_fwd(*args, depth="accumulated", background=[0.2, 0.3, 0.4])
    np.testing.assert_array_equal(bg["image"][far], [0.2, 0.3, 0.4, 0.0])
    np.testing.assert_allclose(bg["image"][p, 3], A, rtol=1e-12)


@pytest.mark.parametrize("o", [O32, O64], ids=["f32", "f64"])
def test_weight_is_one_minus_final_transmittance(o):
    """sum_k alpha_k T_k telescopes to 1 - T_final."""
    P = OracleParams()
    sc, cams = _scene(n=220, seed=8)
    proj, isect, ras = _fwd(o, P, sc, cams)
    out = o.channels_fwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"],
                         depth="expected")
    tol = 1e-12 if o is O64 else 3e-6
    np.testing.assert_allclose(out["weight"], 1.0 - ras["final_T"], atol=tol)


@pytest.mark.parametrize("depth", ["accumulated", "expected"])
def test_channel_gradients_by_central_differences(depth):
    """L = sum v_image image + sum v_alpha alpha over D = 2 features plus
    depth, differentiated by central differences in float64 for a fixed
    sorted list, against channels_bwd: 2D means, conics, opacities, depths
    and features.  Thresholds are moved out of the way (alpha_min, T_min
    tiny) so the loss is smooth."""
    P = OracleParams(alpha_min=1e-30, T_min=1e-30)
    sc, cams = _scene(n=40, seed=12, n_cams=1, W=32, H=32)
    sc["opacities"] = np.clip(sc["opacities"], 0.05, 0.9).astype(np.float32)
    proj, isect, ras = O64.forward(P, sc, cams)
    C, N = proj["radii"].shape
    g = np.random.default_rng(9)
    feats = g.uniform(-1.0, 1.0, (N, 2))
    ids, ranges = isect["ids"], isect["ranges"]
    opac = np.asarray(sc["opacities"], np.float64)

    def render(pr, op, ft):
        return O64.channels_fwd(P, pr, op, ranges, ids, cams["W"], cams["H"], features=ft, depth=depth)

    base = render(proj, opac, feats)
    v_img = g.normal(size=base["image"].shape)
    v_alpha = g.normal(size=base["alpha"].shape)
    an = O64.channels_bwd(P, proj, opac, ranges, ids, cams["W"], cams["H"], base, v_img, v_alpha, features=feats,
                          depth=depth)

    def loss(pr, op, ft):
        out = render(pr, op, ft)
        return float(np.sum(v_img * out["image"]) + np.sum(v_alpha * out["alpha"]))

    live = np.flatnonzero(proj["radii"][0] > 0)
    checked = 0
    h = 1e-6
    for n in live[:12]:
        for key, idx, grad in (("means2d", (0, n, 0), an["v_means2d"][0, n, 0]),
                               ("means2d", (0, n, 1), an["v_means2d"][0, n, 1]),
                               ("conics", (0, n, 1), an["v_conics"][0, n, 1]),
                               ("depths", (0, n), an["v_depths"][0, n]),
                               ("opac", (n,), an["v_opacities"][0, n]),
                               ("feat", (n, 1), an["v_colors"][n, 1])):
            def at(s):
                pr = {k: (np.array(v, np.float64) if k != "radii" else v) for k, v in proj.items()}
                op, ft = opac.copy(), feats.copy()
                if key == "opac":
                    op[idx] += s
                elif key == "feat":
                    ft[idx] += s
                else:
                    pr[key][idx] += s
                return loss(pr, op, ft)
            fd = (at(h) - at(-h)) / (2 * h)
            assert abs(fd - grad) <= 1e-6 * max(1.0, abs(fd)), (key, n, fd, grad)
            checked += 1
    assert checked >= 36
