"""Pins of the oracle's binning, sort and compositing stages (no GPU).

Rasterization of Gaussians (tile binning, per-tile depth order, front-to-back
compositing), Depth Compositing Gradients; the Figure 1 example.
"""
import json
import os

import numpy as np
import pytest

from oracle import Oracle, OracleParams, camera_layout
from oracle import defs
from paper_2409_06765_amd import scenes
from _util import all_tiles, float_bits, one_gaussian_scene, simple_cam, stack_scenes

O64 = Oracle(np.float64)
O32 = Oracle(np.float32)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _render(o, P, sc, cam, background=None):
    proj, isect, ras = o.forward(P, sc, cam, background=background)
    return proj, isect, ras


# ---------------------------------------------------------------- Figure 1
@pytest.mark.parametrize("o", [O32, O64], ids=["f32", "f64"])
def test_figure1_example(o):
    fx = json.load(open(os.path.join(GOLDEN, "fig1_example.json")))
    i, e = fx["inputs"], fx["expected"]
    sc = one_gaussian_scene(i["mean"], i["quat"], i["scale"], i["opacity"], i["color"])
    cam = dict(viewmats=np.array([i["viewmat"]], np.float32), Ks=np.array([i["K"]], np.float32),
               W=np.array([i["width"]], np.int32), H=np.array([i["height"]], np.int32))
    P = OracleParams()
    proj, isect, ras = _render(o, P, sc, cam)
    np.testing.assert_array_equal(proj["means2d"][0, 0], e["mean2d"])
    assert proj["radii"][0, 0] == e["radius"]
    np.testing.assert_allclose(proj["conics"][0, 0], [1 / e["cov2d_dilated_diag"], 0, 1 / e["cov2d_dilated_diag"]],
                               rtol=1e-6)
    W, H = i["width"], i["height"]
    img = ras["image"].reshape(H, W, 3)
    alpha = ras["alpha"].reshape(H, W)
    for x, y in e["center_pixels"]:
        np.testing.assert_allclose(img[y, x], e["center_rgb"], rtol=1e-6)
        np.testing.assert_allclose(alpha[y, x], e["center_alpha"], rtol=1e-6)
    for x, y in e["black_pixels"]:
        assert np.all(img[y, x] == 0) and alpha[y, x] == 0
    # four-fold mirror symmetry about (120, 120), exactly
    np.testing.assert_array_equal(img, img[:, ::-1])
    np.testing.assert_array_equal(img, img[::-1, :])
    # lit region: a disc of radius ~166.4 px around the pixel corner (120, 120)
    ys, xs = np.mgrid[0:H, 0:W]
    rho = np.hypot(xs + 0.5 - 120, ys + 0.5 - 120)
    lit = alpha > 0
    assert np.all(lit[rho < e["lit_radius_px"] - 0.5]) and not np.any(lit[rho > e["lit_radius_px"] + 0.5])


# ---------------------------------------------------------------- closed forms
def _pixel_centre_cam(W=32, H=32, f=40.0, x0=16, y0=16):
    return simple_cam(W, H, f, cx=x0 + 0.5, cy=y0 + 0.5)


@pytest.mark.parametrize("op", [0.3, 0.99, 1.0, 0.5])
def test_alpha_at_the_mean(op):
    """A mean on a pixel centre gives alpha = min(0.99, o) there."""
    sc = one_gaussian_scene((0.0, 0.0, 2.0), scale=(0.05, 0.05, 0.05), opacity=op, color=(0.25, 0.5, 1.0))
    proj, isect, ras = _render(O32, OracleParams(), sc, _pixel_centre_cam())
    a = np.float32(min(0.99, np.float32(op)))
    p = 16 * 32 + 16
    np.testing.assert_array_equal(ras["image"][p], np.array([0.25, 0.5, 1.0], np.float32) * a)
    assert ras["final_T"][p] == np.float32(1) - a
    assert ras["last_ids"][p] == isect["ranges"][3, 0]       # tile (1, 1) of the 2 x 2 grid


def test_two_gaussians_over_operator():
    c1, c2 = (0.9, 0.1, 0.3), (0.2, 0.8, 0.5)
    s1 = one_gaussian_scene((0.0, 0.0, 2.0), scale=(0.05,) * 3, opacity=0.6, color=c1)
    s2 = one_gaussian_scene((0.0, 0.0, 3.0), scale=(0.05,) * 3, opacity=0.7, color=c2)
    sc = stack_scenes(s2, s1)              # back one first: order must come from depth
    proj, isect, ras = _render(O64, OracleParams(), sc, _pixel_centre_cam())
    p = 16 * 32 + 16
    a1, a2 = float(np.float32(0.6)), float(np.float32(0.7))
    c1, c2 = np.float32(c1).astype(np.float64), np.float32(c2).astype(np.float64)
    expect = c1 * a1 + c2 * a2 * (1 - a1)
    np.testing.assert_allclose(ras["image"][p], expect, rtol=1e-12)
    np.testing.assert_allclose(ras["final_T"][p], (1 - a1) * (1 - a2), rtol=1e-12)


@pytest.mark.parametrize("o", [O32, O64], ids=["f32", "f64"])
def test_weights_plus_final_transmittance_is_one(o):
    sc = scenes.scene_tiny(150, seed=21, log_scale_mean=-2.0)
    sc["sh"] = np.ones_like(sc["sh"])              # colour 1: the image is the sum of weights
    cam = scenes.cams_tiny(W=80, H=64, f=60.0)
    proj, isect, ras = _render(o, OracleParams(), sc, cam)
    tol = 1e-12 if o is O64 else 2e-6
    np.testing.assert_allclose(ras["image"][:, 0] + ras["final_T"], 1.0, atol=tol)
    assert np.all(ras["final_T"] >= np.float32(1e-4))
    np.testing.assert_array_equal(ras["alpha"], o.dtype.type(1) - ras["final_T"])
    assert (ras["final_T"] < 0.05).mean() > 0.05         # the scene is dense enough to stop pixels


def test_stop_rule_keeps_only_the_first_of_stacked_opaque_gaussians():
    """o = 0.99 stacked at a pixel centre: T' after the second would be
    (1 - 0.99f)^2 = 9.99998e-5 < 1e-4, so exactly one is composited."""
    layers = [one_gaussian_scene((0.0, 0.0, 2.0 + 0.1 * k), scale=(0.05,) * 3, opacity=0.99,
                                 color=(0.3, 0.6, 0.9)) for k in range(4)]
    sc = stack_scenes(*layers)
    proj, isect, ras = _render(O32, OracleParams(), sc, _pixel_centre_cam())
    p = 16 * 32 + 16
    a = np.float32(0.99)
    np.testing.assert_array_equal(ras["image"][p], np.array((0.3, 0.6, 0.9), np.float32) * a)
    assert ras["final_T"][p] == np.float32(1) - a
    start = isect["ranges"][3, 0]
    assert ras["last_ids"][p] == start and isect["ids"][start] == 0
    assert ras["n_eval"][p] == 2        # the second one is evaluated and stops the pixel


def test_skip_rule_straddles_one_over_255():
    for op, kept in ((0.0039, False), (0.0040, True)):
        sc = one_gaussian_scene((0.0, 0.0, 2.0), scale=(0.05,) * 3, opacity=op)
        proj, isect, ras = _render(O32, OracleParams(), sc, _pixel_centre_cam())
        p = 16 * 32 + 16
        assert (ras["last_ids"][p] >= 0) == kept
        assert (ras["alpha"][p] > 0) == kept


# ---------------------------------------------------------------- binning and sort
def test_tile_counts_by_brute_force_box_overlap():
    P = OracleParams()
    sc = scenes.scene_tiny(200, seed=31, log_scale_mean=-2.2, spread=1.5)
    cam = scenes.cams_tiny(W=93, H=70, f=60.0, n_cams=3, seed=31)
    proj = O64.project(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], cam["viewmats"],
                       cam["Ks"], cam["W"], cam["H"])
    isect = O64.intersect(P, proj, cam["W"], cam["H"])
    C, N = proj["radii"].shape
    for c in range(C):
        TX, TY = -(-int(cam["W"][c]) // 16), -(-int(cam["H"][c]) // 16)
        kx, ky = np.arange(TX), np.arange(TY)
        for n in range(N):
            r = proj["radii"][c, n]
            if r == 0:
                assert isect["counts"][c, n] == 0
                continue
            mx, my = proj["means2d"][c, n]
            ox = (16 * kx <= mx + r) & (16 * kx + 16 > mx - r)
            oy = (16 * ky <= my + r) & (16 * ky + 16 > my - r)
            assert isect["counts"][c, n] == ox.sum() * oy.sum()
    assert isect["M"] == isect["counts"].sum()
    np.testing.assert_array_equal(isect["offsets"].reshape(-1),
                                  np.concatenate([[0], np.cumsum(isect["counts"].reshape(-1))[:-1]]))


def test_sorted_ids_equal_lexsort_of_tile_depth_id():
    P = OracleParams()
    sc = scenes.scene_tiny(300, seed=32, log_scale_mean=-2.2, spread=1.5)
    cam = scenes.cams_tiny(W=100, H=77, f=60.0, n_cams=2, seed=32)
    proj = O32.project(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], cam["viewmats"],
                       cam["Ks"], cam["W"], cam["H"])
    isect = O32.intersect(P, proj, cam["W"], cam["H"])
    ke, ie = isect["keys_emitted"], isect["ids_emitted"]
    tile = (ke >> np.uint64(32)).astype(np.int64)
    dbits = (ke & np.uint64(0xFFFFFFFF)).astype(np.int64)
    np.testing.assert_array_equal(dbits, float_bits(proj["depths"].reshape(-1)[ie]))
    order = np.lexsort((ie, dbits, tile))
    np.testing.assert_array_equal(isect["ids"], ie[order])
    np.testing.assert_array_equal(isect["keys"], ke[order])
    # ranges: every tile's run is exactly the entries with that tile id
    _, tile_off, _, _ = camera_layout(cam["W"], cam["H"])
    st = (isect["keys"] >> np.uint64(32)).astype(np.int64)
    for t in range(int(tile_off[-1])):
        idx = np.nonzero(st == t)[0]
        if idx.size == 0:
            assert tuple(isect["ranges"][t]) == (0, 0)
        else:
            assert tuple(isect["ranges"][t]) == (idx[0], idx[-1] + 1)


# ---------------------------------------------------------------- tiled == untiled
@pytest.mark.parametrize("deg", [-1, 3])
def test_tiled_equals_definition_equals_numpy(deg):
    P = OracleParams(sh_degree=deg)
    sc = scenes.scene_tiny(120, sh_degree=deg, seed=41, log_scale_mean=-2.0)
    cam = scenes.cams_tiny(W=70, H=50, f=55.0, n_cams=2, seed=41)
    bg = np.array([[0.1, 0.2, 0.3], [0.0, 0.5, 1.0]])
    proj, isect, ras = O64.forward(P, sc, cam, background=bg)
    tiles = all_tiles(cam["W"], cam["H"])
    dfn = O64.render_tiles_fwd(P, proj, sc["opacities"], tiles, cam["W"], cam["H"], background=bg)
    np.testing.assert_array_equal(ras["image"], dfn["image"])
    np.testing.assert_array_equal(ras["final_T"], dfn["final_T"])
    lid = ras["last_ids"]
    np.testing.assert_array_equal(np.where(lid >= 0, isect["ids"][np.maximum(lid, 0)], -1), dfn["last_gid"])
    npix = 70 * 50
    for c in range(2):
        d = defs.project(P, sc["means"], sc["quats"], sc["scales"], sc["sh"], cam["viewmats"][c], cam["Ks"][c],
                         70, 50)
        ref = defs.render(P, d, sc["opacities"].astype(np.float64), 70, 50, background=bg[c], mode="rect")
        img = ras["image"][c * npix:(c + 1) * npix].reshape(50, 70, 3)
        np.testing.assert_allclose(img, ref["image"], atol=1e-10)
        gid = dfn["last_gid"][c * npix:(c + 1) * npix].reshape(50, 70)
        np.testing.assert_array_equal(np.where(gid >= 0, gid - c * sc["means"].shape[0], -1), ref["last"])


def test_fully_untiled_equals_tiled_when_opacity_below_bound():
    """Outside the 3-sigma square box sigma >= 4.5, so alpha < 1/255 there
    whenever o < 255^-1 e^4.5 = 0.35301: dropping the tile test changes nothing."""
    P = OracleParams()
    sc = scenes.scene_tiny(150, seed=42, log_scale_mean=-2.0)
    sc["opacities"] = (sc["opacities"] * 0.35).astype(np.float32)
    cam = scenes.cams_tiny(W=64, H=64, f=55.0)
    proj, isect, ras = O64.forward(P, sc, cam)
    ref = defs.render(P, defs.project(P, sc["means"], sc["quats"], sc["scales"], sc["sh"], cam["viewmats"][0],
                                      cam["Ks"][0], 64, 64), sc["opacities"].astype(np.float64), 64, 64,
                      mode="untiled")
    np.testing.assert_allclose(ras["image"].reshape(64, 64, 3), ref["image"], atol=1e-10)
    un = O64.render_tiles_fwd(P, proj, sc["opacities"], all_tiles(64, 64), 64, 64, untiled=True)
    np.testing.assert_allclose(un["image"], ras["image"], atol=1e-12)
    # and with opaque Gaussians the untiled render really does differ
    sc2 = dict(sc)
    sc2["opacities"] = np.full_like(sc["opacities"], 0.99)
    proj2, _, ras2 = O64.forward(P, sc2, cam)
    un2 = O64.render_tiles_fwd(P, proj2, sc2["opacities"], all_tiles(64, 64), 64, 64, untiled=True)
    assert np.abs(un2["image"] - ras2["image"]).max() > 1e-6


def test_empty_scene_and_ragged_image():
    P = OracleParams()
    sc = scenes.scene_tiny(0)
    cam = scenes.cams_tiny(W=37, H=19)
    proj, isect, ras = O32.forward(P, sc, cam, background=np.array([[0.2, 0.3, 0.4]]))
    assert isect["M"] == 0
    np.testing.assert_array_equal(ras["final_T"], 1.0)
    np.testing.assert_array_equal(ras["last_ids"], -1)
    np.testing.assert_allclose(ras["image"], np.tile(np.float32([0.2, 0.3, 0.4]), (37 * 19, 1)))


# ---------------------------------------------------------------- single-Gaussian gradients
def test_single_gaussian_gradients_closed_form():
    """T = 1: dC/dc = alpha, dC/do = c e^-sigma (0 when clamped),
    dC/dmu' = -c o e^-sigma Sigma'^-1 (mu' - p)."""
    P = OracleParams()
    for op in (0.6, 0.999):
        sc = one_gaussian_scene((0.013, -0.021, 2.0), quat=(0.9, 0.1, -0.2, 0.3), scale=(0.08, 0.05, 0.03),
                                opacity=op, color=(0.3, 0.7, 0.2))
        cam = _pixel_centre_cam()
        proj, isect, ras = O64.forward(P, sc, cam)
        x, y, ch = 17, 15, 1
        p = y * 32 + x
        v_image = np.zeros((32 * 32, 3))
        v_image[p, ch] = 1.0
        g = O64.rasterize_bwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cam["W"], cam["H"],
                              ras["final_T"], ras["last_ids"], v_image)
        mx, my = proj["means2d"][0, 0]
        a, b, c = proj["conics"][0, 0]
        dx, dy = mx - (x + 0.5), my - (y + 0.5)
        sig = 0.5 * (a * dx * dx + c * dy * dy) + b * dx * dy
        o = float(sc["opacities"][0])
        e = np.exp(-sig)
        alpha = min(float(np.float32(0.99)), o * e)
        col = float(sc["sh"][0, ch])
        assert ras["last_ids"][p] >= 0
        np.testing.assert_allclose(g["v_colors"][0, 0], [0, alpha, 0][:3], rtol=1e-12, atol=1e-15)
        clamped = o * e > float(np.float32(0.99))
        np.testing.assert_allclose(g["v_opacities"][0, 0], 0.0 if clamped else col * e, rtol=1e-12, atol=1e-15)
        vm = np.zeros(2) if clamped else -col * o * e * np.array([a * dx + b * dy, b * dx + c * dy])
        np.testing.assert_allclose(g["v_means2d"][0, 0], vm, rtol=1e-10, atol=1e-15)
        vc = np.zeros(3) if clamped else -col * o * e * np.array([0.5 * dx * dx, dx * dy, 0.5 * dy * dy])
        np.testing.assert_allclose(g["v_conics"][0, 0], vc, rtol=1e-10, atol=1e-15)


def test_two_gaussian_alpha_gradients():
    """C = c1 a1 + c2 a2 (1 - a1): dC/da1 = c1 - c2 a2, dC/da2 = c2 (1 - a1)."""
    P = OracleParams()
    c1, c2 = (0.9, 0.1, 0.3), (0.2, 0.8, 0.5)
    s1 = one_gaussian_scene((0.0, 0.0, 2.0), scale=(0.05,) * 3, opacity=0.6, color=c1)
    s2 = one_gaussian_scene((0.0, 0.0, 3.0), scale=(0.05,) * 3, opacity=0.7, color=c2)
    sc = stack_scenes(s1, s2)
    cam = _pixel_centre_cam()
    proj, isect, ras = O64.forward(P, sc, cam)
    p = 16 * 32 + 16
    v_image = np.zeros((32 * 32, 3))
    v_image[p] = [1.0, -2.0, 0.5]
    g = O64.rasterize_bwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cam["W"], cam["H"],
                          ras["final_T"], ras["last_ids"], v_image)
    a1, a2 = float(np.float32(0.6)), float(np.float32(0.7))
    c1, c2 = np.float32(c1).astype(float), np.float32(c2).astype(float)
    # at the mean e^-sigma = 1, so dC/do = dC/dalpha
    np.testing.assert_allclose(g["v_opacities"][0, 0], np.dot(c1 - c2 * a2, v_image[p]), rtol=1e-12)
    np.testing.assert_allclose(g["v_opacities"][0, 1], np.dot(c2 * (1 - a1), v_image[p]), rtol=1e-12)


def test_absolute_term_sums_bound_and_match_single_signed_terms():
    """The per-element term magnitudes that the gradient tolerance uses: they
    bound |gradient|, equal it when every term has one sign and no parts to
    cancel (colour gradient under a non-negative upstream gradient: alpha T
    v_C >= 0), are linear in the upstream gradients, and leave the gradients
    themselves unchanged."""
    P = OracleParams(sh_degree=1)
    sc = scenes.scene_tiny(150, sh_degree=1, seed=41, log_scale_mean=-2.4)
    cams = scenes.cams_tiny(W=48, H=40, f=50.0, n_cams=2, seed=41)
    proj, isect, ras = O64.forward(P, sc, cams)
    v_image, v_alpha = scenes.upstream_grads("tiny", ras["final_T"].shape[0], seed=42, with_alpha=True)
    args = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"], ras["final_T"],
            ras["last_ids"])
    plain = O64.rasterize_bwd(*args, v_image, v_alpha)
    g = O64.rasterize_bwd(*args, v_image, v_alpha, abs_sums=True)
    for k in ("v_means2d", "v_conics", "v_colors", "v_opacities"):
        np.testing.assert_array_equal(g[k], plain[k])
        assert (g["abs_" + k] >= np.abs(g[k]) * (1 - 1e-12)).all(), k
    assert g["abs_v_means2d"].max() > 0 and g["abs_v_opacities"].max() > 0
    pos = O64.rasterize_bwd(*args, np.abs(v_image), None, abs_sums=True)
    np.testing.assert_allclose(pos["abs_v_colors"], pos["v_colors"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(pos["abs_v_colors"], g["abs_v_colors"], rtol=1e-12, atol=1e-300)
    two = O64.rasterize_bwd(*args, 2 * v_image, 2 * v_alpha, abs_sums=True)
    for k in ("v_means2d", "v_conics", "v_colors", "v_opacities"):
        np.testing.assert_allclose(two["abs_" + k], 2 * g["abs_" + k], rtol=1e-12, atol=1e-300)


def test_absgrad_is_the_sum_of_per_pixel_absolute_mean_gradients():
    """Absgrad: per Gaussian, the sum over pixels of |dL_p/dmu'| (each pixel's
    own contribution, x and y apart), checked by brute force: one backward
    per pixel with that pixel's upstream gradient alone, absolute values
    summed.  It bounds the signed gradient and equals it where every
    contribution has one sign."""
    P = OracleParams(sh_degree=1, antialiased=1)
    sc = scenes.scene_tiny(40, sh_degree=1, seed=51, log_scale_mean=-2.0)
    cams = scenes.cams_tiny(W=22, H=17, f=18.0, n_cams=2, seed=51)
    proj, isect, ras = O64.forward(P, sc, cams)
    npix = ras["final_T"].shape[0]
    v_image, v_alpha = scenes.upstream_grads("tiny", npix, seed=52, with_alpha=True)
    args = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"], ras["final_T"],
            ras["last_ids"])
    full = O64.rasterize_bwd(*args, v_image, v_alpha, absgrad=True)
    brute = np.zeros_like(full["v_means2d"])
    for p in range(npix):
        vi = np.zeros_like(v_image)
        va = np.zeros_like(v_alpha)
        vi[p], va[p] = v_image[p], v_alpha[p]
        brute += np.abs(O64.rasterize_bwd(*args, vi, va)["v_means2d"])
    np.testing.assert_allclose(full["v_means2d_abs"], brute, rtol=1e-12, atol=1e-14)
    assert (full["v_means2d_abs"] >= np.abs(full["v_means2d"]) - 1e-12).all()
    assert full["v_means2d_abs"].max() > 0
    # one pixel alone: absgrad is the absolute signed gradient
    vi = np.zeros_like(v_image)
    p = int(np.argmax(ras["last_ids"] >= 0))
    vi[p] = v_image[p]
    one = O64.rasterize_bwd(*args, vi, None, absgrad=True)
    np.testing.assert_allclose(one["v_means2d_abs"], np.abs(one["v_means2d"]), rtol=1e-12, atol=1e-300)
