"""HIP path against the CPU oracle, element by element, through the C ABI.

Bit-exact: radii, 2D means, depths, conics, tile counts, offsets, M, sorted
keys and ids, tile ranges, last_ids and evaluation counts (outside pixels the
oracle flags as near a skip/stop threshold).  Images within 1e-4 max-abs per
pixel; gradients within 1e-3 relative (tests/_gpu.assert_grad_close).
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes
from _util import wide_cone_scene

pytestmark = pytest.mark.gpu

O32 = Oracle(np.float32)
O64 = Oracle(np.float64)


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


CASES = {
    # name: (scene factory, cameras factory, sh_degree, antialiased, background)
    "tiny_direct_3cams_ragged": (lambda: scenes.scene_tiny(300, seed=1, log_scale_mean=-2.3, spread=1.2),
                                 lambda: scenes.cameras(
                                     [scenes.look_at(e) for e in ([0, 0, 4.0], [3.0, 1.0, 2.5], [-1.0, 3.5, 1.0])],
                                     [scenes.intrinsics(f, w, h) for f, w, h in ((90, 100, 75), (60, 64, 64), (25, 33, 17))],
                                     [100, 64, 33], [75, 64, 17]),
                                 -1, False, [[0.2, 0.3, 0.4], [0.0, 0.0, 0.0], [1.0, 0.5, 0.25]]),
    "tiny_sh3_aa": (lambda: scenes.scene_tiny(400, sh_degree=3, seed=2, log_scale_mean=-2.5),
                    lambda: scenes.cams_tiny(W=97, H=61, f=70.0, n_cams=2, seed=2), 3, True, None),
    "tiny_sh1": (lambda: scenes.scene_tiny(200, sh_degree=1, seed=3, log_scale_mean=-2.0),
                 lambda: scenes.cams_tiny(W=48, H=48, f=40.0, seed=3), 1, False, None),
    # views of 1,024 tiles or more take the one-wave-per-tile RGB backward, fewer the four-wave one
    "ragged_3cams_bg_1065tiles": (lambda: scenes.scene_tiny(1500, seed=4, log_scale_mean=-2.6, spread=1.2),
                                  lambda: scenes.cameras(
                                      [scenes.look_at(e) for e in ([0, 0, 4.0], [3.0, 1.0, 2.5], [-1.0, 3.5, 1.0])],
                                      [scenes.intrinsics(f, w, h) for f, w, h in ((400, 512, 512), (90, 100, 75),
                                                                                  (25, 33, 17))],
                                      [512, 100, 33], [512, 75, 17]),
                                  -1, False, [[0.2, 0.3, 0.4], [0.0, 0.0, 0.0], [1.0, 0.5, 0.25]]),
    "sh3_aa_1050tiles": (lambda: scenes.scene_tiny(1500, sh_degree=3, seed=5, log_scale_mean=-2.7),
                         lambda: scenes.cams_tiny(W=400, H=330, f=300.0, n_cams=2, seed=5), 3, True, None),
    # the paper-literal Jacobian (no clamp of t_x/t_z, t_y/t_z): Gaussians up to twice the depth off axis,
    # where the clamped and literal Jacobians differ
    "wide_cone_sh3_jac_literal": (lambda: wide_cone_scene(500, seed=9),
                                  lambda: scenes.cams_tiny(W=120, H=90, f=60.0, seed=9), 3, False, None,
                                  dict(jac_clamp=0.0)),
    "uniform10k_256": (scenes.scene_uniform10k_256, scenes.cams_uniform10k_256, -1, False, None),
    "uniform100k_sh3_800": (scenes.scene_uniform100k_sh3_800, scenes.cams_uniform100k_sh3_800, 3, False, None),
}


def _run(name):
    scene_f, cams_f, deg, aa, bg = CASES[name][:5]
    extra = CASES[name][5] if len(CASES[name]) > 5 else {}
    sc, cams = scene_f(), cams_f()
    bg = None if bg is None else np.asarray(bg, np.float32)
    P = OracleParams(sh_degree=deg, antialiased=int(aa), **extra)
    from _gpu import gpu_forward, params
    p = params(sh_degree=deg, antialiased=aa, **extra)
    _say(f"{name}: N={sc['means'].shape[0]} cams={len(cams['W'])} sizes={list(zip(cams['W'], cams['H']))}")
    st = gpu_forward(p, sc, cams, background=bg, want_keys=True)
    proj, isect, ras = O32.forward(P, sc, cams, background=bg)
    return sc, cams, bg, P, p, st, proj, isect, ras


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    return (request.param,) + _run(request.param)


def test_projection_bit_exact(case):
    from _gpu import np_
    name, sc, cams, bg, P, p, st, proj, isect, ras = case
    gp = st["proj"]
    np.testing.assert_array_equal(np_(gp["radii"]), proj["radii"], err_msg=name)
    np.testing.assert_array_equal(np_(gp["means2d"]), proj["means2d"], err_msg=name)
    np.testing.assert_array_equal(np_(gp["depths"]), proj["depths"], err_msg=name)
    np.testing.assert_array_equal(np_(gp["conics"]), proj["conics"], err_msg=name)
    np.testing.assert_allclose(np_(gp["colors"]), proj["colors"], rtol=0, atol=2e-6, err_msg=name)
    if P.antialiased:
        np.testing.assert_allclose(np_(gp["comps"]), proj["comps"], rtol=1e-6, atol=0, err_msg=name)
    assert (proj["radii"] > 0).sum() > 0


def test_binning_and_sort_bit_exact(case):
    """The pipeline's binning (depth order, then 32-bit tile keys)."""
    from _gpu import np_
    name, sc, cams, bg, P, p, st, proj, isect, ras = case
    gi = st["isect"]
    assert gi["M"] == isect["M"], name
    np.testing.assert_array_equal(np_(gi["ids"]), isect["ids"])
    np.testing.assert_array_equal(np_(gi["keys"]), isect["keys"])
    np.testing.assert_array_equal(np_(gi["ranges"])[:len(isect["ranges"])], isect["ranges"])


def test_count_emit_sort_ranges_bit_exact(case):
    """The general path: counts, offsets, emitted keys, 64-bit radix sort, ranges."""
    from _gpu import np_, scene_to_dev, to_dev
    from paper_2409_06765_amd import rasterize as R
    name, sc, cams, bg, P, p, st, proj, isect, ras = case
    gi = R.intersect(p, st["proj"], st["W"], st["H"], method="keys64")
    assert gi["M"] == isect["M"], name
    np.testing.assert_array_equal(np_(gi["counts"]), isect["counts"])
    np.testing.assert_array_equal(np_(gi["offsets"]), isect["offsets"])
    np.testing.assert_array_equal(np_(gi["keys"]), isect["keys"])
    np.testing.assert_array_equal(np_(gi["ids"]), isect["ids"])
    np.testing.assert_array_equal(np_(gi["ranges"])[:len(isect["ranges"])], isect["ranges"])


def test_rasterize_forward(case):
    from _gpu import np_
    name, sc, cams, bg, P, p, st, proj, isect, ras = case
    f = st["fwd"]
    ok = ras["flags"] == 0
    frac = 1.0 - ok.mean()
    _say(f"{name}: flagged pixels {int((~ok).sum())} of {ok.size}")
    assert frac < 1e-3, frac
    err = np.abs(np_(f["image"]) - ras["image"]).max(axis=1)
    assert err[ok].max(initial=0) <= 1e-4, (name, err[ok].max())
    assert np.abs(np_(f["final_T"]) - ras["final_T"])[ok].max(initial=0) <= 1e-4
    np.testing.assert_array_equal(np_(f["alpha"])[ok], 1 - np_(f["final_T"])[ok])
    np.testing.assert_array_equal(np_(f["last_ids"])[ok], ras["last_ids"][ok])
    ne = np_(f["n_eval"])
    np.testing.assert_array_equal(ne[ok, 0], ras["n_eval"][ok])
    np.testing.assert_array_equal(ne[ok, 1], ras["n_comp"][ok])


def test_rasterize_backward_and_projection_backward(case):
    from _gpu import assert_grad_close, gpu_backward, np_
    name, sc, cams, bg, P, p, st, proj, isect, ras = case
    npix = ras["final_T"].shape[0]
    v_image, v_alpha = scenes.upstream_grads("tiny", npix, seed=7, with_alpha=True)
    # pixels whose decisions sit on a threshold get no upstream gradient on either side
    v_image[ras["flags"] != 0] = 0
    v_alpha[ras["flags"] != 0] = 0
    g2, g3 = gpu_backward(p, st, v_image, v_alpha, absgrad=True)
    o2 = O32.rasterize_bwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"],
                           ras["final_T"], ras["last_ids"], v_image, v_alpha, background=bg, absgrad=True)
    for k in ("v_means2d", "v_conics", "v_colors", "v_opacities", "v_means2d_abs"):
        assert_grad_close(np_(g2[k]), o2[k], f"{name}:{k}")
    # projection backward: both sides from the same (oracle) upstream gradients
    o3 = O32.project_bwd(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], cams["viewmats"],
                         cams["Ks"], cams["W"], cams["H"], o2["v_means2d"], o2["v_conics"], o2["v_colors"],
                         o2["v_opacities"])
    from _gpu import to_dev
    from paper_2409_06765_amd import rasterize as R
    d = st["d"]
    g2o = {k: to_dev(o2[k]) for k in ("v_means2d", "v_conics", "v_colors", "v_opacities")}
    g3o = R.project_backward(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], st["vm"], st["Ks"],
                             st["W"], st["H"], st["proj"], g2o)
    for k, ko in (("v_means", "v_means"), ("v_quats", "v_quats"), ("v_scales", "v_scales"),
                  ("v_opacities", "v_opacities"), ("v_sh", "v_sh")):
        assert_grad_close(np_(g3o[k]), o3[ko], f"{name}:{k}")
    # end to end: the GPU chain against the float64 oracle chain
    from _gpu import assert_chain_close, oracle_project_bwd
    a = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"])
    r64 = O64.rasterize_fwd(*a, background=bg)
    o2x = O64.rasterize_bwd(*a, r64["final_T"], r64["last_ids"], v_image, v_alpha, background=bg)
    pb32, pb64 = oracle_project_bwd(O32, P, sc, cams), oracle_project_bwd(O64, P, sc, cams)
    assert_chain_close({k: np_(v) for k, v in g3.items() if v is not None},
                       {k: np_(v) for k, v in g2.items() if v is not None}, o2x, pb64(o2x), pb32, pb64, name)


def test_forward_is_deterministic_and_backward_reproducible(case):
    from _gpu import gpu_backward, gpu_forward, np_
    name, sc, cams, bg, P, p, st, proj, isect, ras = case
    st2 = gpu_forward(p, sc, cams, background=bg)
    for k in ("image", "final_T", "last_ids", "n_eval"):
        np.testing.assert_array_equal(np_(st2["fwd"][k]), np_(st["fwd"][k]), err_msg=k)
    npix = ras["final_T"].shape[0]
    v_image, _ = scenes.upstream_grads("tiny", npix, seed=9)
    a2, a3 = gpu_backward(p, st, v_image)
    b2, b3 = gpu_backward(p, st2, v_image)
    # the compositing backward sums with float atomics, in whatever order they land: two runs agree to
    # 1e-6 of the norm; the projection backward has no atomics: the same inputs give the same bits (so
    # its outputs differ between the runs only as far as the compositing gradients carry through it)
    for k in ("v_means2d", "v_conics", "v_colors", "v_opacities"):
        x, y = np_(a2[k]), np_(b2[k])
        assert np.linalg.norm(x - y) <= 1e-6 * max(np.linalg.norm(x), 1e-30), k
    from paper_2409_06765_amd import rasterize as R
    d = st["d"]
    c3 = R.project_backward(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], st["vm"], st["Ks"],
                            st["W"], st["H"], st["proj"], a2)
    for k in ("v_means", "v_quats", "v_scales", "v_opacities", "v_sh"):
        np.testing.assert_array_equal(np_(c3[k]), np_(a3[k]), err_msg=k)
