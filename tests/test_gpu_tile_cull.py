"""Culled binning (params tile_cull = 1) on the GPU.

Lists: every tile's culled list is a sub-list, in the same order, of the
oracle's 3-sigma-square list; it holds every entry that a pixel centre of the
tile sees at alpha >= alpha_min (oracle/tiles.py, float64 brute force, with
alpha_min lowered by 1e-4 so entries at the threshold count as seen); and it
is not much longer than the exact continuous-rectangle set.  Outputs:
compositing the culled lists gives the forward of whole squares bit for bit
(image, alpha, final T, composited counts, and the Gaussian each pixel
composited last) and the same gradients up to the atomics' rounding order.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from oracle import tiles
from paper_2409_06765_amd import scenes

pytestmark = pytest.mark.gpu

O32 = Oracle(np.float32)


def _say(msg):
    print(f"[gpu-tile-cull] {msg}", flush=True)


CASES = {
    "tiny_direct_3cams_ragged": (lambda: scenes.scene_tiny(300, seed=1, log_scale_mean=-2.3, spread=1.2),
                                 lambda: scenes.cameras(
                                     [scenes.look_at(e) for e in ([0, 0, 4.0], [3.0, 1.0, 2.5], [-1.0, 3.5, 1.0])],
                                     [scenes.intrinsics(f, w, h) for f, w, h in ((90, 100, 75), (60, 64, 64), (25, 33, 17))],
                                     [100, 64, 33], [75, 64, 17]), -1, False),
    "tiny_sh3_aa": (lambda: scenes.scene_tiny(400, sh_degree=3, seed=2, log_scale_mean=-2.5),
                    lambda: scenes.cams_tiny(W=97, H=61, f=70.0, n_cams=2, seed=2), 3, True),
    "uniform10k_256": (scenes.scene_uniform10k_256, scenes.cams_uniform10k_256, -1, False),
    "uniform100k_sh3_800": (scenes.scene_uniform100k_sh3_800, scenes.cams_uniform100k_sh3_800, 3, False),
}


@pytest.mark.parametrize("name", list(CASES))
def test_culled_lists_are_filtered_square_lists(name):
    from _gpu import gpu_forward, np_, params
    scene_f, cams_f, deg, aa = CASES[name]
    sc, cams = scene_f(), cams_f()
    P = OracleParams(sh_degree=deg, antialiased=int(aa))
    st = gpu_forward(params(sh_degree=deg, antialiased=aa, tile_cull=1), sc, cams)
    proj = O32.project(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], cams["viewmats"],
                       cams["Ks"], cams["W"], cams["H"])
    box = O32.intersect(P, proj, cams["W"], cams["H"])
    T = len(box["ranges"])
    g_ranges = np_(st["isect"]["ranges"])[:T].astype(np.int64)
    g_ids = np_(st["isect"]["ids"]).astype(np.int64)
    sup = tiles.tile_support(P, proj, sc["opacities"], box["ranges"], box["ids"], cams["W"], cams["H"])
    # position of each (tile, id) in the square lists
    key = sup["tile"] * (1 << 32) + sup["gid"]
    order = np.argsort(key)
    g_tile = np.repeat(np.arange(T), g_ranges[:, 1] - g_ranges[:, 0])
    g_key = g_tile * (1 << 32) + g_ids[np.concatenate([np.arange(s, e) for s, e in g_ranges])
                                       if len(g_tile) else np.zeros(0, np.int64)]
    k = np.searchsorted(key[order], g_key)
    assert np.all(k < len(key)) and np.all(key[order][np.minimum(k, len(key) - 1)] == g_key), "entry not in a square"
    g_pos = sup["pos"][order][k]
    # same order as the square lists inside every tile
    same_tile = g_tile[1:] == g_tile[:-1]
    assert np.all(np.diff(g_pos)[same_tile] > 0)
    # every entry a pixel centre sees is kept
    seen = sup["max_alpha_centres"] >= P.alpha_min * (1 - 1e-4)
    kept = np.zeros(len(key), bool)
    kept[sup["pos"].searchsorted(g_pos)] = True      # sup["pos"] is increasing
    assert np.all(kept[seen]), f"{int((seen & ~kept).sum())} seen entries dropped"
    exact = int((sup["min_sigma"] <= sup["threshold"]).sum())
    _say(f"{name}: square M={box['M']} culled M={len(g_key)} exact rectangle set={exact} seen={int(seen.sum())}")
    assert len(g_key) <= 1.02 * exact + 16
    assert len(g_key) < box["M"]


def _equal_outputs(st0, st1, v_image, rtol=1e-3):
    from _gpu import assert_grad_close, np_, to_dev
    from paper_2409_06765_amd import rasterize as R
    f0, f1 = st0["fwd"], st1["fwd"]
    for k in ("image", "alpha", "final_T"):
        np.testing.assert_array_equal(np_(f0[k]), np_(f1[k]), err_msg=k)
    np.testing.assert_array_equal(np_(f0["n_eval"])[:, 1], np_(f1["n_eval"])[:, 1], err_msg="composited counts")
    l0, l1 = np_(f0["last_ids"]), np_(f1["last_ids"])
    np.testing.assert_array_equal(l0 >= 0, l1 >= 0)
    lit = l0 >= 0
    i0, i1 = np_(st0["isect"]["ids"]), np_(st1["isect"]["ids"])
    np.testing.assert_array_equal(i0[l0[lit]], i1[l1[lit]], err_msg="last composited Gaussian")
    d = st0["d"]
    v = to_dev(v_image)
    g0 = R.rasterize_backward(st0["p"], st0["proj"], d["opacities"], st0["isect"], st0["W"], st0["H"], f0, v)
    g1 = R.rasterize_backward(st1["p"], st1["proj"], d["opacities"], st1["isect"], st1["W"], st1["H"], f1, v)
    for k in ("v_means2d", "v_conics", "v_colors", "v_opacities"):
        assert_grad_close(np_(g1[k]), np_(g0[k]), k, rtol=rtol)


@pytest.mark.parametrize("name", ["tiny_direct_3cams_ragged", "tiny_sh3_aa", "uniform100k_sh3_800"])
def test_culled_lists_composite_like_squares(name):
    from _gpu import gpu_forward, params
    scene_f, cams_f, deg, aa = CASES[name]
    sc, cams = scene_f(), cams_f()
    sts = []
    for cull in (0, 1):
        p = params(sh_degree=deg, antialiased=aa, tile_cull=cull)
        st = gpu_forward(p, sc, cams)
        st["p"] = p
        sts.append(st)
    npix = sts[0]["fwd"]["image"].shape[0]
    v_image, _ = scenes.upstream_grads("tiny", npix, seed=5)
    _equal_outputs(sts[0], sts[1], v_image)


def test_full_size_view_culled_like_squares():
    """1M Gaussians, 1920 x 1080, view 0: the culled lists are well under
    half as long and composite to the same forward, bit for bit."""
    from _gpu import gpu_forward, params
    sc = scenes.scene_clusters1m_sh3_1080p()
    cams = scenes.cams_clusters1m_sh3_1080p()
    one = {k: (v[:1] if isinstance(v, np.ndarray) else v) for k, v in cams.items()}
    sts = []
    for cull in (0, 1):
        p = params(sh_degree=3, tile_cull=cull)
        st = gpu_forward(p, sc, one)
        st["p"] = p
        sts.append(st)
    M0, M1 = sts[0]["isect"]["M"], sts[1]["isect"]["M"]
    _say(f"1M view 0: square M={M0} culled M={M1}")
    assert M1 < 0.5 * M0
    v_image, _ = scenes.upstream_grads("clusters1m_sh3_1080p", sts[0]["fwd"]["image"].shape[0], seed=0)
    _equal_outputs(sts[0], sts[1], v_image)
