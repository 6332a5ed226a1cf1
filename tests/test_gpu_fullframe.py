"""Whole-frame parity at the configuration the benchmark times.

Views 0-3 of the 1M-Gaussian, 1920 x 1080 workload go through
pipeline.ViewPipeline as one step, the exact step bench.py times: the four
cameras in one call of every stage, culled tile lists, the forward
compositing without counters, the dispatch order, the one-wave-per-tile RGB
backward and the projection backward (which sums the views' gradients),
every buffer allocated once.  The float32 oracle computes the same views
with the paper's whole 3-sigma tile lists over all 32,640 tiles
(Rasterization of Gaussians; Depth Compositing Gradients; Projection
Gradients), on every host core.  Checked:

* projection bit for bit;
* images and final transmittance within 1e-4, and the last composited
  Gaussian (an id, compared through each side's own list) bit for bit, on
  every pixel the oracle does not flag (flagged share below 1e-3);
* compositing gradients element-wise at 1e-3 relative (plus the float32
  summation scale of each element's terms), the upstream gradient being
  zero on flagged pixels on both sides;
* the projection backward of the GPU's own compositing gradients against
  the float64 oracle's, at 1e-3 relative or within four times the float32
  oracle's distance from it, elementwise; and the projection gradients end
  to end against the float64 oracle chain (double-precision compositing of
  the same float32 projected values, then the double projection backward)
  at 1e-3 relative plus the measured compositing error carried through the
  projection backward (tests/_gpu.py assert_chain_close).

The 3M-Gaussian scene seen from inside is checked the same way on 512
tiles (the 64 with the longest lists and 448 more at random), whose pixels
alone carry an upstream gradient.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes

pytestmark = pytest.mark.gpu
O32 = Oracle(np.float32)
O64 = Oracle(np.float64)


def _say(msg):
    print(f"[gpu-fullframe] {msg}", flush=True)


def _gpu_view(wl, views, v_image):
    """The timed step for the consecutive views ``views`` (one call of every
    stage over their cameras): ViewPipeline with the pipeline's default
    parameters, on the device; returns host copies of everything checked."""
    from _gpu import np_, to_dev
    from paper_2409_06765_amd import rasterize as R
    from paper_2409_06765_amd.pipeline import ViewPipeline
    sc = getattr(scenes, f"scene_{wl}")()
    cams = getattr(scenes, f"cams_{wl}")()
    v0, C = views[0], len(views)
    W, H = [int(w) for w in cams["W"][v0:v0 + C]], [int(h) for h in cams["H"][v0:v0 + C]]
    d = {k: to_dev(x) for k, x in sc.items() if isinstance(x, np.ndarray)}
    vm, Ks = to_dev(cams["viewmats"][v0:v0 + C]), to_dev(cams["Ks"][v0:v0 + C])
    p = R.make_params(sh_degree=3)
    assert p.tile_cull == 1
    # list capacity from an eager count of the same views
    proj = R.project(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, Ks, W, H)
    cap = int(R.intersect(p, proj, W, H)["M"] * 1.1) + 1024
    del proj
    pipe = ViewPipeline(p, d, W, H, cap)
    assert pipe.order is not None, "the dispatch order is part of the timed step"
    pipe.set_cameras(vm, Ks)
    pipe.step(to_dev(v_image))
    torch.cuda.synchronize()
    M = pipe.counts()[0]
    assert M <= cap
    out = dict(sc=sc, cams={k: x[v0:v0 + C] for k, x in cams.items()}, W=W, H=H, M=M,
               proj={k: np_(x) for k, x in pipe.proj.items() if x is not None},
               ids=np_(pipe.ids[:M]), ranges=np_(pipe.ranges),
               image=np_(pipe.image), final_T=np_(pipe.final_T), last_ids=np_(pipe.last_ids),
               g2={k: np_(x) for k, x in pipe.g2.items() if x is not None},
               g3={k: np_(x) for k, x in pipe.g3.items()})
    del pipe, d
    torch.cuda.empty_cache()
    return out


def _last_gid(last_pos, ids):
    return np.where(last_pos >= 0, ids[np.maximum(last_pos, 0)], -1)


def _check_view(wl, choose_tiles=None, flag_bar=1e-3, n_views=1):
    cams_all = getattr(scenes, f"cams_{wl}")()
    W, H = int(cams_all["W"][0]), int(cams_all["H"][0])
    TX, TY = (W + 15) // 16, (H + 15) // 16
    P = OracleParams(sh_degree=3)
    # the oracle's forward first: the upstream gradient is zero on its flagged pixels (and off the checked tiles)
    sc = getattr(scenes, f"scene_{wl}")()
    cams = {k: x[:n_views] for k, x in cams_all.items()}
    assert all(int(w) == W for w in cams["W"]) and all(int(h) == H for h in cams["H"])
    oracle.set_threads(16)
    try:
        _say(f"{wl}: oracle projection and binning (square lists)")
        proj = O32.project(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], cams["viewmats"],
                           cams["Ks"], cams["W"], cams["H"])
        isect = O32.intersect(P, proj, cams["W"], cams["H"])
        tiles_mask = None if choose_tiles is None else choose_tiles(isect["ranges"], TX * TY * n_views)
        _say(f"{wl}: oracle forward over {'all' if tiles_mask is None else int(tiles_mask.sum())} tiles, "
             f"M={isect['M']}")
        args = (P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"])
        ras = O32.rasterize_fwd(*args, tile_mask=tiles_mask)
        pix_in = np.ones(n_views * W * H, bool)
        if tiles_mask is not None:
            cc, rest = np.divmod(np.arange(n_views * W * H), W * H)
            ys, xs = np.divmod(rest, W)
            pix_in = tiles_mask[cc * TX * TY + (ys // 16) * TX + xs // 16] == 1
        ok = (ras["flags"] == 0) & pix_in
        frac = 1.0 - ok[pix_in].mean()
        _say(f"{wl}: flagged {int((~ok & pix_in).sum())} of {int(pix_in.sum())} pixels ({frac:.2e})")
        assert frac < flag_bar
        v_image, _ = scenes.upstream_grads(wl, n_views * W * H, seed=0)
        v_image[~ok] = 0.0
        _say(f"{wl}: GPU step (timed configuration, {n_views} views in one call)")
        g = _gpu_view(wl, list(range(n_views)), v_image)

        gp = g["proj"]
        np.testing.assert_array_equal(gp["radii"], proj["radii"])
        np.testing.assert_array_equal(gp["means2d"], proj["means2d"])
        np.testing.assert_array_equal(gp["depths"], proj["depths"])
        np.testing.assert_array_equal(gp["conics"], proj["conics"])
        np.testing.assert_allclose(gp["colors"], proj["colors"], rtol=0, atol=2e-6)
        _say(f"{wl}: culled lists M={g['M']} against square M={isect['M']}")

        err = np.abs(g["image"] - ras["image"]).max(axis=1)
        assert err[ok].max() <= 1e-4, err[ok].max()
        assert np.abs(g["final_T"] - ras["final_T"])[ok].max() <= 1e-4
        np.testing.assert_array_equal(_last_gid(g["last_ids"], g["ids"])[ok],
                                      _last_gid(ras["last_ids"], isect["ids"])[ok])
        _say(f"{wl}: forward ok (max image error {err[ok].max():.2e}); oracle backward")

        o2 = O32.rasterize_bwd(*args, ras["final_T"], ras["last_ids"], v_image, tile_mask=tiles_mask, abs_sums=True)
        from _gpu import assert_chain_close, assert_grad_close, oracle_project_bwd
        for k in ("v_means2d", "v_conics", "v_colors", "v_opacities"):
            assert_grad_close(g["g2"][k], o2[k], f"{wl}:{k}", abs_ref=o2["abs_" + k])
        # the chain: the float64 oracle's compositing of the same float32 projected values, then its projection
        # backward; the GPU's projection backward of its own compositing gradients checked stage-wise
        _say(f"{wl}: compositing gradients ok; float64 oracle forward")
        r64 = O64.rasterize_fwd(*args, tile_mask=tiles_mask)
        _say(f"{wl}: float64 oracle backward")
        o2x = O64.rasterize_bwd(*args, r64["final_T"], r64["last_ids"], v_image, tile_mask=tiles_mask)
        _say(f"{wl}: projection gradients against the float64 chain")
        pb32, pb64 = oracle_project_bwd(O32, P, sc, cams), oracle_project_bwd(O64, P, sc, cams)
        assert_chain_close(g["g3"], g["g2"], o2x, pb64(o2x), pb32, pb64, wl)
        _say(f"{wl}: gradients ok")
    finally:
        oracle.set_threads(1)


def test_full_frame_at_the_timed_configuration():
    # the benchmark's step: four consecutive views through one call of every stage
    _check_view("clusters1m_sh3_1080p", n_views=4)


def _longest_and_random(ranges, T, n_long=64, n_rand=448, seed=5):
    """The n_long tiles with the longest square lists and n_rand more at
    random among the other non-empty ones, as a tile mask."""
    lens = ranges[:, 1] - ranges[:, 0]
    busy = np.nonzero(lens > 0)[0]
    heavy = busy[np.argsort(-lens[busy])[:n_long]]
    rest = np.random.default_rng(seed).choice(np.setdiff1d(busy, heavy), size=n_rand, replace=False)
    mask = np.zeros(T, np.uint8)
    mask[np.concatenate([heavy, rest])] = 1
    return mask


def test_large_scene_512_tiles():
    _check_view("box3m_sh3_1080p", choose_tiles=_longest_and_random, flag_bar=3e-3)
