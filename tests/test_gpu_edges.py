"""Edge cases of the HIP path through the C ABI: empty scenes, fully culled
views, a screen-filling Gaussian, the stand-alone radix sort, and batch
independence of multi-view renders."""
import numpy as np
import pytest
import torch

from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes
from _util import one_gaussian_scene

pytestmark = pytest.mark.gpu
O32 = Oracle(np.float32)


def _say(msg):
    print(f"[gpu-edges] {msg}", flush=True)


def test_pose_gradient_of_an_empty_scene_is_zero():
    from _gpu import np_, params, scene_to_dev, to_dev
    from paper_2409_06765_amd import rasterize as R
    sc = scenes.scene_tiny(0)
    cams = scenes.cams_tiny(W=40, H=30, n_cams=2, seed=3)
    d = scene_to_dev(sc)
    p = params()
    W, H = [int(w) for w in cams["W"]], [int(h) for h in cams["H"]]
    vm, Ks = to_dev(cams["viewmats"]), to_dev(cams["Ks"])
    proj = R.project(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, Ks, W, H)
    z = torch.zeros((2, 0, 3), device="cuda")
    g2 = dict(v_means2d=torch.zeros((2, 0, 2), device="cuda"), v_conics=z, v_colors=z,
              v_opacities=torch.zeros((2, 0), device="cuda"))
    g3 = R.project_backward(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, Ks, W, H, proj, g2,
                            viewmat_grad=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(g3["v_viewmats"]), 0.0)


def test_empty_scene_renders_background():
    from _gpu import gpu_forward, np_, params
    _say("empty scene")
    sc = scenes.scene_tiny(0)
    cams = scenes.cams_tiny(W=40, H=30)
    bg = np.array([[0.1, 0.2, 0.3]], np.float32)
    st = gpu_forward(params(), sc, cams, background=bg)
    assert st["isect"]["M"] == 0
    np.testing.assert_array_equal(np_(st["fwd"]["final_T"]), 1.0)
    np.testing.assert_array_equal(np_(st["fwd"]["last_ids"]), -1)
    np.testing.assert_allclose(np_(st["fwd"]["image"]), np.tile(bg, (1200, 1)))


def test_all_gaussians_behind_the_camera():
    from _gpu import gpu_backward, gpu_forward, np_, params
    _say("all culled")
    sc = scenes.scene_tiny(500, seed=4)
    sc["means"][:, 2] += 10.0      # every mean behind the camera at z = 4 looking at -z
    cams = scenes.cams_tiny(W=64, H=64)
    st = gpu_forward(params(), sc, cams)
    assert st["isect"]["M"] == 0 and int(np_(st["proj"]["radii"]).max()) == 0
    g2, g3 = gpu_backward(params(), st, np.ones((64 * 64, 3), np.float32))
    assert float(np.abs(np_(g3["v_means"])).max()) == 0.0


def test_screen_filling_gaussian_matches_oracle():
    from _gpu import gpu_forward, np_, params
    _say("screen-filling gaussian")
    sc = one_gaussian_scene((0.02, -0.01, 1.0), scale=(0.8, 0.6, 0.5), opacity=0.97, color=(0.3, 0.6, 0.9))
    cams = scenes.cams_tiny(W=300, H=200, f=250.0, radius=1.5)
    st = gpu_forward(params(), sc, cams)
    proj, isect, ras = O32.forward(OracleParams(), sc, cams)
    assert isect["M"] == st["isect"]["M"] == 19 * 13
    ok = ras["flags"] == 0
    assert np.abs(np_(st["fwd"]["image"]) - ras["image"]).max(axis=1)[ok].max() <= 1e-4


@pytest.mark.parametrize("M,key_bits,dups", [(1, 40, 1), (2, 33, 1), (3000, 45, 20), (100_003, 45, 1000),
                                             (250_000, 64, 1), (70_001, 17, 5)])
def test_radix_sort_is_stable_and_exact(M, key_bits, dups):
    from paper_2409_06765_amd import _lib as L
    _say(f"sort M={M} bits={key_bits}")
    g = np.random.default_rng(M)
    mask = np.uint64((1 << key_bits) - 1) if key_bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    base = g.integers(0, 2 ** 63, size=max(M // dups, 1), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    keys = (base[g.integers(0, base.size, M)] & mask).astype(np.uint64)
    ids = np.arange(M, dtype=np.int32)
    order = np.argsort(keys, kind="stable")
    dk = torch.from_numpy(keys).cuda()
    di = torch.from_numpy(ids).cuda()
    ka, ia = torch.empty_like(dk), torch.empty_like(di)
    ws = torch.empty(max(L.workspace_bytes(L.GSR_OP_SORT, 0, 0, M), 1), dtype=torch.uint8, device="cuda")
    L.gsr_sort_pairs(M, key_bits, dk, di, ka, ia, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dk.cpu().numpy(), keys[order])
    np.testing.assert_array_equal(di.cpu().numpy(), ids[order])


def test_multiview_batch_equals_each_view_alone():
    """The forward has no atomics: a view rendered inside a batch of views of
    different sizes is bit-identical to the same view rendered alone."""
    from _gpu import gpu_forward, np_, params
    sc = scenes.scene_tiny(800, sh_degree=3, seed=5, log_scale_mean=-2.6)
    eyes = [[0, 0, 4.0], [2.0, 2.0, 2.0], [-3.0, 0.5, 2.0], [0.5, -3.5, 1.0]]
    sizes = [(100, 80), (64, 64), (130, 47), (32, 200)]
    cams = scenes.cameras([scenes.look_at(e) for e in eyes], [scenes.intrinsics(1.2 * w, w, h) for w, h in sizes],
                          [w for w, _ in sizes], [h for _, h in sizes])
    p = params(sh_degree=3)
    _say("batch of 4 uneven views")
    st = gpu_forward(p, sc, cams)
    off = 0
    for c, (w, h) in enumerate(sizes):
        one = {k: v[c:c + 1] for k, v in cams.items()}
        s1 = gpu_forward(p, sc, one)
        img_b = np_(st["fwd"]["image"])[off:off + w * h]
        np.testing.assert_array_equal(np_(s1["fwd"]["image"]), img_b)
        np.testing.assert_array_equal(np_(s1["fwd"]["final_T"]), np_(st["fwd"]["final_T"])[off:off + w * h])
        off += w * h


def test_backward_flags_overwrite_repack_and_accumulate():
    """gsr_rasterize_bwd with flags 0 (overwrite, pack anew) on buffers full of
    garbage gives what the default path (records reused from the forward,
    added into zeroed buffers) gives; accumulating a second call doubles it."""
    from _gpu import gpu_backward, gpu_forward, np_, params, to_dev
    from paper_2409_06765_amd import _lib as L
    from paper_2409_06765_amd import rasterize as R
    _say("backward flags")
    sc = scenes.scene_tiny(400, sh_degree=2, seed=12, log_scale_mean=-2.6)
    cams = scenes.cams_tiny(W=75, H=53, f=60.0, n_cams=2, seed=12)
    p = params(sh_degree=2, antialiased=True)
    st = gpu_forward(p, sc, cams)
    v_image, v_alpha = scenes.upstream_grads("tiny", int(np.sum(cams["W"] * cams["H"])), seed=13, with_alpha=True)
    ref, _ = gpu_backward(p, st, v_image, v_alpha, absgrad=True)
    C, N = st["proj"]["radii"].shape
    keys = ("v_means2d", "v_conics", "v_colors", "v_opacities", "v_means2d_abs")
    junk = {k: torch.full_like(ref[k], 7.0) for k in keys}
    vi, va = to_dev(v_image), to_dev(v_alpha)
    d, pr, fw = st["d"], st["proj"], st["fwd"]
    ws = R.raster_workspace(C, N, vi.device)      # fresh workspace: must be packed again

    def call(g, ws, flags):
        L.gsr_rasterize_bwd(p, C, N, 3, st["W"], st["H"], pr["means2d"], pr["conics"], pr["colors"], None,
                            d["opacities"], pr["comps"], None, st["isect"]["ranges"], st["isect"]["ids_buf"], None, None,
                            fw["final_T"], fw["last_ids"], vi, va, g["v_means2d"], g["v_conics"], g["v_colors"], None,
                            g["v_opacities"], g["v_means2d_abs"], ws=ws, flags=flags)

    call(junk, ws, 0)
    torch.cuda.synchronize()
    for k in keys:
        x, y = np_(junk[k]), np_(ref[k])
        assert np.abs(x - y).max() <= 1e-5 * max(np.abs(y).max(), 1e-30), k
    call(junk, fw["ws"], L.GSR_BWD_ACCUMULATE | L.GSR_BWD_PACKED)
    torch.cuda.synchronize()
    for k in keys:
        x, y = np_(junk[k]), 2 * np_(ref[k])
        assert np.abs(x - y).max() <= 1e-5 * max(np.abs(y).max(), 1e-30), k
    with pytest.raises(L.GsrError):
        call(junk, ws, 4)


@pytest.mark.parametrize("capacity", [1, 37, 10 ** 6])
def test_binning_capacity_below_and_above_the_count(capacity):
    """gsr_bin_finish with a list capacity below the true count writes nothing
    past it and the wrapper rebuilds the lists once the count is known; with
    a capacity far above the count the extra sort blocks are empty.  Either
    way ids and ranges equal those of the oracle, bit for bit."""
    from _gpu import np_, params, scene_to_dev, to_dev
    from paper_2409_06765_amd import rasterize as R
    _say(f"binning capacity {capacity}")
    sc = scenes.scene_tiny(300, seed=8, log_scale_mean=-2.5)
    cams = scenes.cams_tiny(W=70, H=50, f=60.0, n_cams=2, seed=8)
    P = OracleParams()
    proj_o = O32.project(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], cams["viewmats"],
                         cams["Ks"], cams["W"], cams["H"])
    ref = O32.intersect(P, proj_o, cams["W"], cams["H"])
    assert ref["M"] > 37
    p = params()
    d = scene_to_dev(sc)
    W, H = [int(w) for w in cams["W"]], [int(h) for h in cams["H"]]
    proj = R.project(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], to_dev(cams["viewmats"]),
                     to_dev(cams["Ks"]), W, H)
    isect = R.intersect(p, proj, W, H, capacity=capacity)
    assert isect.check() == (capacity < ref["M"])
    assert isect["M"] == ref["M"]
    np.testing.assert_array_equal(np_(isect["ids"]), ref["ids"])
    np.testing.assert_array_equal(np_(isect["ranges"])[:len(ref["ranges"])], ref["ranges"])


def test_tile_order_is_longest_first_and_changes_nothing():
    """gsr_tile_order: a permutation of the tiles whose list lengths, taken
    in bucket units of an eighth of an octave, never increase; compositing
    in that order gives the same forward outputs bit for bit and the same
    gradients (up to the atomics' rounding order) as tile-index order."""
    from _gpu import assert_grad_close, gpu_forward, np_, params, to_dev
    from paper_2409_06765_amd import rasterize as R
    _say("tile order")
    sc = scenes.scene_tiny(700, sh_degree=1, seed=31, log_scale_mean=-2.3)
    cams = scenes.cams_tiny(W=131, H=77, f=80.0, n_cams=3, seed=31)
    p = params(sh_degree=1)
    st = gpu_forward(p, sc, cams)
    import torch
    from paper_2409_06765_amd import _lib as L
    T = int(st["isect"]["total_tiles"])
    # the pipeline orders only views of ORDER_MIN_TILES tiles or more; here the order is asked for directly
    assert T < R.ORDER_MIN_TILES and st["isect"].get("order") is None
    order_t = torch.empty(T, device="cuda:0", dtype=torch.int32)
    ws = torch.empty(L.workspace_bytes(L.GSR_OP_TILE_ORDER, 0, 0, 0), device="cuda:0", dtype=torch.uint8)
    L.gsr_tile_order(T, st["isect"]["ranges"], order_t, ws)
    isect = R.Intersections(**{k: v for k, v in st["isect"].items() if k != "order"}, order=order_t)
    isect._set_count(st["isect"]["M"])
    order = np_(order_t)[:T]
    np.testing.assert_array_equal(np.sort(order), np.arange(T))
    rg = np_(isect["ranges"])[:T]
    lens = (rg[:, 1] - rg[:, 0]).astype(np.int64)

    def bucket(n):
        if n <= 0:
            return 0
        o = int(n).bit_length() - 1
        m = (n >> (o - 3)) & 7 if o >= 3 else (n << (3 - o)) & 7
        return min(255, 1 + 8 * o + m)
    b = np.array([bucket(n) for n in lens[order]])
    assert np.all(np.diff(b) <= 0) and lens.max() > 4 * max(np.median(lens), 1)
    d = st["d"]
    plain = R.Intersections(**{k: v for k, v in isect.items() if k != "order"})
    plain._set_count(isect["M"])
    f0 = R.rasterize_forward(p, st["proj"], d["opacities"], plain, st["W"], st["H"], n_eval=True)
    f1 = R.rasterize_forward(p, st["proj"], d["opacities"], isect, st["W"], st["H"], n_eval=True)
    for k in ("image", "alpha", "final_T", "last_ids", "n_eval"):
        np.testing.assert_array_equal(np_(f0[k]), np_(f1[k]), err_msg=k)
    v = to_dev(scenes.upstream_grads("tiny", f0["image"].shape[0], seed=32)[0])
    g0 = R.rasterize_backward(p, st["proj"], d["opacities"], plain, st["W"], st["H"], f0, v)
    g1 = R.rasterize_backward(p, st["proj"], d["opacities"], isect, st["W"], st["H"], f1, v)
    for k in ("v_means2d", "v_conics", "v_colors", "v_opacities"):
        assert_grad_close(np_(g1[k]), np_(g0[k]), k)


@pytest.mark.parametrize("C,N", [(1, 2), (1, 63), (1, 64), (1, 1025), (1, 16384), (2, 8192), (1, 16385)])
def test_binning_keeps_equal_depths_in_id_order(C, N):
    """Many projected Gaussians share one depth bit pattern (means on three
    planes z = const seen by cameras whose rotation is exact): the depth
    order of gsr_bin_prepare (one block up to 16,384 keys, the multi-block
    sort beyond) must keep ties in id order, so that every tile's list is in
    (depth, id) order; ids and ranges bit for bit against the oracle's
    stable order (Rasterization of Gaussians: per-tile depth sort)."""
    from _gpu import gpu_forward, np_, params
    _say(f"equal-depth binning C={C} N={N}")
    g = np.random.default_rng(N + C)
    sc = scenes.scene_tiny(N, seed=N, log_scale_mean=-3.5)
    plane = g.integers(0, 3, N)
    plane[:2] = 1                                      # at least one tie, also for N = 2
    sc["means"][:, 2] = np.float32([-0.25, 0.0, 0.5])[plane]
    sc["means"][:, :2] = g.uniform(-1.2, 1.2, (N, 2)).astype(np.float32)
    # eyes on the z axis looking down -z: rotation diag(1, -1, -1) and t = (0, 0, d) are exact, so
    # t_z = d - z has one bit pattern per plane
    eyes = [[0.0, 0.0, 4.0], [0.0, 0.0, 5.0]][:C]
    cams = scenes.cameras([scenes.look_at(e) for e in eyes], [scenes.intrinsics(60.0, 96, 80)] * C, 96, 80)
    st = gpu_forward(params(), sc, cams)
    proj, isect, _ = O32.forward(OracleParams(), sc, cams)
    dep = proj["depths"][proj["radii"] > 0]
    assert np.unique(dep).size <= 3 * C and dep.size > np.unique(dep).size, "the scene must hold ties"
    np.testing.assert_array_equal(np_(st["proj"]["depths"]), proj["depths"])
    assert st["isect"]["M"] == isect["M"]
    np.testing.assert_array_equal(np_(st["isect"]["ids"]), isect["ids"])
    np.testing.assert_array_equal(np_(st["isect"]["ranges"]), isect["ranges"])


@pytest.mark.parametrize("C,N", [(1, 800), (1, 16384), (2, 5000), (1, 20000)])
def test_binning_skips_gaussians_of_no_tiles(C, N):
    """A third of the projected Gaussians lie behind the cameras and a third
    beside the image (radius 0 or an empty tile rectangle, so no tiles): the
    one-block depth sort (up to 16,384 keys) keeps them, last, with records of
    no tiles, and the multi-block sort drops them in its first pass; either
    way ids and ranges equal the oracle's bit for bit (Rasterization of
    Gaussians: tile binning)."""
    from _gpu import gpu_forward, np_, params
    _say(f"binning with Gaussians of no tiles C={C} N={N}")
    g = np.random.default_rng(7 * N + C)
    sc = scenes.scene_tiny(N, seed=N + 1, log_scale_mean=-3.0)
    part = g.integers(0, 3, N)
    sc["means"][part == 1, 2] = g.uniform(6.0, 9.0, int((part == 1).sum())).astype(np.float32)   # behind
    sc["means"][part == 2, 0] = g.uniform(4.0, 6.0, int((part == 2).sum())).astype(np.float32)   # beside
    eyes = [[0.0, 0.0, 4.0], [0.0, 0.3, 4.5]][:C]
    cams = scenes.cameras([scenes.look_at(e) for e in eyes], [scenes.intrinsics(80.0, 90, 70)] * C, 90, 70)
    st = gpu_forward(params(), sc, cams)
    proj, isect, _ = O32.forward(OracleParams(), sc, cams)
    vis = proj["radii"] > 0
    assert 0 < vis.sum() < vis.size, "the scene must hold Gaussians with and without tiles"
    assert st["isect"]["M"] == isect["M"]
    np.testing.assert_array_equal(np_(st["isect"]["ids"]), isect["ids"])
    np.testing.assert_array_equal(np_(st["isect"]["ranges"]), isect["ranges"])


@pytest.mark.parametrize("opaque,tile_cull", [(False, 0), (True, 0), (True, 1)])
def test_timed_forward_matches_the_counting_forward(opaque, tile_cull):
    """With the default thresholds and no per-pixel counts, plain RGB takes a walk of its own (the
    per-pixel state in vector registers, each condition applied by a select); its image, final T and
    last composited index equal the counting instance's bit for bit.  Opaque Gaussians make most
    pixels stop at T < 1e-4, the logit-normal opacities of the other scene put many alphas near 1/255."""
    from _gpu import gpu_forward, np_, params
    _say(f"timed forward vs counting forward, opaque={opaque} tile_cull={tile_cull}")
    sc = scenes.scene_tiny(4000, seed=21, log_scale_mean=-2.8)
    if opaque:
        sc["opacities"][:] = 0.995
    cams = scenes.cams_tiny(W=200, H=136, f=150.0, n_cams=2, seed=7)
    p = params(tile_cull=tile_cull)
    a = gpu_forward(p, sc, cams, n_eval=True)
    b = gpu_forward(p, sc, cams, n_eval=False)
    assert a["isect"]["M"] > 0
    for k in ("image", "final_T", "last_ids"):
        np.testing.assert_array_equal(np_(b["fwd"][k]), np_(a["fwd"][k]), err_msg=k)
    if opaque:   # the stopping rule is exercised: many pixels stop before the end of their tile's list
        W, H, TX, TY = 200, 136, 13, 9
        c, y, x = np.divmod(np.arange(2 * H * W), H * W)[0], *np.divmod(np.arange(2 * H * W) % (H * W), W)
        tile = c * TX * TY + (y // 16) * TX + x // 16
        ranges = np_(a["isect"]["ranges"])
        list_len = ranges[tile, 1] - ranges[tile, 0]
        stopped = np_(a["fwd"]["n_eval"])[:, 0] < list_len
        assert stopped.sum() > 2000, stopped.sum()
