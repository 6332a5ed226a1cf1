"""The gradient-record layout (params.grad_records): the compositing backward
writes each (camera, Gaussian)'s nine 2D gradients as one record, and the
projection backward reads them there.  Both layouts hold the same sums: the
compositing backward's agree to the rounding order of its float atomics, and
the projection backward, given the same values in either layout, returns the
same bits."""
import numpy as np
import pytest
import torch

from paper_2409_06765_amd import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-grad-records] {msg}", flush=True)


# 64 x 48: 12 tiles, the four-waves-per-tile backward; 1280 x 720: 3,600 tiles, the one-wave RGB backward
@pytest.mark.parametrize("W,H,absgrad,aa", [(64, 48, False, False), (64, 48, True, True), (1280, 720, False, False),
                                             (1280, 720, True, False), (1280, 720, False, True)])
def test_records_hold_the_sums_of_the_four_arrays(W, H, absgrad, aa):
    from _gpu import gpu_backward, gpu_forward, np_, params, to_dev
    from paper_2409_06765_amd import _lib as L
    from paper_2409_06765_amd import rasterize as R
    _say(f"{W}x{H} absgrad={absgrad} antialiased={aa}")
    p = params(sh_degree=3, tile_cull=1, antialiased=aa)
    sc = scenes.scene_tiny(3000, sh_degree=3, seed=31, log_scale_mean=-3.0)
    cams = scenes.cams_tiny(W=W, H=H, f=0.8 * W, n_cams=2, seed=3)
    st = gpu_forward(p, sc, cams, n_eval=False)
    C, N = st["proj"]["radii"].shape
    P = sum(int(w) * int(h) for w, h in zip(st["W"], st["H"]))
    v_image = to_dev(np.random.default_rng(5).normal(size=(P, 3)).astype(np.float32))
    a2, a3 = gpu_backward(p, st, np_(v_image), absgrad=absgrad)

    pr = R._with(p, grad_records=1)
    rec = torch.zeros((C, N, L.GSR_GRAD_RECORD), device="cuda")
    ab = torch.zeros((C, N, 2), device="cuda") if absgrad else None
    proj, isect, fwd, d = st["proj"], st["isect"], st["fwd"], st["d"]
    L.gsr_rasterize_bwd(pr, C, N, 3, st["W"], st["H"], proj["means2d"], proj["conics"], proj["colors"],
                        proj["depths"], d["opacities"], proj["comps"], None, isect["ranges"], isect["ids_buf"],
                        isect.get("order"), fwd["image"], fwd["final_T"], fwd["last_ids"], v_image, None, rec,
                        None, None, None, None, ab, ws=fwd["ws"], flags=L.GSR_BWD_ACCUMULATE | L.GSR_BWD_PACKED)
    torch.cuda.synchronize()
    r = np_(rec)
    fields = dict(v_means2d=r[..., 0:2], v_conics=r[..., 2:5], v_colors=r[..., 5:8], v_opacities=r[..., 8])
    if absgrad:
        fields["v_means2d_abs"] = np_(ab)
    assert np.abs(np_(a2["v_conics"])).max() > 0
    for k, x in fields.items():
        y = np_(a2[k])
        assert np.linalg.norm(x - y) <= 1e-6 * max(np.linalg.norm(y), 1e-30), k

    # the projection backward: the arrays' values laid out as records give the same bits
    rec2 = torch.cat([a2["v_means2d"], a2["v_conics"], a2["v_colors"], a2["v_opacities"][..., None]], dim=-1)
    rec2 = rec2.contiguous()
    b3 = {k: torch.empty_like(v) for k, v in a3.items() if v is not None}
    L.gsr_project_bwd(pr, C, N, st["W"], st["H"], d["means"], d["quats"], d["scales"], d["opacities"], d["sh"],
                      st["vm"], st["Ks"], proj["radii"], proj["comps"], rec2, None, None, None, None,
                      b3["v_means"], b3["v_quats"], b3["v_scales"], b3["v_opacities"], b3["v_sh"])
    torch.cuda.synchronize()
    for k in ("v_means", "v_quats", "v_scales", "v_opacities", "v_sh"):
        np.testing.assert_array_equal(np_(b3[k]), np_(a3[k]), err_msg=k)
