"""The oracle's analytic gradients (Depth Compositing Gradients, Projection
Gradients, Scale and rotation gradients, SH backward) against float64 central
finite differences of the rendered loss (no GPU)."""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2409_06765_amd import scenes
from _fd import fd_check

O64 = Oracle(np.float64)


def _check(rows, rejected, min_rows):
    assert len(rows) >= min_rows, (len(rows), rejected)
    scale = np.median([abs(r[3]) for r in rows]) + 1e-12
    bad = [r for r in rows if abs(r[2] - r[3]) > 1e-4 * max(abs(r[2]), abs(r[3])) + 1e-6 * scale]
    assert not bad, bad[:10]


@pytest.mark.parametrize("deg,aa,bg", [(3, 0, True), (-1, 0, False), (1, 1, False)])
def test_rendered_loss_gradients_match_fd(deg, aa, bg):
    P = OracleParams(sh_degree=deg, antialiased=aa)
    sc = scenes.scene_tiny(120, sh_degree=deg, seed=51, log_scale_mean=-2.0)
    cams = scenes.cams_tiny(W=72, H=56, f=60.0, n_cams=2, seed=51)
    npix = int(np.sum(cams["W"].astype(np.int64) * cams["H"]))
    v_image, v_alpha = scenes.upstream_grads("tiny", npix, seed=51, with_alpha=True)
    background = np.array([[0.3, 0.1, 0.7], [0.0, 0.2, 0.4]]) if bg else None
    rows, rejected = fd_check(O64, P, sc, cams, v_image.astype(np.float64), v_alpha.astype(np.float64),
                              background=background, n_params=48, eps=1e-4, seed=deg + 1 + 10 * aa)
    _check(rows, rejected, min_rows=48)


@pytest.mark.slow
def test_uniform100k_sh3_800_fd_on_64_sampled_parameters():
    """The finite-difference protocol on the 100k scene: 100k Gaussians, SH3, 800x800, eps = 1e-3, 64 sampled
    parameters (eight per Gaussian; a sample whose decision trace changes
    within +-eps is redrawn), float64 oracle."""
    P = OracleParams(sh_degree=3)
    sc = scenes.scene_uniform100k_sh3_800()
    cams = scenes.cams_uniform100k_sh3_800()
    v_image, _ = scenes.upstream_grads("uniform100k_sh3_800", 800 * 800)
    rows, rejected = fd_check(O64, P, sc, cams, v_image.astype(np.float64), None, n_params=64, eps=1e-3)
    _check(rows, rejected, min_rows=64)
