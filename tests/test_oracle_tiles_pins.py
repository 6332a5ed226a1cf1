"""Pins of the oracle's tile-support statement (oracle/tiles.py; no GPU).

The exact minimum of sigma over a tile's rectangle of pixel centres is
checked against dense sampling of the rectangle (it is a lower bound, and
attained up to the grid spacing) and against the closed form at the
rectangle's corner for a diagonal conic; the brute-force maximum alpha over
pixel centres can never exceed o exp(-min); on a rendered scene every pixel
that composites an entry sits in a tile whose entry passes both tests.
"""
import numpy as np

from oracle import Oracle, OracleParams
from oracle import tiles
from paper_2409_06765_amd import scenes


def _random_conics(n, seed):
    g = np.random.default_rng(seed)
    th = g.uniform(0, np.pi, n)
    s1, s2 = np.exp(g.uniform(-1, 4, n)), np.exp(g.uniform(-1, 4, n))
    ca, sa = np.cos(th), np.sin(th)
    # Sigma' = R diag(s1^2, s2^2) R^T; conic = Sigma'^-1
    S = np.stack([np.stack([ca * ca * s1 ** 2 + sa * sa * s2 ** 2, ca * sa * (s1 ** 2 - s2 ** 2)], -1),
                  np.stack([ca * sa * (s1 ** 2 - s2 ** 2), sa * sa * s1 ** 2 + ca * ca * s2 ** 2], -1)], -2)
    inv = np.linalg.inv(S)
    return inv[:, 0, 0], inv[:, 0, 1], inv[:, 1, 1]


def test_min_over_rectangle_matches_dense_sampling():
    n = 400
    a, b, c = _random_conics(n, 3)
    g = np.random.default_rng(4)
    u0 = g.uniform(-80, 80, n)
    v0 = g.uniform(-80, 80, n)
    u1, v1 = u0 + 15.0, v0 + 15.0
    m = tiles.min_sigma_rect(a, b, c, u0, u1, v0, v1)
    k = 301
    uu = u0[:, None] + (u1 - u0)[:, None] * np.linspace(0, 1, k)[None, :]
    vv = v0[:, None] + (v1 - v0)[:, None] * np.linspace(0, 1, k)[None, :]
    dense = np.full(n, np.inf)
    for j in range(k):
        q = 0.5 * a[:, None] * uu ** 2 + b[:, None] * uu * vv[:, j:j + 1] + 0.5 * c[:, None] * vv[:, j:j + 1] ** 2
        dense = np.minimum(dense, q.min(axis=1))
    assert np.all(m <= dense + 1e-9 * np.maximum(1.0, dense))
    # the grid spacing bounds how far above the true minimum the samples can be
    grad = np.abs(a) * 100 + np.abs(b) * 100 + np.abs(c) * 100
    assert np.all(dense - m <= grad * (15.0 / (k - 1)) * 2 + 1e-9)
    # a rectangle holding the mean has minimum 0
    s0, t0 = -g.uniform(0, 15, n), -g.uniform(0, 15, n)
    assert np.all(tiles.min_sigma_rect(a, b, c, s0, s0 + 15.0, t0, t0 + 15.0) == 0.0)


def test_diagonal_conic_corner_closed_form():
    """b = 0 and a rectangle in the first quadrant: the minimum is at its
    corner nearest the mean, a u0^2 / 2 + c v0^2 / 2."""
    a, b, c = np.array([0.3, 2.0]), np.array([0.0, 0.0]), np.array([0.7, 0.05])
    u0, v0 = np.array([3.0, 10.0]), np.array([4.5, 0.25])
    m = tiles.min_sigma_rect(a, b, c, u0, u0 + 15, v0, v0 + 15)
    np.testing.assert_allclose(m, 0.5 * a * u0 ** 2 + 0.5 * c * v0 ** 2, rtol=1e-15)


def test_support_of_a_rendered_scene():
    P = OracleParams()
    o = Oracle(np.float64)
    sc = scenes.scene_tiny(300, seed=17, log_scale_mean=-2.2)
    cams = scenes.cams_tiny(W=64, H=48, f=50.0, n_cams=2, seed=17)
    proj, isect, ras = o.forward(P, sc, cams)
    sup = tiles.tile_support(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"])
    bound = np.exp(-sup["min_sigma"]) * np.exp(sup["threshold"]) * P.alpha_min   # = o exp(-min sigma)
    assert np.all(sup["max_alpha_centres"] <= bound * (1 + 1e-12))
    seen = sup["max_alpha_centres"] >= P.alpha_min
    assert np.all(sup["min_sigma"][seen] <= sup["threshold"][seen] + 1e-12)
    # every composited (pixel, entry) pair lies in a tile whose entry is seen: the last
    # composited entry of every lit pixel is one of them
    lit = ras["last_ids"] >= 0
    last = np.asarray(ras["last_ids"])[lit]
    seen_pos = set(sup["pos"][seen].tolist())
    assert all(int(p) in seen_pos for p in last)
    # the 3-sigma squares hold many pairs no pixel centre sees
    assert seen.mean() < 0.8
