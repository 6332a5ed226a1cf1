"""Which tiles a projected Gaussian can be seen in (TEST INFRASTRUCTURE ONLY).

Rasterization of Gaussians bins every projected Gaussian into the 16x16
tiles of its 3-sigma square, and a pixel skips a Gaussian whose
alpha = o exp(-sigma) is below 1/255.  So a (Gaussian, tile) pair of the
lists matters only if some pixel centre of the tile has
sigma <= ln(o / alpha_min).  This module states that in float64 NumPy, for
every entry of the oracle's per-tile lists:

* ``min_sigma_rect``: the exact minimum of sigma(u, v) = a u^2 / 2 + b u v +
  c v^2 / 2 over the rectangle spanned by the tile's pixel centres, with
  (u, v) = mean - pixel: 0 when the rectangle holds the mean, else the
  smallest of the four edge minima (for a convex quadratic on a segment, the
  unconstrained minimiser clamped to the segment);
* ``max_alpha_centres``: o exp(-sigma) maximised over the 256 pixel centres
  themselves, by brute force (no skip, stop or clamp rules).

Shares no code with the HIP library.
"""
import numpy as np


def _entries(ranges, ids, W, H, tile=16):
    """(entry position, tile id, camera, tile x, tile y, list id) of every
    entry of the per-tile lists."""
    W = np.asarray(W, np.int64)
    H = np.asarray(H, np.int64)
    TX, TY = (W + tile - 1) // tile, (H + tile - 1) // tile
    tile_off = np.concatenate([[0], np.cumsum(TX * TY)])
    ranges = np.asarray(ranges, np.int64)
    lens = ranges[:, 1] - ranges[:, 0]
    t = np.repeat(np.arange(len(ranges)), lens)
    pos = np.concatenate([np.arange(s, e) for s, e in ranges]) if len(t) else np.zeros(0, np.int64)
    cam = np.searchsorted(tile_off, t, side="right") - 1
    lt = t - tile_off[cam]
    ty, tx = lt // TX[cam], lt % TX[cam]
    return pos, t, cam, tx, ty, np.asarray(ids, np.int64)[pos]


def _quad(a, b, c, u, v):
    return 0.5 * a * u * u + b * u * v + 0.5 * c * v * v


def _edge_min(a, b, c, u0, v0, v1):
    """min over v in [v0, v1] of the quadratic at u = u0: dq/dv = b u + c v."""
    v = np.clip(-b * u0 / c, v0, v1)
    return _quad(a, b, c, u0, v)


def min_sigma_rect(a, b, c, u0, u1, v0, v1):
    """Exact minimum of sigma over [u0, u1] x [v0, v1] (a, c > 0, ac > b^2)."""
    inside = (u0 <= 0) & (u1 >= 0) & (v0 <= 0) & (v1 >= 0)
    m = np.minimum(_edge_min(a, b, c, u0, v0, v1), _edge_min(a, b, c, u1, v0, v1))
    # edges v = const: swap the roles of u and v
    m = np.minimum(m, np.minimum(_edge_min(c, b, a, v0, u0, u1), _edge_min(c, b, a, v1, u0, u1)))
    return np.where(inside, 0.0, m)


def tile_support(P, proj, opacities, ranges, ids, W, H, brute=True):
    """Per list entry: position, tile id, min_sigma_rect, the threshold
    ln(o / alpha_min) and (``brute``) max_alpha_centres.  ``ids`` are c*N + n."""
    tile = P.tile
    pos, t, cam, tx, ty, g = _entries(ranges, ids, W, H, tile)
    C, N = np.asarray(proj["radii"]).shape
    m2 = np.asarray(proj["means2d"], np.float64).reshape(-1, 2)[g]
    con = np.asarray(proj["conics"], np.float64).reshape(-1, 3)[g]
    o = np.asarray(opacities, np.float64)[g % N]
    if P.antialiased:
        o = o * np.asarray(proj["comps"], np.float64).reshape(-1)[g]
    x0, y0 = tile * tx + 0.5, tile * ty + 0.5
    x1, y1 = x0 + tile - 1, y0 + tile - 1
    a, b, c = con[:, 0], con[:, 1], con[:, 2]
    ms = min_sigma_rect(a, b, c, m2[:, 0] - x1, m2[:, 0] - x0, m2[:, 1] - y1, m2[:, 1] - y0)
    with np.errstate(divide="ignore"):
        thr = np.log(o / P.alpha_min)
    out = dict(pos=pos, tile=t, gid=g, min_sigma=ms, threshold=thr)
    if brute:
        best = np.full(len(g), np.inf)
        offs = np.arange(tile) + 0.5
        for j in range(tile):                      # pixel rows of the tile, all columns at once
            py = tile * ty + offs[j]
            v = m2[:, 1] - py
            u = m2[:, 0][:, None] - (tile * tx)[:, None] - offs[None, :]
            s = _quad(a[:, None], b[:, None], c[:, None], u, v[:, None]).min(axis=1)
            best = np.minimum(best, s)
        out["max_alpha_centres"] = o * np.exp(-best)
    return out
