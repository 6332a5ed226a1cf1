"""Shared test helpers (inputs and comparisons only; no rasterizer arithmetic)."""
import numpy as np


def float_bits(x):
    return np.asarray(x, np.float32).view(np.uint32)


def one_gaussian_scene(mean, quat=(1.0, 0.0, 0.0, 0.0), scale=(0.5, 0.5, 0.5), opacity=1.0,
                       color=(0.2, 0.4, 0.6)):
    f32 = np.float32
    return dict(means=np.array([mean], f32), quats=np.array([quat], f32), scales=np.array([scale], f32),
                opacities=np.array([opacity], f32), sh=np.array([color], f32), sh_degree=-1)


def stack_scenes(*scenes):
    out = {k: np.concatenate([s[k] for s in scenes]) for k in ("means", "quats", "scales", "opacities", "sh")}
    out["sh_degree"] = scenes[0]["sh_degree"]
    return out


def simple_cam(W, H, f, cx=None, cy=None, viewmat=None):
    f32 = np.float32
    V = np.eye(4) if viewmat is None else np.asarray(viewmat)
    cx = W / 2.0 if cx is None else cx
    cy = H / 2.0 if cy is None else cy
    K = np.array([[f, 0, cx], [0, f, cy], [0, 0, 1]])
    return dict(viewmats=V[None].astype(f32), Ks=K[None].astype(f32),
                W=np.array([W], np.int32), H=np.array([H], np.int32))


def all_tiles(W, H, tile=16):
    W = np.atleast_1d(W)
    H = np.atleast_1d(H)
    out = []
    for c in range(len(W)):
        TX, TY = -(-int(W[c]) // tile), -(-int(H[c]) // tile)
        for ty in range(TY):
            for tx in range(TX):
                out.append((c, tx, ty))
    return np.array(out, np.int32)


def wide_cone_scene(n, seed, sh_degree=3, higher_band_std=0.6):
    """Gaussians in front of a camera at z = 4 looking at -z (cams_tiny's
    single camera), at depths 0.5 .. 3.5 and lateral offsets up to twice the
    depth: with a 1.3 x half-field Jacobian clamp many means fall outside it
    in x and in y.  Higher SH bands are strong so the view-direction gradient
    matters."""
    from paper_2409_06765_amd import scenes
    sc = scenes.scene_tiny(n, sh_degree=sh_degree, seed=seed, log_scale_mean=-1.5, spread=1.0)
    g = np.random.default_rng(seed)
    depth = g.uniform(0.5, 3.5, n)
    lat = g.uniform(-2.0, 2.0, (n, 2)) * depth[:, None]
    sc["means"] = np.stack([lat[:, 0], lat[:, 1], 4.0 - depth], 1).astype(np.float32)
    if sh_degree > 0:
        sc["sh"][:, 1:, :] = g.normal(0.0, higher_band_std, sc["sh"][:, 1:, :].shape).astype(np.float32)
    return sc
