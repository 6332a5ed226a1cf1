"""Seeded synthetic inputs: Gaussian scenes, cameras, upstream gradients and
serving traces.

This module only draws random numbers and lays them out; it holds none of the
rasterizer's arithmetic, so both the HIP path and the CPU oracle can be fed
from it.  Every draw goes through ``numpy.random.Generator(PCG64)`` seeded by
``SeedSequence([workload, stream, seed])`` with the streams

    0 = scene, 1 = cameras, 2 = upstream gradients, 3 = finite-difference
    samples, 4 = serving trace.

Activated parameters are produced here (scales = exp(log-scales), opacities =
sigmoid(logits)), because the rasterizer takes activated values.
"""
from dataclasses import dataclass

import numpy as np

STREAM_SCENE, STREAM_CAMS, STREAM_GRADS, STREAM_FD, STREAM_TRACE = 0, 1, 2, 3, 4

WORKLOADS = {
    "tiny": "Small parity case: N Gaussians in [-1,1]^3, one camera on the +z axis",
    "uniform10k_256": "Forward only: 10k Gaussians, direct RGB, 256x256, fx=fy=256, camera at (0,0,4)",
    "uniform100k_sh3_800": "Forward+backward: 100k Gaussians, SH degree 3, 800x800, fx=fy=1100, camera on a "
                           "radius-4 sphere",
    "clusters1m_sh3_1080p": "Training-step shape: 1M Gaussians in 32 clusters, SH degree 3, 1920x1080, fx=fy=1500, "
            "16 viewpoints on a radius-6 sphere",
    "box3m_sh3_1080p": "Large scene: 3M Gaussians (2.4M in a 20x20x5 box + 0.6M on a radius-50 shell), SH degree 3, "
            "1920x1080, fx=fy=1200, camera inside the box",
    "serving_mix": "Serving: the 1M-Gaussian cluster scene resident, 2000 Poisson requests over "
            "{256^2, 512^2, 800^2, 1280x720, 1920x1080}, focal 1.2 W",
}
_WL_INDEX = {name: i for i, name in enumerate(WORKLOADS)}


def rng(workload, stream, seed=0):
    ss = np.random.SeedSequence([_WL_INDEX[workload], stream, seed])
    return np.random.Generator(np.random.PCG64(ss))


def _unit_quats(g, n):
    q = g.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _sh_coeffs(g, n, degree, dc_low=0.0, dc_high=1.0, hi_std=0.05):
    k = (degree + 1) ** 2
    sh = np.empty((n, k, 3))
    sh[:, 0, :] = g.uniform(dc_low, dc_high, (n, 3))
    if k > 1:
        sh[:, 1:, :] = g.normal(0.0, hi_std, (n, k - 1, 3))
    return sh


def _pack(means, quats, log_scales, logits, sh, sh_degree):
    f32 = np.float32
    return dict(means=np.ascontiguousarray(means, f32), quats=np.ascontiguousarray(quats, f32),
                scales=np.ascontiguousarray(np.exp(log_scales), f32),
                opacities=np.ascontiguousarray(_sigmoid(logits), f32),
                sh=np.ascontiguousarray(sh, f32), sh_degree=sh_degree)


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World->camera 4x4 (OpenCV axes: x right, y down, z forward).
    Rows of the rotation are (right, down, forward); t = -R eye."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f = f / np.linalg.norm(f)
    u = np.asarray(up, np.float64)
    if abs(np.dot(f, u / np.linalg.norm(u))) > 0.999:
        u = np.array([0.0, 0.0, 1.0])
    right = np.cross(f, u)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])
    V = np.eye(4)
    V[:3, :3] = R
    V[:3, 3] = -R @ eye
    return V


def intrinsics(f, W, H):
    return np.array([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]])


def cameras(viewmats, Ks, W, H):
    C = len(viewmats)
    return dict(viewmats=np.ascontiguousarray(np.stack(viewmats), np.float32),
                Ks=np.ascontiguousarray(np.stack(Ks), np.float32),
                W=np.broadcast_to(np.asarray(W, np.int32), (C,)).copy(),
                H=np.broadcast_to(np.asarray(H, np.int32), (C,)).copy())


def _sphere_eyes(g, n, radius):
    v = g.standard_normal((n, 3))
    return radius * v / np.linalg.norm(v, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def scene_tiny(n=64, sh_degree=-1, seed=0, log_scale_mean=-2.5, spread=1.0):
    g = rng("tiny", STREAM_SCENE, seed)
    means = g.uniform(-spread, spread, (n, 3))
    quats = _unit_quats(g, n)
    log_scales = g.normal(log_scale_mean, 0.5, (n, 3))
    logits = g.normal(0.0, 1.0, n)
    if sh_degree < 0:
        sh = g.uniform(0.0, 1.0, (n, 3))
    else:
        sh = _sh_coeffs(g, n, sh_degree)
    return _pack(means, quats, log_scales, logits, sh, sh_degree)


def cams_tiny(W=64, H=48, f=60.0, n_cams=1, seed=0, radius=4.0):
    if n_cams == 1:
        eyes = [np.array([0.0, 0.0, radius])]
    else:
        eyes = list(_sphere_eyes(rng("tiny", STREAM_CAMS, seed), n_cams, radius))
    Ws = np.broadcast_to(np.asarray(W), (n_cams,))
    Hs = np.broadcast_to(np.asarray(H), (n_cams,))
    return cameras([look_at(e) for e in eyes], [intrinsics(f, w, h) for w, h in zip(Ws, Hs)], Ws, Hs)


def scene_uniform10k_256(seed=0, n=10_000):
    g = rng("uniform10k_256", STREAM_SCENE, seed)
    means = g.uniform(-1.0, 1.0, (n, 3))
    log_scales = g.normal(-4.0, 0.5, (n, 3))
    quats = _unit_quats(g, n)
    logits = g.normal(0.0, 1.0, n)
    rgb = g.uniform(0.0, 1.0, (n, 3))
    return _pack(means, quats, log_scales, logits, rgb, -1)


def cams_uniform10k_256():
    return cameras([look_at((0.0, 0.0, 4.0))], [intrinsics(256.0, 256, 256)], 256, 256)


def scene_uniform100k_sh3_800(seed=0, n=100_000):
    g = rng("uniform100k_sh3_800", STREAM_SCENE, seed)
    means = g.uniform(-1.0, 1.0, (n, 3))
    log_scales = g.normal(-4.0, 0.5, (n, 3))
    quats = _unit_quats(g, n)
    logits = g.normal(0.0, 1.0, n)
    sh = _sh_coeffs(g, n, 3)
    return _pack(means, quats, log_scales, logits, sh, 3)


def cams_uniform100k_sh3_800(seed=0):
    eye = _sphere_eyes(rng("uniform100k_sh3_800", STREAM_CAMS, seed), 1, 4.0)[0]
    return cameras([look_at(eye)], [intrinsics(1100.0, 800, 800)], 800, 800)


def scene_clusters1m_sh3_1080p(seed=0, n=1_000_000, n_clusters=32):
    g = rng("clusters1m_sh3_1080p", STREAM_SCENE, seed)
    centres = g.uniform(-3.0, 3.0, (n_clusters, 3))
    which = g.integers(0, n_clusters, n)
    means = centres[which] + g.normal(0.0, 0.3, (n, 3))
    log_scales = g.normal(-5.0, 1.0, (n, 3))
    quats = _unit_quats(g, n)
    logits = g.normal(0.0, 1.0, n)
    sh = _sh_coeffs(g, n, 3)
    return _pack(means, quats, log_scales, logits, sh, 3)


def cams_clusters1m_sh3_1080p(seed=0, n_views=16):
    eyes = _sphere_eyes(rng("clusters1m_sh3_1080p", STREAM_CAMS, seed), n_views, 6.0)
    return cameras([look_at(e) for e in eyes], [intrinsics(1500.0, 1920, 1080)] * n_views, 1920, 1080)


def scene_box3m_sh3_1080p(seed=0, n=3_000_000, far_fraction=0.2):
    g = rng("box3m_sh3_1080p", STREAM_SCENE, seed)
    n_far = int(round(n * far_fraction))
    n_box = n - n_far
    box = g.uniform([-10.0, -10.0, -2.5], [10.0, 10.0, 2.5], (n_box, 3))
    v = g.standard_normal((n_far, 3))
    shell = 50.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
    means = np.concatenate([box, shell])
    log_scales = np.minimum(g.normal(-5.0, 1.5, (n, 3)), 0.0)
    quats = _unit_quats(g, n)
    logits = g.normal(-1.0, 2.0, n)
    sh = _sh_coeffs(g, n, 3)
    return _pack(means, quats, log_scales, logits, sh, 3)


def cams_box3m_sh3_1080p(seed=0, n_views=4):
    g = rng("box3m_sh3_1080p", STREAM_CAMS, seed)
    eyes = g.uniform([-5.0, -5.0, -1.25], [5.0, 5.0, 1.25], (n_views, 3))
    th = g.uniform(0.0, 2.0 * np.pi, n_views)
    vms = [look_at(e, e + np.array([np.cos(t), np.sin(t), 0.0]), up=(0.0, 0.0, 1.0)) for e, t in zip(eyes, th)]
    return cameras(vms, [intrinsics(1200.0, 1920, 1080)] * n_views, 1920, 1080)


SERVE_RESOLUTIONS = [(256, 256), (512, 512), (800, 800), (1280, 720), (1920, 1080)]


@dataclass
class Request:
    rid: int
    arrival: float        # seconds from the start of the trace
    W: int
    H: int
    viewmat: np.ndarray   # [4,4] float32
    K: np.ndarray         # [3,3] float32


def serving_trace(rate_hz, n_requests=2000, seed=0, resolutions=None):
    """Poisson arrivals at ``rate_hz``, resolutions uniform over the set,
    focal 1.2 W, principal point at the image centre, poses on a radius-6
    sphere looking at the origin."""
    g = rng("serving_mix", STREAM_TRACE, seed)
    res = resolutions or SERVE_RESOLUTIONS
    gaps = g.exponential(1.0 / rate_hz, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    which = g.integers(0, len(res), n_requests)
    eyes = _sphere_eyes(g, n_requests, 6.0)
    out = []
    for i in range(n_requests):
        W, H = res[which[i]]
        out.append(Request(i, float(arrivals[i]), W, H, look_at(eyes[i]).astype(np.float32),
                           intrinsics(1.2 * W, W, H).astype(np.float32)))
    return out


def upstream_grads(workload, n_pix, seed=0, with_alpha=False):
    g = rng(workload, STREAM_GRADS, seed)
    v_image = g.standard_normal((n_pix, 3)).astype(np.float32)
    v_alpha = g.standard_normal(n_pix).astype(np.float32) if with_alpha else None
    return v_image, v_alpha
