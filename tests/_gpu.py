"""Helpers for GPU tests: run the HIP path stage by stage on seeded numpy
inputs and bring results back as numpy; comparisons against the oracle."""
import numpy as np
import torch

from paper_2409_06765_amd import rasterize as R

DEV = "cuda:0"


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def params(sh_degree=-1, antialiased=False, **kw):
    return R.make_params(sh_degree=sh_degree, antialiased=antialiased, **kw)


def scene_to_dev(sc):
    return {k: (to_dev(v) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}


def np_(t):
    return None if t is None else t.detach().cpu().numpy()


def gpu_forward(p, sc, cams, background=None, n_eval=True, method="bin", want_keys=False):
    d = scene_to_dev(sc)
    vm, Ks = to_dev(cams["viewmats"]), to_dev(cams["Ks"])
    W, H = [int(w) for w in cams["W"]], [int(h) for h in cams["H"]]
    bg = None if background is None else to_dev(np.asarray(background, np.float32))
    proj = R.project(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, Ks, W, H)
    isect = R.intersect(p, proj, W, H, method=method, want_keys=want_keys)
    fwd = R.rasterize_forward(p, proj, d["opacities"], isect, W, H, bg, n_eval=n_eval)
    torch.cuda.synchronize()
    return dict(d=d, vm=vm, Ks=Ks, W=W, H=H, bg=bg, proj=proj, isect=isect, fwd=fwd)


def gpu_backward(p, st, v_image, v_alpha=None, absgrad=False):
    vi = to_dev(np.asarray(v_image, np.float32))
    va = None if v_alpha is None else to_dev(np.asarray(v_alpha, np.float32))
    d = st["d"]
    g2 = R.rasterize_backward(p, st["proj"], d["opacities"], st["isect"], st["W"], st["H"], st["fwd"], vi, va,
                              st["bg"], absgrad=absgrad)
    g3 = R.project_backward(p, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], st["vm"], st["Ks"],
                            st["W"], st["H"], st["proj"], g2)
    torch.cuda.synchronize()
    return g2, g3


def assert_grad_close(gpu, ref, name, rtol=1e-3, floor=1e-2):
    """Element-wise |gpu - ref| <= rtol * max(|ref|, floor * max|ref|), and
    norm-wise ||gpu - ref|| <= rtol ||ref||."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max() if ref.size else 0.0
    if scale == 0.0:
        assert np.abs(gpu).max(initial=0.0) == 0.0, name
        return
    tol = rtol * np.maximum(np.abs(ref), floor * scale)
    err = np.abs(gpu - ref)
    bad = err > tol
    assert not bad.any(), (f"{name}: {bad.sum()} of {bad.size} beyond tolerance; worst "
                           f"{err.max():.3e} at ref {ref.reshape(-1)[np.argmax(err)]:.3e}, scale {scale:.3e}")
    assert np.linalg.norm(gpu - ref) <= rtol * np.linalg.norm(ref), name
