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


def params(sh_degree=-1, antialiased=False, tile_cull=0, **kw):
    """Library parameters for the tests: by default the paper's whole-square
    binning, whose lists (and list positions) the oracle reproduces bit for
    bit; tile_cull=1 is the culled binning the pipeline uses by default."""
    return R.make_params(sh_degree=sh_degree, antialiased=antialiased, tile_cull=tile_cull, **kw)


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
    if method == "bin" and isect.check():
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


# Per-term relative error a float32 evaluation may carry into a gradient sum
# (transmittance restored over up to ~1,500 entries, exp and rounding order):
# the budget of the summation term when the oracle supplies the sums of the
# terms' absolute values.
SUM_TERM_RTOL = 1e-4


def assert_grad_close(gpu, ref, name, rtol=1e-3, floor=1e-2, abs_ref=None):
    """Element-wise |gpu - ref| <= rtol * max(|ref|, floor * max|ref|)
    (+ SUM_TERM_RTOL * sum of the element's |terms| when ``abs_ref`` gives
    them: a sum of many terms of both signs is only known to that scale), and
    norm-wise ||gpu - ref|| <= rtol ||ref||."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max() if ref.size else 0.0
    if scale == 0.0:
        assert np.abs(gpu).max(initial=0.0) == 0.0, name
        return
    tol = rtol * np.maximum(np.abs(ref), floor * scale)
    if abs_ref is not None:
        tol = tol + SUM_TERM_RTOL * np.asarray(abs_ref, np.float64)
    err = np.abs(gpu - ref)
    bad = err > tol
    if bad.any():
        i = int(np.argmax((err / tol).reshape(-1)))
        raise AssertionError(f"{name}: {bad.sum()} of {bad.size} beyond tolerance; worst at flat index {i}: "
                             f"gpu {gpu.reshape(-1)[i]:.6e} ref {ref.reshape(-1)[i]:.6e} tol {tol.reshape(-1)[i]:.3e}"
                             f" (scale {scale:.3e})")
    assert np.linalg.norm(gpu - ref) <= rtol * np.linalg.norm(ref), name


def assert_as_accurate_as_f32(gpu, refs32, ref64, name, rtol=1e-3, floor=1e-2, factor=4.0):
    """Element-wise |gpu - ref64| <= max(rtol * max(|ref64|, floor * max|ref64|),
    factor * max_i |refs32[i] - ref64|): the GPU result is within the usual bar
    of the exact (float64) result, or no further from it than a few times
    plain float32 evaluations are (``refs32``: the float32 oracle on the same
    inputs and on inputs perturbed by an ulp, which samples how far float32
    can be from the exact result where the evaluation cancels); and the same
    norm-wise, ||gpu - ref64|| <= max(rtol ||ref64||, factor max_i ||refs32[i]
    - ref64||).  (The quaternion gradients of the 1M-Gaussian frame are an
    example: the float32 oracle's own projection backward is 8.5e-4 of the
    norm from the float64 one, so a float32 evaluation in another order can
    land above 1e-3.)"""
    gpu, ref64 = np.asarray(gpu, np.float64), np.asarray(ref64, np.float64)
    refs32 = [np.asarray(r, np.float64) for r in (refs32 if isinstance(refs32, (list, tuple)) else [refs32])]
    ref32 = refs32[0]
    scale = np.abs(ref64).max() if ref64.size else 0.0
    if scale == 0.0:
        assert np.abs(gpu).max(initial=0.0) == 0.0, name
        return
    spread = np.max([np.abs(r - ref64) for r in refs32], axis=0)
    tol = np.maximum(rtol * np.maximum(np.abs(ref64), floor * scale), factor * spread)
    err = np.abs(gpu - ref64)
    bad = err > tol
    if bad.any():
        i = int(np.argmax((err / tol).reshape(-1)))
        raise AssertionError(f"{name}: {bad.sum()} of {bad.size} beyond tolerance; worst at flat index {i}: gpu "
                             f"{gpu.reshape(-1)[i]:.6e} f32 oracle {ref32.reshape(-1)[i]:.6e} exact "
                             f"{ref64.reshape(-1)[i]:.6e} tol {tol.reshape(-1)[i]:.3e}")
    nspread = max(np.linalg.norm(r - ref64) for r in refs32)
    assert np.linalg.norm(gpu - ref64) <= max(rtol * np.linalg.norm(ref64), factor * nspread), \
        f"{name}: norm {np.linalg.norm(gpu - ref64):.3e} vs {np.linalg.norm(ref64):.3e} (float32 spread {nspread:.3e})"


G2_KEYS = ("v_means2d", "v_conics", "v_colors", "v_opacities")
G3_KEYS = ("v_means", "v_quats", "v_scales", "v_opacities", "v_sh")


def _g2_keys(g2):
    return [k for k in G2_KEYS + ("v_depths",) if g2.get(k) is not None]


def oracle_project_bwd(O, P, sc, cams, viewmat_grad=False):
    """The oracle's projection backward of a scene and cameras as a function
    of the compositing gradients (a dict of the G2_KEYS arrays [C,N,...] and
    optionally v_depths [C,N]); with viewmat_grad its outputs include
    v_viewmats."""
    def pb(g2):
        vd = g2.get("v_depths")
        return O.project_bwd(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"],
                             cams["viewmats"], cams["Ks"], cams["W"], cams["H"], *(np.asarray(g2[k]) for k in G2_KEYS),
                             v_depths=None if vd is None else np.asarray(vd), viewmat_grad=viewmat_grad)
    return pb


def propagated_error(pb64, dg2):
    """Element-wise bound on how far the projection backward's outputs move
    when its inputs, the compositing gradients, move by at most dg2 (absolute
    values, [C,N,...]).  The projection backward is linear in them (Projection
    Gradients), so the bound is sum over cameras c and input components j of
    |J_cj| dg2_cj, each column applied by one float64 oracle call."""
    C = np.asarray(dg2["v_opacities"]).shape[0]
    keys = _g2_keys(dg2)
    out = None
    for c in range(C):
        for k in keys:
            a = np.asarray(dg2[k], np.float64)
            for j in range(a.shape[-1] if a.ndim == 3 else 1):
                g = {kk: np.zeros(np.shape(dg2[kk])) for kk in keys}
                if a.ndim == 3:
                    g[k][c, :, j] = a[c, :, j]
                else:
                    g[k][c] = a[c]
                r = pb64(g)
                out = {kk: np.abs(v) for kk, v in r.items()} if out is None else \
                    {kk: out[kk] + np.abs(r[kk]) for kk in out}
    return out


def assert_chain_close(g3, g2, g2_ref64, g3_ref64, pb32, pb64, name, rtol=1e-3, floor=1e-2, keys=G3_KEYS):
    """The GPU chain (compositing backward g2, then projection backward g3)
    against the float64 oracle chain (g2_ref64, g3_ref64).

    1. Stage: g3 against the float64 oracle's projection backward of the GPU's
       own g2, as accurate as a float32 evaluation (assert_as_accurate_as_f32).
    2. End to end: |g3 - g3_ref64| <= rtol max(|ref|, floor max|ref|) + four
       times the float32 spread of stage 1 + E, where E is the measured
       compositing error |g2 - g2_ref64| (held to its own bar by the caller)
       carried through the projection backward (propagated_error); and
       norm-wise the same three terms.  E matters where the projection backward cancels: one
       scale gradient of the 1M-Gaussian frame is the sum of three terms of
       about 4.7e4 that cancel to about 10, so a 1e-5 relative change of a
       conic gradient moves it by 0.5%."""
    g2n = {k: np.asarray(g2[k], np.float64) for k in _g2_keys(g2_ref64)}
    s64, s32 = pb64(g2n), pb32(g2n)
    for k in keys:
        assert_as_accurate_as_f32(g3[k], [s32[k]], s64[k], f"{name}:stage:{k}", rtol=rtol, floor=floor)
    E = propagated_error(pb64, {k: np.abs(g2n[k] - np.asarray(g2_ref64[k], np.float64)) for k in g2n})
    for k in keys:
        gpu, ref = np.asarray(g3[k], np.float64), np.asarray(g3_ref64[k], np.float64)
        scale = np.abs(ref).max() if ref.size else 0.0
        if scale == 0.0:
            assert np.abs(gpu).max(initial=0.0) == 0.0, f"{name}:chain:{k}"
            continue
        tol = rtol * np.maximum(np.abs(ref), floor * scale) + 4.0 * np.abs(np.asarray(s32[k], np.float64) - s64[k]) \
            + E[k] * (1.0 + 1e-6)
        err = np.abs(gpu - ref)
        bad = err > tol
        if bad.any():
            i = int(np.argmax((err / tol).reshape(-1)))
            raise AssertionError(f"{name}:chain:{k}: {bad.sum()} of {bad.size} beyond tolerance; worst at flat "
                                 f"index {i}: gpu {gpu.reshape(-1)[i]:.6e} exact {ref.reshape(-1)[i]:.6e} tol "
                                 f"{tol.reshape(-1)[i]:.3e} (propagated {E[k].reshape(-1)[i]:.3e})")
        spread = np.asarray(s32[k], np.float64) - s64[k]
        bound = rtol * np.linalg.norm(ref) + 4.0 * np.linalg.norm(spread) + np.linalg.norm(E[k])
        assert np.linalg.norm(gpu - ref) <= bound, f"{name}:chain:{k} (norm {np.linalg.norm(gpu - ref):.3e} > {bound:.3e})"
