"""Float64 NumPy definitions for tiny scenes (TEST INFRASTRUCTURE ONLY).

A second, independent statement of what the rasterizer computes, written with
library primitives wherever one exists: ``numpy.linalg.inv`` for the conic,
``numpy.linalg.eigvalsh`` for the largest eigenvalue of the 2D covariance,
``scipy.special.sph_harm_y`` for the view-dependent colour, matrix products
for Sigma' = J R_cw Sigma R_cw^T J^T (Forward Pass, Projection of Gaussians).
The render is the plain definition of Rasterization of Gaussians: every pixel
composites, front to back in (depth, id) order, every projected Gaussian
(``mode="untiled"``) or those whose tile rectangle contains the pixel's tile
(``mode="rect"``), with the skip/stop rules.  No tiles, keys or sorts of
intersections.  Only for scenes of a few hundred Gaussians and pixels.
"""
import numpy as np
from scipy.special import sph_harm_y


def quat_to_R(q):
    """Data Conventions: Hamilton quaternion (w, x, y, z) -> rotation."""
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def real_sh(degree, d):
    """Real SH with the Condon-Shortley phase, ordered k = l^2 + l + m, from
    scipy's complex harmonics: m>0 -> sqrt2 Re Y_l^m, m<0 -> sqrt2 Im Y_l^|m|."""
    d = np.asarray(d, np.float64)
    polar = np.arccos(np.clip(d[2], -1.0, 1.0))
    azim = np.arctan2(d[1], d[0])
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), polar, azim)
            if m > 0:
                out.append(np.sqrt(2.0) * Y.real)
            elif m < 0:
                out.append(np.sqrt(2.0) * Y.imag)
            else:
                out.append(Y.real)
    return np.array(out)


def project(P, means, quats, scales, sh_or_colors, viewmat, K, W, H):
    """One camera.  Returns per-Gaussian dict arrays (valid, mean2d, conic,
    radius, depth, color, rect)."""
    means = np.asarray(means, np.float64)
    N = means.shape[0]
    V = np.asarray(viewmat, np.float64)
    Kc = np.asarray(K, np.float64)
    Rcw, tcw = V[:3, :3], V[:3, 3]
    fx, fy, cx, cy = Kc[0, 0], Kc[1, 1], Kc[0, 2], Kc[1, 2]
    TX, TY = -(-W // P.tile), -(-H // P.tile)
    out = dict(valid=np.zeros(N, bool), mean2d=np.zeros((N, 2)), conic=np.zeros((N, 3)),
               radius=np.zeros(N, np.int64), depth=np.zeros(N), color=np.zeros((N, 3)),
               rect=np.zeros((N, 4), np.int64), comp=np.ones(N))
    campos = -Rcw.T @ tcw
    for n in range(N):
        t = Rcw @ means[n] + tcw
        if t[2] < P.near_plane or t[2] > P.far_plane:
            continue
        q = np.asarray(quats[n], np.float64)
        if np.linalg.norm(q) == 0:
            continue
        R = quat_to_R(q)
        M = R @ np.diag(np.asarray(scales[n], np.float64))
        Sig = M @ M.T
        tx, ty, tz = t
        if P.jac_clamp > 0:
            limx = P.jac_clamp * 0.5 * W / fx
            limy = P.jac_clamp * 0.5 * H / fy
            tx = np.clip(tx / tz, -limx, limx) * tz
            ty = np.clip(ty / tz, -limy, limy) * tz
        J = np.array([[fx / tz, 0.0, -fx * tx / tz ** 2], [0.0, fy / tz, -fy * ty / tz ** 2]])
        cov2 = J @ Rcw @ Sig @ Rcw.T @ J.T
        covd = cov2 + P.eps2d * np.eye(2)
        if np.linalg.det(covd) <= 0:
            continue
        Y = np.linalg.inv(covd)
        lam = np.linalg.eigvalsh(covd)[-1]
        r = int(np.ceil(3.0 * np.sqrt(lam)))
        mx = fx * t[0] / t[2] + cx
        my = fy * t[1] / t[2] + cy
        x0 = int(np.clip(np.floor((mx - r) / P.tile), 0, TX))
        x1 = int(np.clip(np.floor((mx + r) / P.tile) + 1, 0, TX))
        y0 = int(np.clip(np.floor((my - r) / P.tile), 0, TY))
        y1 = int(np.clip(np.floor((my + r) / P.tile) + 1, 0, TY))
        if x0 >= x1 or y0 >= y1:
            continue
        if P.sh_degree < 0:
            col = np.asarray(sh_or_colors[n], np.float64)
        else:
            d = means[n] - campos
            d = d / np.linalg.norm(d)
            Yk = real_sh(P.sh_degree, d)
            col = np.maximum(Yk @ np.asarray(sh_or_colors[n], np.float64) + 0.5, 0.0)
        if P.antialiased:
            out["comp"][n] = np.sqrt(max(np.linalg.det(cov2) / np.linalg.det(covd), 0.0))
        out["valid"][n] = True
        out["mean2d"][n] = (mx, my)
        out["conic"][n] = (Y[0, 0], Y[0, 1], Y[1, 1])
        out["radius"][n] = r
        out["depth"][n] = t[2]
        out["color"][n] = col
        out["rect"][n] = (x0, x1, y0, y1)
    return out


def render(P, proj, opacities, W, H, background=None, mode="untiled"):
    """Plain definition; vectorised over pixels, looping over Gaussians in
    (depth, id) order.  Returns image [H,W,3], final_T [H,W], last [H,W]
    (Gaussian id of the last composited one, -1), n_comp [H,W] and margin
    [H,W]: the smallest |ln(value / threshold)| over the pixel's decisions
    against alpha_min and alpha_max (o exp(-sigma) of every entry it
    evaluates) and against T_min (the transmittance after every entry that
    passes the skip test, composited or stopping)."""
    ys, xs = np.mgrid[0:H, 0:W]
    px, py = xs + 0.5, ys + 0.5
    tx_of, ty_of = xs // P.tile, ys // P.tile
    T = np.ones((H, W))
    Cimg = np.zeros((H, W, 3))
    done = np.zeros((H, W), bool)
    last = np.full((H, W), -1, np.int64)
    n_comp = np.zeros((H, W), np.int64)
    margin = np.full((H, W), np.inf)
    valid = np.nonzero(proj["valid"])[0]
    order = valid[np.lexsort((valid, proj["depth"][valid]))]
    for n in order:
        a, b, c = proj["conic"][n]
        dx = proj["mean2d"][n, 0] - px
        dy = proj["mean2d"][n, 1] - py
        sigma = 0.5 * (a * dx * dx + c * dy * dy) + b * dx * dy
        o = opacities[n] * proj["comp"][n]
        araw = o * np.exp(-sigma)
        alpha = np.minimum(P.alpha_max, araw)
        seen = ~done
        if mode == "rect":
            x0, x1, y0, y1 = proj["rect"][n]
            seen &= (tx_of >= x0) & (tx_of < x1) & (ty_of >= y0) & (ty_of < y1)
        use = seen & (sigma >= 0) & (alpha >= P.alpha_min)
        Tn = T * (1.0 - alpha)
        with np.errstate(divide="ignore"):
            m = np.minimum(np.abs(np.log(araw / P.alpha_min)), np.abs(np.log(araw / P.alpha_max)))
            margin = np.where(seen & (sigma >= 0) & (araw > 0), np.minimum(margin, m), margin)
            margin = np.where(use, np.minimum(margin, np.abs(np.log(Tn / P.T_min))), margin)
        stop = use & (Tn < P.T_min)
        done |= stop
        comp = use & ~stop
        Cimg += np.where(comp[..., None], proj["color"][n] * (alpha * T)[..., None], 0.0)
        T = np.where(comp, Tn, T)
        last = np.where(comp, n, last)
        n_comp += comp
    if background is not None:
        Cimg += T[..., None] * np.asarray(background, np.float64)
    return dict(image=Cimg, final_T=T, last=last, n_comp=n_comp, margin=margin)
