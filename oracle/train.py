"""Training-loop steps around the rasterizer (TEST INFRASTRUCTURE ONLY).

Plain float64 NumPy statements of what one optimisation step of a synthetic
fit computes on top of the rasterizer's gradients, following the paper's
appendix on densification strategies (ADC, Absgrad, MCMC):

* ``l1_loss``: L = scale * sum |image - target| and its gradient
  scale * sign(image - target) (sign(0) = 0).  The paper does not state the
  photometric loss; the mean absolute error is the reading taken here.
* ``activate`` / ``raw_gradient``: the rasterizer takes activated scales
  exp(raw) and opacities sigmoid(raw); the optimiser updates the raw values,
  so the chain rule multiplies the activated gradient by exp(raw) or
  sigmoid(raw)(1 - sigmoid(raw)).  An L1 penalty reg * a on a positive
  activated value a adds reg to its gradient (the MCMC strategy's opacity
  and scale regularisers).
* ``adam``: Adam (Kingma and Ba, Algorithm 1) with bias correction.
* ``densify_stats``: ADC tracks, per Gaussian, the norm of the gradient of
  the loss with respect to its projected 2D mean, summed over the views that
  see it, and the number of such views.  Reading: the threshold 0.0002 is
  stated for gradients with respect to normalised device coordinates of a
  per-view loss, so the pixel-space gradient is scaled by (W/2, H/2) and by
  the number of views the step's loss averages over (``scale``).  With
  Absgrad the caller passes the per-axis absolute sums instead.
* ``densify_plan``: prune when the opacity is below the prune threshold;
  otherwise, when the average statistic exceeds the gradient threshold
  (accum > threshold * count, taken in float32 as the kernels take it),
  split when the largest scale exceeds the scale threshold, else clone.
  Output slots per Gaussian: prune 0, keep 1, clone 2, split 2, laid out in
  input order.
* ``densify_apply``: keep copies; clone writes the original and a copy;
  split writes two children whose means are mu + R(q) diag(s) eta_k (a draw
  of N(mu, Sigma)) and whose scales are s / shrink.  Optimiser moments are
  copied for kept Gaussians and for the original of a clone, zero for new
  Gaussians.
* ``opacity_reset``: o <- min(o, value) (in the raw logit domain) and its
  moments cleared.
* ``mcmc_noise``: the SGLD noise term on the centres,
  mu += coeff * sigmoid(-k (o - t)) * Sigma eta with Sigma = R S^2 R^T,
  coeff = lambda_noise * lr (reading of the MCMC strategy: the noise is
  shaped by the covariance and gated to low-opacity Gaussians, with k = 100
  and t = 0.005 as in the cited work).

Random draws (eta) are inputs.  Shares no code with the HIP library.
"""
import numpy as np

ACT_NONE, ACT_EXP, ACT_SIGMOID = 0, 1, 2
PRUNE, KEEP, CLONE, SPLIT = 0, 1, 2, 3
SLOTS = np.array([0, 1, 2, 2], np.int64)
COL_COPY, COL_MEANS, COL_LOG_SCALES, COL_STATE = 0, 1, 2, 3


def _f64(a):
    return np.asarray(a, np.float64)


# ---- loss --------------------------------------------------------------------
def l1_loss(image, target, scale):
    d = _f64(image) - _f64(target)
    return float(scale * np.abs(d).sum()), scale * np.sign(d)


# ---- activations ---------------------------------------------------------------
def activate(raw, kind):
    raw = _f64(raw)
    if kind == ACT_EXP:
        return np.exp(raw)
    if kind == ACT_SIGMOID:
        return 1.0 / (1.0 + np.exp(-raw))
    return raw.copy()


def raw_gradient(raw, g_act, kind, reg=0.0):
    """d L / d raw for L depending on a = act(raw), plus reg * a."""
    a = activate(raw, kind)
    g = _f64(g_act) + reg
    if kind == ACT_EXP:
        return g * a
    if kind == ACT_SIGMOID:
        return g * a * (1.0 - a)
    return g


# ---- Adam ------------------------------------------------------------------------
def adam(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam update at step t >= 1 (lr may be an array, one per element)."""
    g = _f64(grad)
    m = beta1 * _f64(m) + (1.0 - beta1) * g
    v = beta2 * _f64(v) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return _f64(param) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def group_lr(n, lr, lr_rest=None, row=0, row_first=0):
    """Per-element learning rates: lr_rest where i % row >= row_first."""
    if row <= 0:
        return np.full(n, lr)
    i = np.arange(n) % row
    return np.where(i < row_first, lr, lr_rest)


def adam_group(raw, g_act, m, v, step, lr, kind=ACT_NONE, reg=0.0, lr_rest=None, row=0, row_first=0,
               beta1=0.9, beta2=0.999, eps=1e-15):
    """Adam on a raw parameter whose activated value received g_act; returns
    (raw, m, v, activated) after the update."""
    raw = _f64(raw).reshape(-1)
    g = raw_gradient(raw, _f64(g_act).reshape(-1), kind, reg)
    lrs = group_lr(raw.size, lr, lr_rest, row, row_first)
    p, m, v = adam(raw, g, _f64(m).reshape(-1), _f64(v).reshape(-1), step, lrs, beta1, beta2, eps)
    return p, m, v, activate(p, kind)


# ---- ADC ---------------------------------------------------------------------------
def densify_stats(radii, v_means2d, W, H, scale, accum, count):
    """accum[n] += sum over views c with radii[c, n] > 0 of
    |(v_x W_c / 2, v_y H_c / 2)| * scale; count[n] += those views."""
    radii = np.asarray(radii)
    v = _f64(v_means2d)
    C, N = radii.shape
    acc = _f64(accum).copy()
    cnt = np.asarray(count, np.int64).copy()
    for c in range(C):
        seen = radii[c] > 0
        gx = v[c, :, 0] * (W[c] / 2.0) * scale
        gy = v[c, :, 1] * (H[c] / 2.0) * scale
        acc += np.where(seen, np.hypot(gx, gy), 0.0)
        cnt += seen
    return acc, cnt


def densify_plan(accum, count, scales, opacities, grad_threshold, scale_threshold, prune_opacity):
    """Action per Gaussian and exclusive output offsets (the last entry is
    the new count).  Decisions in float32, as the kernels take them."""
    f = np.float32
    acc = np.asarray(accum, f)
    cnt = np.asarray(count, np.int64)
    smax = np.asarray(scales, f).reshape(len(acc), 3).max(axis=1)
    o = np.asarray(opacities, f)
    thr = f(grad_threshold) * cnt.astype(f)
    grow = (cnt > 0) & (acc > thr)
    action = np.where(grow, np.where(smax > f(scale_threshold), SPLIT, CLONE), KEEP)
    action = np.where(o < f(prune_opacity), PRUNE, action).astype(np.int32)
    offsets = np.concatenate([[0], np.cumsum(SLOTS[action])]).astype(np.int64)
    return action, offsets


def quat_to_rot(q):
    """Rotation matrices of quaternions (w, x, y, z), normalised first."""
    q = _f64(q).reshape(-1, 4)
    w, x, y, z = (q / np.linalg.norm(q, axis=1, keepdims=True)).T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)


def split_means(means, quats, log_scales, normals):
    """Children means mu + R diag(s) eta_k, k = 0, 1 -> [N, 2, 3]."""
    R = quat_to_rot(quats)
    s = np.exp(_f64(log_scales).reshape(-1, 3))
    eta = _f64(normals).reshape(-1, 2, 3)
    return _f64(means).reshape(-1, 1, 3) + np.einsum("nij,nkj->nki", R, s[:, None, :] * eta)


def densify_apply(action, offsets, columns, quats, log_scales, normals, shrink=1.6):
    """columns: list of (src [N, width], kind).  Returns the new arrays."""
    action = np.asarray(action)
    offsets = np.asarray(offsets, np.int64)
    N = len(action)
    total = int(offsets[-1])
    children = None
    out = []
    for src, kind in columns:
        src = _f64(src).reshape(N, -1)
        dst = np.zeros((total, src.shape[1]))
        for n in range(N):
            a, o = action[n], offsets[n]
            if a == PRUNE:
                continue
            if a == KEEP:
                dst[o] = src[n]
            elif a == CLONE:
                dst[o] = src[n]
                dst[o + 1] = 0.0 if kind == COL_STATE else src[n]
            else:                                      # split
                for k in range(2):
                    if kind == COL_STATE:
                        dst[o + k] = 0.0
                    elif kind == COL_MEANS:
                        if children is None:
                            children = split_means(src, quats, log_scales, normals)
                        dst[o + k] = children[n, k]
                    elif kind == COL_LOG_SCALES:
                        dst[o + k] = np.log(np.exp(src[n]) / shrink)
                    else:
                        dst[o + k] = src[n]
        out.append(dst)
    return out


def opacity_reset(logits, m, v, value):
    """o <- min(o, value) on the raw logits; moments cleared."""
    cap = np.log(value / (1.0 - value))
    return np.minimum(_f64(logits), cap), np.zeros_like(_f64(m)), np.zeros_like(_f64(v))


# ---- MCMC --------------------------------------------------------------------------
def mcmc_noise(means, quats, scales, opacities, normals, coeff, k=100.0, t=0.005):
    """mu + coeff * sigmoid(-k (o - t)) * R S^2 R^T eta."""
    R = quat_to_rot(quats)
    s2 = _f64(scales).reshape(-1, 3) ** 2
    Sigma = np.einsum("nij,nj,nkj->nik", R, s2, R)
    gate = 1.0 / (1.0 + np.exp(k * (_f64(opacities) - t)))
    return _f64(means).reshape(-1, 3) + coeff * gate[:, None] * np.einsum("nij,nj->ni", Sigma,
                                                                          _f64(normals).reshape(-1, 3))


# ---- one whole step -------------------------------------------------------------------
def train_step(o, P, raw, state, cams, targets, step, lrs, views, absgrad=False, opacity_reg=0.0,
               scale_reg=0.0, beta1=0.9, beta2=0.999, eps=1e-15):
    """One step: render the chosen views of the activated scene with the
    oracle ``o``, L1 against the targets (mean over the views' pixels and
    channels), back-propagate, accumulate the ADC statistics and update every
    raw parameter with Adam.  ``raw``: means, quats, log_scales, logits, sh;
    ``state``: per parameter (m, v), plus "accum" and "count"; ``lrs``: lr of
    each parameter and "sh_rest".  Returns (loss, new raw, new state,
    gradients): the raw-parameter gradients by name, and under "activated"
    the gradients with respect to what the rasterizer took."""
    scales = np.exp(_f64(raw["log_scales"]))
    opac = 1.0 / (1.0 + np.exp(-_f64(raw["logits"])))
    scene = dict(means=raw["means"], quats=raw["quats"], scales=scales, opacities=opac, sh=raw["sh"])
    cv = {k: (np.asarray(v)[views] if k in ("viewmats", "Ks", "W", "H") else v) for k, v in cams.items()}
    proj, isect, ras = o.forward(P, scene, cv)
    tgt = _f64(targets)[views].reshape(ras["image"].shape)
    scale = 1.0 / tgt.size
    loss, v_image = l1_loss(ras["image"], tgt, scale)
    g2 = o.rasterize_bwd(P, proj, opac, isect["ranges"], isect["ids"], cv["W"], cv["H"], ras["final_T"],
                         ras["last_ids"], v_image, absgrad=absgrad)
    g3 = o.project_bwd(P, scene["means"], scene["quats"], scales, opac, scene["sh"], cv["viewmats"], cv["Ks"],
                       cv["W"], cv["H"], g2["v_means2d"], g2["v_conics"], g2["v_colors"], g2["v_opacities"])
    v2 = g2["v_means2d_abs"] if absgrad else g2["v_means2d"]
    acc, cnt = densify_stats(proj["radii"], v2, cv["W"], cv["H"], float(len(views)), state["accum"], state["count"])
    new_raw, new_state, grads = {}, {"accum": acc, "count": cnt}, {"activated": {}}
    groups = (("means", "v_means", ACT_NONE, 0.0), ("quats", "v_quats", ACT_NONE, 0.0),
              ("log_scales", "v_scales", ACT_EXP, scale_reg / max(np.size(raw["log_scales"]), 1)),
              ("logits", "v_opacities", ACT_SIGMOID, opacity_reg / max(np.size(raw["logits"]), 1)),
              ("sh", "v_sh", ACT_NONE, 0.0))
    for name, gname, kind, reg in groups:
        g_act = g3[gname]
        grads["activated"][name] = _f64(g_act)
        grads[name] = raw_gradient(_f64(raw[name]).reshape(-1), _f64(g_act).reshape(-1), kind, reg)
        kw = {}
        if name == "sh" and np.ndim(raw["sh"]) == 3:
            kw = dict(lr_rest=lrs["sh_rest"], row=int(np.prod(np.shape(raw["sh"])[1:])), row_first=3)
        m, v = state[name]
        p, m, v, _ = adam_group(raw[name], g_act, m, v, step, lrs[name], kind, reg, beta1=beta1, beta2=beta2,
                                eps=eps, **kw)
        new_raw[name] = p.reshape(np.shape(raw[name]))
        new_state[name] = (m.reshape(np.shape(raw[name])), v.reshape(np.shape(raw[name])))
    return loss, new_raw, new_state, grads
