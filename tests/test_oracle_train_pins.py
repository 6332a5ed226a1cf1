"""Pins of the oracle's training-loop steps (oracle/train.py), no GPU.

Hand-computed values (L1, densification statistics, plans, layouts), closed
forms (Adam's first step and constant-gradient steps, split children,
isotropic MCMC noise), independent library routines (torch.optim.Adam,
scipy's quaternion rotations), sampled covariances, central differences of
the whole step's loss with respect to the raw parameters, the ground truth
as a fixed point of a step, and a fit that lowers the loss.
"""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import Oracle, OracleParams
from oracle import train as T
from paper_2409_06765_amd import scenes

O64 = Oracle(np.float64)


def test_l1_values_and_gradient():
    img = np.array([0.5, 0.2, 0.7, -1.0])
    tgt = np.array([0.1, 0.2, 0.9, 1.0])
    loss, g = T.l1_loss(img, tgt, 0.25)
    assert loss == pytest.approx((0.4 + 0.0 + 0.2 + 2.0) / 4, abs=1e-15)
    np.testing.assert_array_equal(g, [0.25, 0.0, -0.25, -0.25])
    rng = np.random.default_rng(1)
    a, b = rng.uniform(0, 1, 50), rng.uniform(0, 1, 50)
    _, g = T.l1_loss(a, b, 0.1)
    h = 1e-7
    for i in range(50):
        e = np.zeros(50)
        e[i] = h
        fd = (T.l1_loss(a + e, b, 0.1)[0] - T.l1_loss(a - e, b, 0.1)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], abs=1e-8)


@pytest.mark.parametrize("kind", [T.ACT_NONE, T.ACT_EXP, T.ACT_SIGMOID])
def test_activation_chain_by_central_differences(kind):
    """L(raw) = sum w * act(raw) + reg * sum act(raw) differentiated by
    central differences against raw_gradient(raw, w, kind, reg)."""
    rng = np.random.default_rng(kind)
    raw = rng.normal(0, 1.5, 40)
    w = rng.normal(0, 1, 40)
    reg = 0.0 if kind == T.ACT_NONE else 0.37

    def L(r):
        return float(np.sum(w * T.activate(r, kind)) + reg * np.sum(T.activate(r, kind)))

    g = T.raw_gradient(raw, w, kind, reg)
    h = 1e-6
    for i in range(40):
        e = np.zeros(40)
        e[i] = h
        fd = (L(raw + e) - L(raw - e)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-7)
    np.testing.assert_allclose(T.activate([0.0], T.ACT_SIGMOID), [0.5])
    np.testing.assert_allclose(T.activate([np.log(3.0)], T.ACT_EXP), [3.0])


@pytest.mark.parametrize("eps", [1e-15, 1e-8])
def test_adam_matches_torch_adam(eps):
    rng = np.random.default_rng(2)
    p0 = rng.normal(size=30)
    grads = rng.normal(size=(6, 30)) * np.array([1, 1e-3, 10, 0.5, 2, 1e-2])[:, None]
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.999), eps=eps)
    mine, m, v = p0.copy(), np.zeros(30), np.zeros(30)
    for t, g in enumerate(grads, 1):
        p.grad = torch.tensor(g)
        opt.step()
        mine, m, v = T.adam(mine, g, m, v, t, 0.01, eps=eps)
        np.testing.assert_allclose(mine, p.detach().numpy(), rtol=0, atol=1e-14)


def test_adam_closed_forms():
    """Step 1 moves by -lr g / (|g| + eps); a constant gradient moves every
    step by that amount (the bias corrections make m_hat = g, v_hat = g^2)."""
    g = np.array([3.0, -0.5, 1e-6, 0.0])
    lr, eps = 0.1, 1e-8
    p, m, v = T.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr, eps=eps)
    np.testing.assert_allclose(p, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    q = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    for t in range(1, 8):
        q2, m, v = T.adam(q, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(q2 - q, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-18)
        q = q2


def test_group_learning_rate_rows():
    rng = np.random.default_rng(3)
    raw = rng.normal(size=(5, 16, 3))
    g = rng.normal(size=raw.shape)
    m, v = np.zeros(raw.size), np.zeros(raw.size)
    p, _, _, _ = T.adam_group(raw, g, m, v, 1, 0.05, lr_rest=0.0, row=48, row_first=3)
    moved = (p != raw.reshape(-1)).reshape(5, 48)
    assert moved[:, :3].all() and not moved[:, 3:].any()
    pa, _, _, _ = T.adam_group(raw, g, m, v, 1, 0.05, lr_rest=0.05, row=48, row_first=3)
    pb, _, _, _ = T.adam_group(raw, g, m, v, 1, 0.05)
    np.testing.assert_array_equal(pa, pb)


def test_densify_stats_hand_example():
    """Two views (100x50 and 40x80), three Gaussians, scale 2: the gradient
    components are scaled by (W/2, H/2) * 2 and form 3-4-5 triangles."""
    radii = np.array([[3, 0, 1], [2, 2, 0]])
    v = np.array([[[0.003, 0.008], [1.0, 1.0], [-0.012, 0.0]],
                  [[0.015, -0.01], [0.0, 0.005], [1.0, 1.0]]])
    acc, cnt = T.densify_stats(radii, v, [100, 40], [50, 80], 2.0, [0.1, 0.0, 0.0], [1, 0, 0])
    np.testing.assert_allclose(acc, [0.1 + 0.5 + 1.0, 0.4, 1.2], rtol=1e-14)
    np.testing.assert_array_equal(cnt, [3, 1, 1])


def test_densify_plan_cases():
    f = np.float32
    thr = f(2e-4)
    acc = np.array([1.0, 1e-3, 1e-3, 1e-5, 0.0, thr * f(3)], f)
    cnt = np.array([1, 2, 2, 1, 0, 3])
    scales = np.array([[0.5, 0.5, 0.5], [0.002, 0.5, 0.003], [0.005, 0.004, 0.003], [0.5] * 3, [0.5] * 3,
                       [0.5] * 3], f)
    opac = np.array([0.001, 0.5, 0.5, 0.5, 0.5, 0.5], f)
    action, offsets = T.densify_plan(acc, cnt, scales, opac, 2e-4, 0.01, 0.005)
    np.testing.assert_array_equal(action, [T.PRUNE, T.SPLIT, T.CLONE, T.KEEP, T.KEEP, T.KEEP])
    np.testing.assert_array_equal(offsets, [0, 0, 2, 4, 5, 6, 7])
    # the opacity threshold is strict, so is the gradient one
    a2, _ = T.densify_plan(acc, cnt, scales, np.full(6, 0.005, f), 2e-4, 0.01, 0.005)
    assert a2[0] == T.SPLIT and a2[5] == T.KEEP


def test_quaternion_rotation_matches_scipy():
    rng = np.random.default_rng(4)
    q = rng.normal(size=(50, 4)) * rng.uniform(0.2, 3.0, (50, 1))
    ref = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).as_matrix()
    np.testing.assert_allclose(T.quat_to_rot(q), ref, atol=1e-14)


def test_split_children_closed_forms_and_covariance():
    mu = np.array([[1.0, -2.0, 0.5]])
    q = np.array([[1.0, 0.0, 0.0, 0.0]])
    ls = np.log([[0.2, 0.3, 0.4]])
    eta = np.array([[[0.0, 0.0, 0.0], [1.0, -1.0, 2.0]]])
    ch = T.split_means(mu, q, ls, eta)
    np.testing.assert_allclose(ch[0, 0], mu[0], atol=1e-15)
    np.testing.assert_allclose(ch[0, 1], mu[0] + [0.2, -0.3, 0.8], atol=1e-15)
    # a rotated Gaussian: the children sample N(mu, R S^2 R^T)
    rng = np.random.default_rng(5)
    n = 200_000
    qr = np.array([0.3, -0.5, 0.7, 0.2])
    ls2 = np.log([0.5, 0.1, 0.25])
    eta = rng.standard_normal((n, 2, 3))
    ch = T.split_means(np.zeros((n, 3)), np.tile(qr, (n, 1)), np.tile(ls2, (n, 1)), eta)
    R = Rotation.from_quat([qr[1], qr[2], qr[3], qr[0]]).as_matrix()
    Sigma = R @ np.diag(np.exp(ls2) ** 2) @ R.T
    emp = np.cov(ch.reshape(-1, 3).T)
    assert np.abs(emp - Sigma).max() < 0.01 * np.abs(Sigma).max()


def test_densify_apply_layout():
    action = np.array([T.KEEP, T.PRUNE, T.CLONE, T.SPLIT])
    offsets = np.array([0, 1, 1, 3, 5])
    means = np.arange(12.0).reshape(4, 3)
    quats = np.tile([1.0, 0.0, 0.0, 0.0], (4, 1))
    ls = np.log(np.full((4, 3), 0.5))
    other = np.arange(8.0).reshape(4, 2) + 100
    state = np.arange(12.0).reshape(4, 3) + 200
    eta = np.zeros((4, 2, 3))
    eta[3] = [[1.0, 0.0, 0.0], [0.0, 0.0, -2.0]]
    cols = [(means, T.COL_MEANS), (ls, T.COL_LOG_SCALES), (other, T.COL_COPY), (state, T.COL_STATE)]
    m2, ls2, o2, s2 = T.densify_apply(action, offsets, cols, quats, ls, eta)
    np.testing.assert_array_equal(m2[:3], [means[0], means[2], means[2]])
    np.testing.assert_allclose(m2[3:], [means[3] + [0.5, 0, 0], means[3] + [0, 0, -1.0]], atol=1e-15)
    np.testing.assert_allclose(np.exp(ls2[3:]), 0.5 / 1.6, rtol=1e-15)
    np.testing.assert_array_equal(ls2[:3], ls[[0, 2, 2]])
    np.testing.assert_array_equal(o2, other[[0, 2, 2, 3, 3]])
    np.testing.assert_array_equal(s2, [state[0], state[2], [0, 0, 0], [0, 0, 0], [0, 0, 0]])


def test_opacity_reset():
    logits = np.array([-6.0, -4.59, -4.6, 0.0, 3.0])
    m, v = np.ones(5), np.ones(5)
    l2, m2, v2 = T.opacity_reset(logits, m, v, 0.01)
    o_old = 1 / (1 + np.exp(-logits))
    np.testing.assert_allclose(1 / (1 + np.exp(-l2)), np.minimum(o_old, 0.01), rtol=1e-14)
    assert not m2.any() and not v2.any()


def test_mcmc_noise_closed_forms():
    rng = np.random.default_rng(6)
    eta = rng.normal(size=(3, 3))
    mu = np.zeros((3, 3))
    q = np.tile([1.0, 0.0, 0.0, 0.0], (3, 1))
    s = np.array([[0.1] * 3, [0.2] * 3, [0.3, 0.1, 0.2]])
    o = np.array([0.005, 1.0, 0.0])
    out = T.mcmc_noise(mu, q, s, o, eta, 2.0)
    np.testing.assert_allclose(out[0], 2.0 * 0.5 * 0.01 * eta[0], rtol=1e-13)    # gate 1/2 at o = t
    assert np.abs(out[1]).max() < 1e-40                                            # opaque: no noise
    gate = 1 / (1 + np.exp(100 * (0.0 - 0.005)))
    np.testing.assert_allclose(out[2], 2.0 * gate * s[2] ** 2 * eta[2], rtol=1e-13)
    # rotated: Sigma = R S^2 R^T with scipy's rotation
    qr = np.array([[0.9, 0.1, -0.3, 0.2]])
    R = Rotation.from_quat([0.1, -0.3, 0.2, 0.9]).as_matrix()
    Sigma = R @ np.diag(s[2] ** 2) @ R.T
    out = T.mcmc_noise(np.ones((1, 3)), qr, s[2:], [0.0], eta[2:], 3.0)
    np.testing.assert_allclose(out[0], 1.0 + 3.0 * gate * Sigma @ eta[2], rtol=1e-12)


def _raw_scene(n, seed, sh_degree=1, W=40, H=32, n_cams=2):
    g = np.random.default_rng(seed)
    sc = scenes.scene_tiny(n, sh_degree=sh_degree, seed=seed, log_scale_mean=-2.0)
    cams = scenes.cams_tiny(W=W, H=H, f=40.0, n_cams=n_cams, seed=seed)
    raw = dict(means=sc["means"].astype(np.float64), quats=sc["quats"].astype(np.float64),
               log_scales=np.log(sc["scales"].astype(np.float64)),
               logits=np.log(sc["opacities"] / (1.0 - sc["opacities"])).astype(np.float64),
               sh=sc["sh"].astype(np.float64))
    return raw, cams, g


def _zero_state(raw):
    st = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in raw.items()}
    st["accum"] = np.zeros(len(raw["means"]))
    st["count"] = np.zeros(len(raw["means"]), np.int64)
    return st


LRS = dict(means=1e-3, quats=1e-3, log_scales=5e-3, logits=5e-2, sh=2.5e-3, sh_rest=1.25e-4)


def _render(P, raw, cams, views):
    sc = dict(means=raw["means"], quats=raw["quats"], scales=np.exp(raw["log_scales"]),
              opacities=1 / (1 + np.exp(-raw["logits"])), sh=raw["sh"])
    cv = {k: (np.asarray(v)[views] if k in ("viewmats", "Ks", "W", "H") else v) for k, v in cams.items()}
    return O64.forward(P, sc, cv)[2]["image"]


def test_ground_truth_is_a_fixed_point():
    P = OracleParams(sh_degree=1)
    raw, cams, _ = _raw_scene(60, 7)
    H, W = int(cams["H"][0]), int(cams["W"][0])
    tgt = _render(P, raw, cams, [0, 1]).reshape(2, H, W, 3)
    loss, new, st, grads = T.train_step(O64, P, raw, _zero_state(raw), cams, tgt, 1, LRS, [0, 1])
    assert loss == 0.0
    for k in raw:
        assert not grads[k].any(), k
        np.testing.assert_array_equal(new[k], raw[k])
    assert not st["accum"].any()


def test_step_gradients_by_central_differences():
    """The raw-parameter gradients of one step (L1 over two views plus the
    opacity and scale regularisers) against central differences of that
    loss; thresholds are lowered so the render is smooth, and a sample is
    used only where the difference quotients at h and h/2 agree."""
    P = OracleParams(sh_degree=1, alpha_min=1e-30, T_min=1e-30)
    raw, cams, g = _raw_scene(24, 8, W=32, H=32)
    views = [0, 1]
    tgt = g.uniform(0.0, 1.0, (2, 32, 32, 3))
    o_reg, s_reg = 0.3, 0.2

    def loss_of(r):
        img = _render(P, r, cams, views)
        t = tgt.reshape(img.shape)
        return (np.abs(img - t).sum() / t.size + o_reg * np.mean(1 / (1 + np.exp(-r["logits"])))
                + s_reg * np.mean(np.exp(r["log_scales"])))

    _, _, _, grads = T.train_step(O64, P, raw, _zero_state(raw), cams, tgt, 1, LRS, views, opacity_reg=o_reg,
                                  scale_reg=s_reg)
    checked = 0
    for name in ("means", "quats", "log_scales", "logits", "sh"):
        flat = raw[name].reshape(-1)
        for i in g.choice(flat.size, 6, replace=False):
            def at(s):
                r = {k: v.copy() for k, v in raw.items()}
                r[name].reshape(-1)[i] += s
                return loss_of(r)
            h = 1e-6
            fd1 = (at(h) - at(-h)) / (2 * h)
            fd2 = (at(h / 2) - at(-h / 2)) / h
            if abs(fd1 - fd2) > 1e-6 * max(1.0, abs(fd1)):
                continue                                  # a kink (L1 tie or a decision) inside +-h
            an = grads[name][i]
            assert abs(an - fd1) <= 1e-5 * max(abs(fd1), 1e-3), (name, i, an, fd1)
            checked += 1
    assert checked >= 24


def test_fitting_lowers_the_loss():
    """Twenty steps from a perturbed copy of a scene towards its own renders
    lower the L1 loss by at least a quarter."""
    P = OracleParams(sh_degree=1)
    gt, cams, g = _raw_scene(40, 9, n_cams=3)
    H, W = int(cams["H"][0]), int(cams["W"][0])
    tgt = _render(P, gt, cams, [0, 1, 2]).reshape(3, H, W, 3)
    raw = {k: v.copy() for k, v in gt.items()}
    raw["means"] = raw["means"] + g.normal(0, 0.05, raw["means"].shape)
    raw["sh"] = raw["sh"] + g.normal(0, 0.2, raw["sh"].shape)
    st = _zero_state(raw)
    losses = []
    for t in range(1, 21):
        views = [(t - 1) % 3]
        loss, raw, st, _ = T.train_step(O64, P, raw, st, cams, tgt, t, LRS, views)
        losses.append(loss)
    assert np.mean(losses[-3:]) < 0.75 * np.mean(losses[:3]), losses
