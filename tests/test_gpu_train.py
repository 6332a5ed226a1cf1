"""The training-loop kernels on the GPU against oracle/train.py.

Element-wise parity on seeded inputs at sizes that span several blocks with
ragged tails (and unaligned views, which take the scalar paths): L1 values
and gradients (gradients bit for bit), Adam with every activation, the SH
learning-rate split and the regulariser, activations, ADC statistics, plans
(bit for bit, float32 decisions on both sides), apply, opacity reset and
MCMC noise.  Then one whole step of the GPU trainer against the oracle's
step, the ground truth as a fixed point, ADC bookkeeping through the
trainer, fits that lower the loss, and the 1M-Gaussian / 16-view 1080p
sizes on sampled elements.
"""
import numpy as np
import pytest
import torch

from oracle import Oracle, OracleParams
from oracle import train as T
from paper_2409_06765_amd import scenes

pytestmark = pytest.mark.gpu

O32 = Oracle(np.float32)


def _say(msg):
    print(f"[gpu-train] {msg}", flush=True)


def _L():
    from paper_2409_06765_amd import _lib
    return _lib


def _dev(a):
    from _gpu import to_dev
    return to_dev(np.ascontiguousarray(a, np.float32))


def _unaligned(a):
    """A device copy of a float32 array whose data starts 4 bytes past a
    16-byte boundary (a view into a larger buffer)."""
    flat = np.ascontiguousarray(a, np.float32).reshape(-1)
    buf = torch.zeros(flat.size + 4, device="cuda:0", dtype=torch.float32)
    v = buf[1:1 + flat.size]
    v.copy_(torch.from_numpy(flat))
    return v


# ---- L1 ----------------------------------------------------------------------------------
@pytest.mark.parametrize("n,aligned", [(3 * 37 * 23, True), (3 * 256 * 256, True), (4 * 1000 + 3, False),
                                       (5, True), (0, True)])
def test_l1_loss(n, aligned):
    from _gpu import np_
    L = _L()
    _say(f"l1 n={n} aligned={aligned}")
    g = np.random.default_rng(n)
    img = g.uniform(0, 1, n).astype(np.float32)
    tgt = g.uniform(0, 1, n).astype(np.float32)
    tie = g.random(n) < 0.1
    tgt[tie] = img[tie]
    scale = np.float32(1.0 / max(n, 1))
    mk = _dev if aligned else _unaligned
    vi = torch.empty(n, device="cuda:0", dtype=torch.float32) if aligned else _unaligned(np.zeros(n))
    loss = torch.empty(1, device="cuda:0", dtype=torch.float32)
    ws = torch.empty(L.workspace_bytes(L.GSR_OP_L1_LOSS, 0, 0, n), device="cuda:0", dtype=torch.uint8)
    L.gsr_l1_loss(mk(img), mk(tgt), float(scale), vi, loss, ws)
    ref_loss, ref_v = T.l1_loss(img, tgt, float(scale))
    np.testing.assert_array_equal(np_(vi), (ref_v / float(scale)).astype(np.float32) * scale)
    assert abs(float(np_(loss)[0]) - ref_loss) <= 1e-6 * max(abs(ref_loss), 1e-30)


# ---- Adam / activations -------------------------------------------------------------------------
def _adam_case(g, n, kind, reg, row, row_first, lr, lr_rest, step):
    raw = g.normal(0, 1.5, n).astype(np.float32)
    grad = g.normal(0, 1, n).astype(np.float32) * np.float32(10.0) ** g.integers(-4, 1, n).astype(np.float32)
    if step == 1:
        m = np.zeros(n, np.float32)
        v = np.zeros(n, np.float32)
    else:
        m = (g.normal(0, 0.1, n)).astype(np.float32)
        v = (g.uniform(0, 0.05, n) ** 2).astype(np.float32)
    return dict(raw=raw, grad=grad, m=m, v=v, kind=kind, reg=reg, row=row, row_first=row_first, lr=lr,
                lr_rest=lr_rest)


@pytest.mark.parametrize("step", [1, 7])
@pytest.mark.parametrize("aligned", [True, False])
def test_adam_step_groups(step, aligned):
    from _gpu import np_
    L = _L()
    _say(f"adam step={step} aligned={aligned}")
    g = np.random.default_rng(11 + step + 2 * aligned)
    cases = [_adam_case(g, 3 * 1001, T.ACT_NONE, 0.0, 0, 0, 1e-3, 1e-3, step),
             _adam_case(g, 4 * 1001, T.ACT_NONE, 0.0, 0, 0, 1e-3, 1e-3, step),
             _adam_case(g, 3 * 1001, T.ACT_EXP, 0.0007, 0, 0, 5e-3, 5e-3, step),
             _adam_case(g, 1001, T.ACT_SIGMOID, 0.003, 0, 0, 5e-2, 5e-2, step),
             _adam_case(g, 48 * 1001, T.ACT_NONE, 0.0, 48, 3, 2.5e-3, 1.25e-4, step),
             _adam_case(g, 0, T.ACT_NONE, 0.0, 0, 0, 1e-3, 1e-3, step)]
    mk = _dev if aligned else _unaligned
    groups, devs = [], []
    for c in cases:
        d = dict(param=mk(c["raw"]), grad=mk(c["grad"]), exp_avg=mk(c["m"]), exp_avg_sq=mk(c["v"]),
                 activated=mk(np.zeros_like(c["raw"])) if c["kind"] != T.ACT_NONE else None, lr=c["lr"],
                 lr_rest=c["lr_rest"], row=c["row"], row_first=c["row_first"], activation=c["kind"], reg=c["reg"])
        groups.append(d)
        devs.append(d)
    L.gsr_adam_step(groups, step, 0.9, 0.999, 1e-15)
    torch.cuda.synchronize()
    for i, (c, d) in enumerate(zip(cases, devs)):
        if c["raw"].size == 0:
            continue
        b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
        p, m, v, a = T.adam_group(c["raw"], c["grad"], c["m"], c["v"], step, c["lr"], c["kind"], c["reg"],
                                  c["lr_rest"], c["row"], c["row_first"], b1, b2, 1e-15)
        lrs = T.group_lr(c["raw"].size, c["lr"], c["lr_rest"], c["row"], c["row_first"])
        ratio = np.abs(c["raw"] - p) / lrs
        tol = 2e-5 * lrs * np.maximum(ratio, 1.0) + 3e-7 * np.abs(p)
        err = np.abs(np_(d["param"]).astype(np.float64) - p)
        assert np.all(err <= tol), (i, float((err / tol).max()))
        np.testing.assert_allclose(np_(d["exp_avg"]), m, rtol=2e-5, atol=1e-30 + 1e-6 * np.abs(m).max(),
                                   err_msg=f"m {i}")
        np.testing.assert_allclose(np_(d["exp_avg_sq"]), v, rtol=2e-5, atol=1e-6 * np.abs(v).max(),
                                   err_msg=f"v {i}")
        if d["activated"] is not None:
            np.testing.assert_allclose(np_(d["activated"]), a, rtol=2e-6, err_msg=f"act {i}")


@pytest.mark.parametrize("kind", [T.ACT_NONE, T.ACT_EXP, T.ACT_SIGMOID])
def test_activate(kind):
    from _gpu import np_
    L = _L()
    g = np.random.default_rng(kind)
    raw = g.normal(0, 3, 70_001).astype(np.float32)
    out = torch.empty(raw.size, device="cuda:0", dtype=torch.float32)
    L.gsr_activate(_dev(raw), kind, out)
    np.testing.assert_allclose(np_(out), T.activate(raw, kind), rtol=2e-6)


# ---- ADC --------------------------------------------------------------------------------------------
def test_densify_stats_two_calls():
    from _gpu import np_
    L = _L()
    g = np.random.default_rng(21)
    C, N = 3, 5003
    W, H = [640, 97, 1920], [480, 211, 1080]
    acc = np.zeros(N)
    cnt = np.zeros(N, np.int64)
    acc_d = torch.zeros(N, device="cuda:0")
    cnt_d = torch.zeros(N, device="cuda:0", dtype=torch.int32)
    for call in range(2):
        radii = (g.integers(0, 4, (C, N)) * (g.random((C, N)) < 0.7)).astype(np.int32)
        v = (g.normal(0, 1e-4, (C, N, 2))).astype(np.float32)
        from _gpu import to_dev
        L.gsr_densify_stats(C, N, W, H, to_dev(radii), _dev(v), 2.0, acc_d, cnt_d)
        acc, cnt = T.densify_stats(radii, v, W, H, 2.0, acc, cnt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np_(cnt_d), cnt)
    np.testing.assert_allclose(np_(acc_d), acc, rtol=2e-6, atol=1e-12)


def _plan_inputs(g, N):
    f = np.float32
    cnt = g.integers(0, 5, N).astype(np.int32)
    acc = (g.uniform(0, 2.5e-4, N) * cnt).astype(f)
    scales = np.exp(g.normal(np.log(0.01), 1.0, (N, 3))).astype(f)
    opac = g.uniform(0, 0.05, N).astype(f)
    # exact boundaries: the gradient and opacity tests are strict
    k = N // 7
    acc[:k] = (f(2e-4) * cnt[:k].astype(f))
    opac[k:2 * k] = f(0.005)
    scales[2 * k:3 * k, 1] = f(0.01)
    return acc, cnt, scales, opac


@pytest.mark.parametrize("N", [1, 1023, 5037, 0])
def test_densify_plan(N):
    from _gpu import np_, to_dev
    L = _L()
    _say(f"plan N={N}")
    g = np.random.default_rng(N + 3)
    acc, cnt, scales, opac = _plan_inputs(g, N)
    action = torch.empty(max(N, 1), device="cuda:0", dtype=torch.int32)
    offsets = torch.empty(N + 1, device="cuda:0", dtype=torch.int64)
    ws = torch.empty(max(L.workspace_bytes(L.GSR_OP_DENSIFY_PLAN, 0, N, 0), 1), device="cuda:0", dtype=torch.uint8)
    n_new = L.gsr_densify_plan(N, _dev(acc), to_dev(cnt), _dev(scales), _dev(opac), 2e-4, 0.01, 0.005, action,
                               offsets, ws)
    a_ref, o_ref = T.densify_plan(acc, cnt, scales, opac, 2e-4, 0.01, 0.005)
    np.testing.assert_array_equal(np_(action)[:N], a_ref)
    np.testing.assert_array_equal(np_(offsets), o_ref)
    assert n_new == o_ref[-1]
    if N > 1000:
        assert len(set(a_ref.tolist())) == 4


def test_densify_apply():
    from _gpu import np_, to_dev
    L = _L()
    g = np.random.default_rng(31)
    N = 3001
    acc, cnt, scales, opac = _plan_inputs(g, N)
    action, offsets = T.densify_plan(acc, cnt, scales, opac, 2e-4, 0.01, 0.005)
    total = int(offsets[-1])
    means = g.normal(0, 2, (N, 3)).astype(np.float32)
    quats = g.normal(0, 1, (N, 4)).astype(np.float32)
    ls = np.log(scales).astype(np.float32)
    logits = g.normal(0, 2, N).astype(np.float32)
    sh = g.normal(0, 1, (N, 16, 3)).astype(np.float32)
    st = g.normal(0, 1, (N, 4)).astype(np.float32)
    eta = g.normal(0, 1, (N, 2, 3)).astype(np.float32)
    srcs = [(means, L.GSR_COLUMN_MEANS, T.COL_MEANS), (quats, L.GSR_COLUMN_COPY, T.COL_COPY),
            (ls, L.GSR_COLUMN_LOG_SCALES, T.COL_LOG_SCALES), (logits, L.GSR_COLUMN_COPY, T.COL_COPY),
            (sh, L.GSR_COLUMN_COPY, T.COL_COPY), (st, L.GSR_COLUMN_STATE, T.COL_STATE)]
    cols, outs = [], []
    for a, kind, _ in srcs:
        dst = torch.full((total,) + a.shape[1:], float("nan"), device="cuda:0", dtype=torch.float32)
        cols.append((_dev(a), dst, kind))
        outs.append(dst)
    L.gsr_densify_apply(N, to_dev(action), to_dev(offsets), _dev(quats), _dev(ls), _dev(eta), 1.6, cols)
    refs = T.densify_apply(action, offsets, [(a, k) for a, _, k in srcs], quats, ls, eta, 1.6)
    torch.cuda.synchronize()
    got = [np_(o).reshape(total, -1) for o in outs]
    split_rows = np.zeros(total, bool)
    bound = np.zeros(total)
    for n in np.flatnonzero(action == T.SPLIT):
        for k in range(2):
            r = offsets[n] + k
            split_rows[r] = True
            bound[r] = np.abs(means[n]).max() + np.sum(scales[n] * np.abs(eta[n, k]))
    # copies and states bit for bit; the split children's means and log-scales to float32 rounding
    for i in (1, 3, 4, 5):
        np.testing.assert_array_equal(got[i], refs[i].astype(np.float32), err_msg=f"column {i}")
    np.testing.assert_array_equal(got[0][~split_rows], refs[0][~split_rows].astype(np.float32))
    np.testing.assert_array_equal(got[2][~split_rows], refs[2][~split_rows].astype(np.float32))
    assert np.all(np.abs(got[0][split_rows] - refs[0][split_rows]) <= 1e-6 * bound[split_rows][:, None])
    assert np.all(np.abs(got[2][split_rows] - refs[2][split_rows]) <= 1e-6 * (np.abs(refs[2][split_rows]) + 1))
    assert split_rows.sum() > 100 and (action == T.CLONE).sum() > 30 and (action == T.PRUNE).sum() > 100


def test_opacity_reset():
    from _gpu import np_
    L = _L()
    g = np.random.default_rng(41)
    N = 4099
    logits = g.normal(-3, 3, N).astype(np.float32)
    m = g.normal(0, 1, N).astype(np.float32)
    v = g.uniform(0, 1, N).astype(np.float32)
    ld, md, vd = _dev(logits), _dev(m), _dev(v)
    od = torch.empty(N, device="cuda:0")
    L.gsr_opacity_reset(N, ld, md, vd, od, 0.01)
    l2, m2, v2 = T.opacity_reset(logits, m, v, 0.01)
    np.testing.assert_allclose(np_(ld), l2, rtol=2e-7, atol=0)
    assert not np_(md).any() and not np_(vd).any()
    np.testing.assert_allclose(np_(od), T.activate(l2, T.ACT_SIGMOID), rtol=2e-6)
    assert np.all(np_(od) <= np.float32(0.01) * (1 + 1e-6))


def test_mcmc_noise():
    from _gpu import np_
    L = _L()
    g = np.random.default_rng(51)
    N = 5001
    means = g.normal(0, 2, (N, 3)).astype(np.float32)
    quats = g.normal(0, 1, (N, 4)).astype(np.float32)
    scales = np.exp(g.normal(-3, 1, (N, 3))).astype(np.float32)
    opac = np.concatenate([g.uniform(0, 0.02, N // 2), g.uniform(0, 1, N - N // 2)]).astype(np.float32)
    eta = g.normal(0, 1, (N, 3)).astype(np.float32)
    md = _dev(means)
    coeff = 5e5 * 1.6e-4
    L.gsr_mcmc_noise(N, md, _dev(quats), _dev(scales), _dev(opac), _dev(eta), coeff, 100.0, 0.005)
    ref = T.mcmc_noise(means, quats, scales, opac, eta, coeff, 100.0, 0.005)
    Rm = T.quat_to_rot(quats)
    Sig = np.einsum("nij,nj,nkj->nik", Rm, scales.astype(np.float64) ** 2, Rm)
    gate = 1 / (1 + np.exp(100 * (opac.astype(np.float64) - 0.005)))
    bound = coeff * gate[:, None] * np.einsum("nij,nj->ni", np.abs(Sig), np.abs(eta))
    err = np.abs(np_(md) - ref)
    assert np.all(err <= 1e-5 * bound + 2.5e-7 * np.abs(ref) + 1e-30)
    assert (np.abs(ref - means) > 1e-4).sum() > 100          # the noise is visible where the gate is open


# ---- the trainer ------------------------------------------------------------------------------------
def _raw_from_scene(sc):
    return dict(means=sc["means"], quats=sc["quats"], log_scales=np.log(sc["scales"]),
                logits=np.log(sc["opacities"] / (1 - sc["opacities"])), sh=sc["sh"])


def _trainer(raw, cams, targets, deg, **cfg):
    from paper_2409_06765_amd.train import GaussianTrainer, TrainConfig
    from _gpu import params
    return GaussianTrainer(raw, cams, torch.as_tensor(targets, dtype=torch.float32), TrainConfig(**cfg),
                           sh_degree=deg, params=params(sh_degree=deg))


LRS = dict(means=1.6e-4, quats=1e-3, log_scales=5e-3, logits=5e-2, sh=2.5e-3, sh_rest=2.5e-3 / 20)


def test_one_step_matches_the_oracle_step():
    """Step 5 of a fit (seeded moments, two views, SH degree 1): loss,
    statistics and every updated raw parameter against the oracle's step."""
    from _gpu import np_, to_dev
    deg = 1
    sc = scenes.scene_tiny(500, sh_degree=deg, seed=61, log_scale_mean=-2.4)
    cams = scenes.cams_tiny(W=72, H=56, f=60.0, n_cams=3, seed=61)
    g = np.random.default_rng(61)
    targets = g.uniform(0, 1, (3, 56, 72, 3)).astype(np.float32)
    raw = _raw_from_scene(sc)
    tr = _trainer(raw, cams, targets, deg, strategy="adc", views_per_step=2, refine_start=10 ** 9,
                  reset_every=10 ** 9, lr_means=LRS["means"], lr_means_final=LRS["means"])
    state = {}
    for k in raw:
        m = g.normal(0, 1e-3, np.shape(raw[k])).astype(np.float32)
        v = (g.uniform(1e-4, 3e-3, np.shape(raw[k])) ** 2).astype(np.float32)
        tr.m[k].copy_(to_dev(m).reshape(tr.m[k].shape))
        tr.v[k].copy_(to_dev(v).reshape(tr.v[k].shape))
        state[k] = (m.astype(np.float64), v.astype(np.float64))
    state["accum"] = np.zeros(500)
    state["count"] = np.zeros(500, np.int64)
    tr.step_no = 4
    views = tr.views_of(5)
    loss = float(np_(tr.step())[0])
    torch.cuda.synchronize()
    P = OracleParams(sh_degree=deg)
    raw32 = {k: np.asarray(v, np.float32) for k, v in raw.items()}
    o_loss, o_raw, o_state, o_grads = T.train_step(O32, P, raw32, state, cams, targets, 5, LRS, views,
                                                   beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)))
    _say(f"step loss gpu {loss:.6f} oracle {o_loss:.6f}")
    assert abs(loss - o_loss) <= 1e-5 * o_loss
    np.testing.assert_array_equal(np_(tr.count), o_state["count"])
    np.testing.assert_allclose(np_(tr.accum), o_state["accum"], rtol=2e-3, atol=2e-3 * o_state["accum"].max())
    gnames = dict(means="v_means", quats="v_quats", log_scales="v_scales", logits="v_opacities", sh="v_sh")
    from _gpu import assert_grad_close
    for k, gk in gnames.items():
        assert_grad_close(np_(tr.last_grads[gk]), o_grads["activated"][k].reshape(np_(tr.last_grads[gk]).shape),
                          f"step:{k}")
    b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
    bc1, bc2 = 1 - b1 ** 5, 1 - b2 ** 5
    for k in raw:
        got = np_(tr.raw[k]).astype(np.float64).reshape(-1)
        ref = o_raw[k].reshape(-1)
        # propagate the gradient bar (1e-3 of max(|g|, 1e-2 max|g|), raw
        # gradients) through one Adam update with the oracle's moments
        gr = o_grads[k].reshape(-1)
        e_g = 1e-3 * np.maximum(np.abs(gr), 1e-2 * np.abs(gr).max())
        m_new, v_new = o_state[k][0].reshape(-1), o_state[k][1].reshape(-1)
        sv = np.sqrt(v_new / bc2)
        lrs = T.group_lr(ref.size, LRS[k], LRS["sh_rest"], 6 * 2, 3) if k == "sh" else LRS[k]
        du = lrs / (sv + 1e-15) * ((1 - b1) / bc1 * e_g + np.abs(m_new / bc1) / (sv + 1e-15) *
                                   (1 - b2) * np.abs(gr) * e_g / (bc2 * (sv + 1e-15)))
        tol = 2 * du + 3e-7 * np.abs(ref) + 1e-6 * np.asarray(lrs)
        bad = np.abs(got - ref) > tol
        assert not bad.any(), (k, int(bad.sum()), float((np.abs(got - ref) / tol).max()))


def test_ground_truth_is_a_fixed_point():
    from _gpu import np_
    deg = 2
    sc = scenes.scene_tiny(400, sh_degree=deg, seed=71, log_scale_mean=-2.3)
    cams = scenes.cams_tiny(W=64, H=48, f=55.0, n_cams=2, seed=71)
    raw = _raw_from_scene(sc)
    tr = _trainer(raw, cams, np.zeros((2, 48, 64, 3), np.float32), deg, strategy="none", views_per_step=2)
    _, _, _, _, _, _, fwd = tr.render([0, 1])
    tr.targets.copy_(fwd["image"].reshape(2, 48, 64, 3))
    before = {k: np_(v).copy() for k, v in tr.raw.items()}
    loss = float(np_(tr.step())[0])
    assert loss == 0.0
    for k, v in tr.raw.items():
        np.testing.assert_array_equal(np_(v), before[k], err_msg=k)


def test_adc_refinement_through_the_trainer():
    """A refinement step splits, clones and prunes by the plan; the counts
    add up, the new Gaussians' moments are zero and the statistics restart."""
    from _gpu import np_
    deg = 0
    sc = scenes.scene_tiny(600, sh_degree=deg, seed=81, log_scale_mean=-2.0)
    cams = scenes.cams_tiny(W=64, H=64, f=60.0, n_cams=2, seed=81)
    sc["opacities"][:50] = 0.003
    raw = _raw_from_scene(sc)
    g = np.random.default_rng(81)
    tr = _trainer(raw, cams, g.uniform(0, 1, (2, 64, 64, 3)).astype(np.float32), deg, strategy="adc",
                  views_per_step=2, refine_start=0, refine_every=1, grad_threshold=2e-5, scale_threshold=0.08,
                  reset_every=10 ** 9)
    N0 = tr.N
    tr.step()
    action, offsets = (np_(x) for x in tr.last_plan)
    torch.cuda.synchronize()
    counts = np.bincount(action, minlength=4)
    _say(f"refinement: prune {counts[0]} keep {counts[1]} clone {counts[2]} split {counts[3]} -> {tr.N}")
    assert counts[0] >= 50 and counts[2] > 0 and counts[3] > 0
    assert tr.N == N0 - counts[0] + counts[2] + counts[3] == offsets[-1]
    new_rows = np.zeros(tr.N, bool)
    for n in np.flatnonzero(action >= T.CLONE):
        o = offsets[n]
        new_rows[o + 1] = True
        if action[n] == T.SPLIT:
            new_rows[o] = True
    for k in tr.m:
        assert not np_(tr.m[k]).reshape(tr.N, -1)[new_rows].any(), k
        assert np_(tr.m[k]).reshape(tr.N, -1)[~new_rows].any(), k
    assert not np_(tr.accum).any() and not np_(tr.count).any()
    s = np_(tr.scales)
    np.testing.assert_allclose(s, np.exp(np_(tr.raw["log_scales"])), rtol=2e-6)
    for _ in range(3):
        tr.step()
    torch.cuda.synchronize()
    assert np.isfinite(np_(tr.raw["means"])).all()


@pytest.mark.parametrize("strategy,absgrad", [("adc", False), ("adc", True), ("mcmc", False)])
def test_fit_lowers_the_loss(strategy, absgrad):
    """150 steps from a perturbed copy of a 2,000-Gaussian scene towards its
    own renders (4 views, 96x72) lower the mean L1 by at least 40 %."""
    from _gpu import np_
    from paper_2409_06765_amd.train import GaussianTrainer, TrainConfig
    deg = 1
    sc = scenes.scene_tiny(2000, sh_degree=deg, seed=91, log_scale_mean=-2.6)
    cams = scenes.cams_tiny(W=96, H=72, f=80.0, n_cams=4, seed=91)
    raw = _raw_from_scene(sc)
    gt = GaussianTrainer(raw, cams, torch.zeros((4, 72, 96, 3)), TrainConfig(strategy="none"), sh_degree=deg)
    targets = torch.stack([gt.render([v])[-1]["image"].reshape(72, 96, 3) for v in range(4)])
    g = np.random.default_rng(92)
    pert = dict(raw)
    pert["means"] = (raw["means"] + g.normal(0, 0.03, raw["means"].shape)).astype(np.float32)
    pert["sh"] = (raw["sh"] + g.normal(0, 0.15, raw["sh"].shape)).astype(np.float32)
    cfg = TrainConfig(strategy=strategy, absgrad=absgrad, views_per_step=1, refine_start=40, refine_every=40,
                      reset_every=10 ** 9, grad_threshold=8e-4 if absgrad else 2e-4, lr_means=1.6e-3,
                      lr_means_final=1.6e-3, seed=3)
    tr = GaussianTrainer(pert, cams, targets, cfg, sh_degree=deg)
    losses = [float(np_(tr.step())[0]) for _ in range(150)]
    first, last = np.mean(losses[:8]), np.mean(losses[-8:])
    _say(f"{strategy} absgrad={absgrad}: loss {first:.5f} -> {last:.5f}, N {2000} -> {tr.N}")
    assert last < 0.6 * first


# ---- full sizes, sampled -------------------------------------------------------------------------------------
def test_full_size_adam_and_l1_sampled():
    """The 1M-Gaussian SH-degree-3 parameter set in one Adam launch (59M
    values) and the L1 over 16 views of 1920x1080 (99.5M values): 20,000
    sampled elements of each output against the oracle, the whole loss
    against a float64 sum."""
    from _gpu import np_
    L = _L()
    N = 1_000_000
    g = np.random.default_rng(101)
    sizes = dict(means=3 * N, quats=4 * N, log_scales=3 * N, logits=N, sh=48 * N)
    kinds = dict(means=T.ACT_NONE, quats=T.ACT_NONE, log_scales=T.ACT_EXP, logits=T.ACT_SIGMOID, sh=T.ACT_NONE)
    host, groups = {}, []
    for k, n in sizes.items():
        a = dict(raw=g.normal(0, 1, n).astype(np.float32), grad=g.normal(0, 1e-3, n).astype(np.float32),
                 m=g.normal(0, 1e-4, n).astype(np.float32), v=(g.uniform(0, 1e-3, n) ** 2).astype(np.float32))
        host[k] = a
        groups.append(dict(param=_dev(a["raw"]), grad=_dev(a["grad"]), exp_avg=_dev(a["m"]), exp_avg_sq=_dev(a["v"]),
                           activated=torch.empty(n, device="cuda:0") if kinds[k] else None, lr=1e-3,
                           lr_rest=5e-5 if k == "sh" else 1e-3, row=48 if k == "sh" else 0,
                           row_first=3 if k == "sh" else 0, activation=kinds[k], reg=1e-8 if kinds[k] else 0.0))
    L.gsr_adam_step(groups, 3, 0.9, 0.999, 1e-15)
    torch.cuda.synchronize()
    b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
    for (k, a), d in zip(host.items(), groups):
        idx = np.sort(g.choice(sizes[k], 20_000, replace=False))
        lrs = T.group_lr(sizes[k], 1e-3, d["lr_rest"], d["row"], d["row_first"])[idx]
        g_raw = T.raw_gradient(a["raw"][idx], a["grad"][idx], kinds[k], d["reg"])
        p_ref, _, _ = T.adam(a["raw"][idx], g_raw, a["m"][idx], a["v"][idx], 3, lrs, b1, b2, 1e-15)
        p = np_(d["param"])[idx].astype(np.float64)
        ratio = np.abs(a["raw"][idx] - p_ref) / lrs
        assert np.all(np.abs(p - p_ref) <= 2e-5 * lrs * np.maximum(ratio, 1) + 3e-7 * np.abs(p_ref)), k
        if d["activated"] is not None:
            np.testing.assert_allclose(np_(d["activated"])[idx], T.activate(p_ref, kinds[k]), rtol=2e-6, err_msg=k)
    del groups
    torch.cuda.empty_cache()
    n = 16 * 1920 * 1080 * 3
    img = torch.rand(n, device="cuda:0", generator=torch.Generator(device="cuda:0").manual_seed(5))
    tgt = torch.rand(n, device="cuda:0", generator=torch.Generator(device="cuda:0").manual_seed(6))
    vi = torch.empty_like(img)
    loss = torch.empty(1, device="cuda:0")
    ws = torch.empty(L.workspace_bytes(L.GSR_OP_L1_LOSS, 0, 0, n), device="cuda:0", dtype=torch.uint8)
    scale = float(np.float32(1.0 / n))
    L.gsr_l1_loss(img, tgt, scale, vi, loss, ws)
    a, b = np_(img), np_(tgt)
    ref_loss, _ = T.l1_loss(a, b, scale)
    assert abs(float(np_(loss)[0]) - ref_loss) <= 1e-6 * ref_loss
    idx = g.choice(n, 20_000, replace=False)
    _, ref_v = T.l1_loss(a[idx], b[idx], scale)
    np.testing.assert_array_equal(np_(vi)[idx], ref_v.astype(np.float32))


def test_store_growth_and_list_rebuild_paths():
    """A refinement that outgrows the parameter stores (capacity factor 1)
    reallocates them and gives the same Gaussians as a run with room to
    spare; a step whose intersection buffer is too small rebuilds the lists
    and sends the forward and backward again, giving the same update as a
    step with the right capacity."""
    from _gpu import np_
    deg = 0
    sc = scenes.scene_tiny(600, sh_degree=deg, seed=83, log_scale_mean=-2.0)
    cams = scenes.cams_tiny(W=64, H=64, f=60.0, n_cams=2, seed=83)
    raw = _raw_from_scene(sc)
    g = np.random.default_rng(83)
    targets = g.uniform(0, 1, (2, 64, 64, 3)).astype(np.float32)
    kw = dict(strategy="adc", views_per_step=2, refine_start=0, refine_every=1, grad_threshold=2e-5,
              scale_threshold=0.08, reset_every=10 ** 9)
    tight = _trainer(raw, cams, targets, deg, capacity_factor=1.0, **kw)
    roomy = _trainer(raw, cams, targets, deg, capacity_factor=3.0, **kw)
    cap0 = tight._stores[0].cap
    tight.step()
    roomy.step()
    torch.cuda.synchronize()
    assert tight.N > cap0 and tight._stores[tight._cur].cap >= tight.N
    assert tight.N == roomy.N
    for k in tight.raw:
        np.testing.assert_allclose(np_(tight.raw[k]), np_(roomy.raw[k]), rtol=0, atol=1e-6, err_msg=k)
    # list rebuild: a capacity far below the count
    a = _trainer(raw, cams, targets, deg, strategy="none", views_per_step=2)
    b = _trainer(raw, cams, targets, deg, strategy="none", views_per_step=2)
    a.step()
    b.step()
    b.M_cap = 1024
    la = float(np_(a.step())[0])
    lb = float(np_(b.step())[0])
    torch.cuda.synchronize()
    assert b.last_M > 1024, b.last_M
    assert abs(la - lb) <= 1e-6 * la
    for k in a.raw:
        np.testing.assert_allclose(np_(b.raw[k]), np_(a.raw[k]), rtol=0, atol=1e-6, err_msg=k)


@pytest.mark.parametrize("absgrad", [False, True])
def test_densify_stats_from_rasterization_meta(absgrad):
    """The autograd entry point's meta feeds the ADC statistics: after
    rasterization() and backward, densify_stats_from_meta against the
    oracle's statistics of the oracle's backward."""
    from _gpu import np_, to_dev
    from paper_2409_06765_amd.rasterize import rasterization
    from paper_2409_06765_amd.train import densify_stats_from_meta
    sc = scenes.scene_tiny(700, sh_degree=1, seed=121, log_scale_mean=-2.3)
    cams = scenes.cams_tiny(W=72, H=56, f=55.0, n_cams=2, seed=121)
    t = {k: to_dev(sc[k]).requires_grad_(True) for k in ("means", "quats", "scales", "opacities", "sh")}
    img, alpha, meta = rasterization(t["means"], t["quats"], t["scales"], t["opacities"], t["sh"],
                                     to_dev(cams["viewmats"]), to_dev(cams["Ks"]), 72, 56, sh_degree=1,
                                     absgrad=absgrad, tile_cull=0)
    P = OracleParams(sh_degree=1)
    proj, isect, ras = O32.forward(P, sc, cams)
    g = np.random.default_rng(122)
    v_image = g.normal(size=ras["image"].shape).astype(np.float32)
    v_image[ras["flags"] != 0] = 0
    (img.reshape(-1, 3) * to_dev(v_image)).sum().backward()
    N = sc["means"].shape[0]
    accum = torch.zeros(N, device="cuda:0")
    count = torch.zeros(N, device="cuda:0", dtype=torch.int32)
    densify_stats_from_meta(meta, accum, count, absgrad=absgrad)
    torch.cuda.synchronize()
    o2 = O32.rasterize_bwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], cams["W"], cams["H"],
                           ras["final_T"], ras["last_ids"], v_image, absgrad=absgrad)
    v2 = o2["v_means2d_abs"] if absgrad else o2["v_means2d"]
    acc_ref, cnt_ref = T.densify_stats(proj["radii"], v2, cams["W"], cams["H"], 2.0, np.zeros(N),
                                       np.zeros(N, np.int64))
    np.testing.assert_array_equal(np_(count), cnt_ref)
    np.testing.assert_allclose(np_(accum), acc_ref, rtol=2e-3, atol=2e-3 * acc_ref.max())
