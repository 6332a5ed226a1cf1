"""Fitting Gaussians to target images with the rasterizer: a synthetic
training loop with the paper's densification strategies (ADC, Absgrad, MCMC
noise).

Every step runs through the C ABI: projection, binning, compositing, the L1
loss, both backward passes, the ADC statistics, one fused Adam launch over
all raw parameters (the activation chain and the MCMC regularisers folded
in, the activated scales and opacities written for the next step), the
MCMC noise on the centres, and, at refinement steps, the ADC plan / apply
and the opacity reset.  torch only allocates device memory and draws the
standard normal numbers the split and the noise take as inputs.

Raw parameters: means [N,3], quats [N,4] (w,x,y,z, normalised by the
projection), log_scales [N,3], logits [N], sh [N,K,3].
"""
import math
from dataclasses import dataclass

import torch

from . import _lib as L
from . import rasterize as R

PARAMS = ("means", "quats", "log_scales", "logits", "sh")


@dataclass
class TrainConfig:
    """Hyper-parameters.  The thresholds of the ADC strategy are the
    paper's (gradient 0.0002, scale 0.01 of the scene extent, opacity
    0.005); learning rates, schedules and the MCMC constants are the values
    the cited 3D Gaussian Splatting and MCMC works use, since the paper
    states none."""
    strategy: str = "adc"          # "adc", "mcmc" or "none"
    views_per_step: int = 1
    lr_means: float = 1.6e-4       # times scene_extent, decayed exponentially to lr_means_final
    lr_means_final: float = 1.6e-6
    lr_decay_steps: int = 30_000
    lr_quats: float = 1e-3
    lr_scales: float = 5e-3
    lr_opacities: float = 5e-2
    lr_sh: float = 2.5e-3          # degree-0 coefficients
    lr_sh_rest: float = 2.5e-3 / 20
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    absgrad: bool = False
    grad_threshold: float = 2e-4
    scale_threshold: float = 0.01  # times scene_extent
    prune_opacity: float = 0.005
    refine_start: int = 500
    refine_stop: int = 15_000
    refine_every: int = 100
    reset_every: int = 3000
    reset_value: float = 0.01
    split_shrink: float = 1.6
    noise_lr: float = 5e5
    noise_k: float = 100.0
    noise_t: float = 0.005
    opacity_reg: float = 0.01      # MCMC only
    scale_reg: float = 0.01        # MCMC only
    capacity_factor: float = 1.5   # ADC: parameter rows allocated per starting Gaussian
    seed: int = 0


def _dev(x, device):
    return torch.as_tensor(x, dtype=torch.float32).to(device).contiguous()


class _ParamStore:
    """Raw parameters and Adam moments of every tensor at a fixed row
    capacity; the trainer works on views of the first N rows, so a
    refinement writes into the other store instead of allocating."""

    def __init__(self, rows, cap, device):
        self.cap = cap
        mk = lambda: {k: torch.zeros((cap,) + shape, device=device, dtype=torch.float32) for k, shape in rows.items()}
        self.raw, self.m, self.v = mk(), mk(), mk()


class GaussianTrainer:
    """Holds the raw parameters, Adam moments and ADC statistics on one GPU
    and runs optimisation steps against target images of the training views.

    cams: viewmats [V,4,4], Ks [V,3,3], W [V], H [V] (all views one size);
    targets [V,H,W,3] on the device."""

    def __init__(self, raw, cams, targets, cfg=None, sh_degree=-1, scene_extent=1.0, params=None, device="cuda"):
        self.cfg = cfg or TrainConfig()
        if self.cfg.strategy not in ("adc", "mcmc", "none"):
            raise ValueError("strategy must be adc, mcmc or none")
        self.device = torch.device(device)
        self.p = params if params is not None else R.make_params(sh_degree=sh_degree)
        self.sh_degree = sh_degree
        self.extent = float(scene_extent)
        self.raw = {k: _dev(raw[k], self.device) for k in PARAMS}
        self.viewmats = _dev(cams["viewmats"], self.device)
        self.Ks = _dev(cams["Ks"], self.device)
        self.W = [int(w) for w in cams["W"]]
        self.H = [int(h) for h in cams["H"]]
        if len(set(self.W)) != 1 or len(set(self.H)) != 1:
            raise ValueError("training views must share one image size")
        self.targets = targets.to(self.device, torch.float32).contiguous()
        self.V = self.viewmats.shape[0]
        if tuple(self.targets.shape) != (self.V, self.H[0], self.W[0], 3):
            raise ValueError("targets must be [V, H, W, 3]")
        self.step_no = 0
        self.gen = torch.Generator(device=self.device)
        self.gen.manual_seed(int(self.cfg.seed))
        self.l1_ws = torch.empty(L.workspace_bytes(L.GSR_OP_L1_LOSS, 0, 0, 0), device=self.device, dtype=torch.uint8)
        self.M_cap = 0                 # intersection-list capacity learned from earlier steps
        N = self.raw["means"].shape[0]
        self._rows = {k: tuple(v.shape[1:]) for k, v in self.raw.items()}
        grow = self.cfg.capacity_factor if self.cfg.strategy == "adc" else 1.0
        first = _ParamStore(self._rows, max(int(N * grow), N, 1), self.device)
        for k in PARAMS:
            first.raw[k][:N].copy_(self.raw[k])
        # ADC refinements write into the second store: allocate it (and the
        # plan's scratch) now, so a refinement step allocates nothing
        second = _ParamStore(self._rows, first.cap, self.device) if self.cfg.strategy == "adc" else None
        self._stores, self._cur = [first, second], 0
        self._act_scales = self._act_opac = None
        self._scratch(first.cap)
        self._bind(N)

    # ---- state -----------------------------------------------------------------------
    @property
    def N(self):
        return self.raw["means"].shape[0]

    def _bind(self, N):
        """Point the working tensors at the first N rows of the current
        store, recompute the activated values and clear the statistics."""
        st = self._stores[self._cur]
        self.raw = {k: st.raw[k][:N] for k in PARAMS}
        self.m = {k: st.m[k][:N] for k in PARAMS}
        self.v = {k: st.v[k][:N] for k in PARAMS}
        if self._act_scales is None or self._act_scales.shape[0] < N:
            cap = st.cap
            self._act_scales = torch.empty((cap, 3), device=self.device, dtype=torch.float32)
            self._act_opac = torch.empty(cap, device=self.device, dtype=torch.float32)
            self._accum = torch.zeros(cap, device=self.device, dtype=torch.float32)
            self._count = torch.zeros(cap, device=self.device, dtype=torch.int32)
        self.scales, self.opacities = self._act_scales[:N], self._act_opac[:N]
        self.accum, self.count = self._accum[:N], self._count[:N]
        L.gsr_activate(self.raw["log_scales"], L.GSR_ACT_EXP, self.scales)
        L.gsr_activate(self.raw["logits"], L.GSR_ACT_SIGMOID, self.opacities)
        self._reset_stats()

    def _scratch(self, cap):
        """Per-Gaussian scratch of the refinement and noise draws."""
        d = self.device
        self._normals = torch.empty((cap, 2, 3), device=d, dtype=torch.float32)
        if self.cfg.strategy == "adc":
            self._action = torch.empty(cap, device=d, dtype=torch.int32)
            self._offsets = torch.empty(cap + 1, device=d, dtype=torch.int64)
            self._plan_ws = torch.empty(max(L.workspace_bytes(L.GSR_OP_DENSIFY_PLAN, 0, cap, 0), 1), device=d,
                                        dtype=torch.uint8)
        self._scratch_cap = cap

    def _reset_stats(self):
        self.accum.zero_()
        self.count.zero_()

    def activated_scene(self):
        return dict(means=self.raw["means"], quats=self.raw["quats"], scales=self.scales, opacities=self.opacities,
                    sh=self.raw["sh"])

    # ---- schedule ----------------------------------------------------------------------
    def lr_means(self, step):
        c = self.cfg
        t = min(max(step, 0) / max(c.lr_decay_steps, 1), 1.0)
        return self.extent * math.exp((1 - t) * math.log(c.lr_means) + t * math.log(c.lr_means_final))

    def views_of(self, step):
        """Views of step t (1-based): a fixed cycle over the training views."""
        k = self.cfg.views_per_step
        return [((step - 1) * k + j) % self.V for j in range(k)]

    # ---- one step ----------------------------------------------------------------------------
    def _pick(self, t, views):
        """Rows of a per-view tensor: a view of it when the views are
        consecutive (no gather launch)."""
        if views == list(range(views[0], views[0] + len(views))):
            return t[views[0]:views[0] + len(views)]
        return t[views].contiguous()

    def render(self, views, check=True):
        vm = self._pick(self.viewmats, views)
        Ks = self._pick(self.Ks, views)
        C = len(views)
        W, H = [self.W[0]] * C, [self.H[0]] * C
        sc = self.activated_scene()
        proj = R.project(self.p, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], vm, Ks, W, H)
        isect = R.intersect(self.p, proj, W, H, capacity=self.M_cap or None)
        fwd = R.rasterize_forward(self.p, proj, sc["opacities"], isect, W, H)
        if check and isect.check():
            fwd = R.rasterize_forward(self.p, proj, sc["opacities"], isect, W, H)
        return vm, Ks, W, H, proj, isect, fwd

    def _gradients(self, views, vm, Ks, W, H, proj, isect, fwd):
        sc = self.activated_scene()
        image = fwd["image"]
        target = self._pick(self.targets, views).reshape(image.shape)
        v_image = torch.empty_like(image)
        loss = torch.empty(1, device=self.device, dtype=torch.float32)
        L.gsr_l1_loss(image, target, 1.0 / image.numel(), v_image, loss, self.l1_ws)
        # the 2D gradients as records (one or two cache lines per Gaussian for the backward's atomics)
        g2 = R.rasterize_backward(self.p, proj, sc["opacities"], isect, W, H, fwd, v_image,
                                  absgrad=self.cfg.absgrad and self.cfg.strategy == "adc",
                                  records=self.p.render_depth == 0 and not self.p.colors_shared)
        g3 = R.project_backward(self.p, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], vm, Ks, W,
                                H, proj, g2)
        return loss, g2, g3

    def step(self):
        """One optimisation step; returns the step's L1 loss as a device
        scalar.  The host does not wait inside the step: the intersection
        count is resolved once the backward is queued, and only a list that
        overflowed its buffer (rebuilt with the true count) sends the
        forward and backward again, before anything is updated."""
        c = self.cfg
        self.step_no += 1
        t = self.step_no
        views = self.views_of(t)
        C = len(views)
        vm, Ks, W, H, proj, isect, fwd = self.render(views, check=False)
        loss, g2, g3 = self._gradients(views, vm, Ks, W, H, proj, isect, fwd)
        if isect.check():
            fwd = R.rasterize_forward(self.p, proj, self.opacities, isect, W, H)
            loss, g2, g3 = self._gradients(views, vm, Ks, W, H, proj, isect, fwd)
        self.last_M = isect["M"]
        self.M_cap = max(self.M_cap, int(self.last_M * 1.25) + 1024)
        self.last_grads = g3
        if c.strategy == "adc" and t < c.refine_stop:
            v2 = g2["v_means2d_abs"] if c.absgrad else g2["v_means2d"].contiguous()   # records: a strided view
            L.gsr_densify_stats(C, self.N, W, H, proj["radii"], v2, float(C), self.accum, self.count)
        self._adam(t, g3)
        if c.strategy == "mcmc":
            eta = self._normals.view(-1, 3)[:self.N]
            torch.randn(eta.shape, generator=self.gen, device=self.device, dtype=torch.float32, out=eta)
            L.gsr_mcmc_noise(self.N, self.raw["means"], self.raw["quats"], self.scales, self.opacities, eta,
                             c.noise_lr * self.lr_means(t), c.noise_k, c.noise_t)
        if c.strategy == "adc" and t < c.refine_stop:
            if t > c.refine_start and t % c.refine_every == 0:
                self.densify()
            if t % c.reset_every == 0:
                self.reset_opacities()
        return loss

    def _adam(self, t, g3):
        c = self.cfg
        N = self.N
        mcmc = c.strategy == "mcmc"
        sh = self.raw["sh"]
        row = sh.shape[1] * 3 if sh.dim() == 3 else 0
        groups = [
            dict(param=self.raw["means"], grad=g3["v_means"], lr=self.lr_means(t)),
            dict(param=self.raw["quats"], grad=g3["v_quats"], lr=c.lr_quats),
            dict(param=self.raw["log_scales"], grad=g3["v_scales"], lr=c.lr_scales, activation=L.GSR_ACT_EXP,
                 activated=self.scales, reg=(c.scale_reg / max(3 * N, 1)) if mcmc else 0.0),
            dict(param=self.raw["logits"], grad=g3["v_opacities"], lr=c.lr_opacities, activation=L.GSR_ACT_SIGMOID,
                 activated=self.opacities, reg=(c.opacity_reg / max(N, 1)) if mcmc else 0.0),
            dict(param=sh, grad=g3["v_sh"], lr=c.lr_sh, lr_rest=c.lr_sh_rest, row=row, row_first=3 if row else 0),
        ]
        names = ("means", "quats", "log_scales", "logits", "sh")
        for g, k in zip(groups, names):
            g["exp_avg"], g["exp_avg_sq"] = self.m[k], self.v[k]
        L.gsr_adam_step(groups, t, c.beta1, c.beta2, c.eps)

    # ---- ADC ---------------------------------------------------------------------------------
    def densify(self):
        """Split, clone and prune by the accumulated statistics (waits for the
        new count), then clear the statistics."""
        c = self.cfg
        N = self.N
        if self._scratch_cap < N:
            self._scratch(self._stores[self._cur].cap)
        action, offsets = self._action[:N], self._offsets[:N + 1]
        n_new = L.gsr_densify_plan(N, self.accum, self.count, self.scales, self.opacities, c.grad_threshold,
                                   c.scale_threshold * self.extent, c.prune_opacity, action, offsets, self._plan_ws)
        self.last_plan = (action, offsets)
        normals = self._normals[:N]
        torch.randn(normals.shape, generator=self.gen, device=self.device, dtype=torch.float32, out=normals)
        kinds = dict(means=L.GSR_COLUMN_MEANS, quats=L.GSR_COLUMN_COPY, log_scales=L.GSR_COLUMN_LOG_SCALES,
                     logits=L.GSR_COLUMN_COPY, sh=L.GSR_COLUMN_COPY)
        nxt = 1 - self._cur
        st = self._stores[nxt]
        if st is None or st.cap < n_new:
            self._stores[nxt] = None
            st = self._stores[nxt] = _ParamStore(self._rows, max(int(n_new * c.capacity_factor), n_new, 1),
                                                 self.device)
        cols = [(self.raw[k], st.raw[k][:n_new], kinds[k]) for k in PARAMS]
        cols += [(self.m[k], st.m[k][:n_new], L.GSR_COLUMN_STATE) for k in PARAMS]
        cols += [(self.v[k], st.v[k][:n_new], L.GSR_COLUMN_STATE) for k in PARAMS]
        if n_new > 0:
            L.gsr_densify_apply(N, action, offsets, self.raw["quats"], self.raw["log_scales"], normals,
                                c.split_shrink, cols)
        self._cur = nxt
        self._bind(n_new)
        return n_new

    def reset_opacities(self):
        L.gsr_opacity_reset(self.N, self.raw["logits"], self.m["logits"], self.v["logits"], self.opacities,
                            self.cfg.reset_value)


def densify_stats_from_meta(meta, accum, count, absgrad=False, views_in_loss=None):
    """ADC statistics from the ``meta`` of ``rasterize.rasterization`` after
    the backward pass (the way a training loop built on the autograd function
    gathers them): adds to ``accum`` [N] and ``count`` [N] (int32) through
    gsr_densify_stats.  ``views_in_loss``: the number of views the loss
    averaged over (default: the views rendered)."""
    radii = meta["radii"]
    C, N = radii.shape
    v2 = meta["means2d_absgrad"] if absgrad else meta["means2d_grad"]
    scale = float(C if views_in_loss is None else views_in_loss)
    L.gsr_densify_stats(C, N, meta["width"], meta["height"], radii, v2, scale, accum, count)
