"""Forward + backward of a batch of views with every buffer allocated once.

``ViewPipeline`` holds the whole per-view state of one scene at fixed image
sizes: projected arrays, the binning workspaces, an intersection-list buffer
of fixed capacity, tile ranges and dispatch order, the compositing records,
the images and every gradient.  A step only enqueues library calls on one
stream: it allocates nothing and never waits for the host.  The library
writes each step's true intersection count to a device slot chosen by the
caller; ``counts()`` reads the slots back after the fact and ``overflowed()``
tells whether a step's lists exceeded the capacity (such a step built its
lists truncated, in bounds, and must be run again with a larger pipeline).

The stages are separate methods so that a caller can time them one by one;
``step`` runs them all.  The same object is what ``graph.CapturedStep``
records into a HIP graph.
"""
import torch

from . import _lib as L
from .rasterize import ORDER_MIN_TILES, _with, layout


class ViewPipeline:
    """scene: device tensors means [N,3], quats [N,4], scales [N,3] and
    opacities [N] (activated), sh [N,K,3] (or colours [N,3] with sh_degree
    -1); read at every step, so update them in place.  W, H: per-camera
    image sizes of the C views of one step.  capacity: entries of the
    intersection-list buffer.  slots: device count slots (one per step the
    caller wants to check later).  With plain RGB the 2D gradients are kept
    as records (``grad_rec`` [C,N,9]) and ``g2`` holds strided views of
    their fields; ``records=False`` keeps four arrays instead."""

    def __init__(self, p, scene, W, H, capacity, slots=1, absgrad=False, stream=None, records=None):
        # plain RGB keeps each (camera, Gaussian)'s 2D gradients in one record (params.grad_records): the
        # compositing backward's atomics for a Gaussian then touch one or two cache lines, not four arrays
        # (records=False asks for the four arrays)
        plain = p.render_depth == 0 and not p.colors_shared
        self.records = plain if records is None else bool(records) and plain
        p = _with(p, grad_records=1) if self.records else p
        self.p = p
        self.scene = scene
        self.W, self.H = [int(w) for w in W], [int(h) for h in H]
        C, N = len(self.W), int(scene["means"].shape[0])
        self.C, self.N = C, N
        d = scene["means"].device
        self.device = d
        self.stream = stream
        self.capacity = int(capacity)
        pix_off, tile_off = layout(self.W, self.H)
        self.P, self.T = pix_off[-1], tile_off[-1]
        f32 = dict(device=d, dtype=torch.float32)
        i32 = dict(device=d, dtype=torch.int32)
        u8 = dict(device=d, dtype=torch.uint8)
        self.vm = torch.zeros((C, 4, 4), **f32)
        self.Ks = torch.zeros((C, 3, 3), **f32)
        self.cam = (self.vm, self.Ks)
        self.proj = dict(means2d=torch.empty((C, N, 2), **f32), conics=torch.empty((C, N, 3), **f32),
                         radii=torch.empty((C, N), **i32), depths=torch.empty((C, N), **f32),
                         colors=torch.empty((C, N, 3), **f32),
                         comps=torch.empty((C, N), **f32) if p.antialiased else None)
        self.totals = torch.zeros(max(int(slots), 1), device=d, dtype=torch.int64)
        self.ws_prep = torch.empty(max(L.workspace_bytes(L.GSR_OP_BIN_PREPARE, C, N, 0), 1), **u8)
        self.ws_fin = torch.empty(max(L.workspace_bytes(L.GSR_OP_BIN_FINISH, C, N, self.capacity), 1), **u8)
        self.ids = torch.empty(max(self.capacity, 1), **i32)
        self.ranges = torch.empty((max(self.T, 1), 2), **i32)
        self.order = torch.empty(max(self.T, 1), **i32) if self.T >= ORDER_MIN_TILES else None
        self.ws_order = torch.empty(max(L.workspace_bytes(L.GSR_OP_TILE_ORDER, 0, 0, 0), 1), **u8)
        self.ws_raster = torch.empty(max(L.workspace_bytes(L.GSR_OP_RASTERIZE, C, N, 0), 1), **u8)
        self.image = torch.empty((self.P, 3), **f32)
        self.alpha = torch.empty(self.P, **f32)
        self.final_T = torch.empty(self.P, **f32)
        self.last_ids = torch.empty(self.P, **i32)
        if self.records:
            sizes = dict(records=(C, N, L.GSR_GRAD_RECORD))
        else:
            sizes = dict(v_means2d=(C, N, 2), v_conics=(C, N, 3), v_colors=(C, N, 3), v_opacities=(C, N))
        if absgrad:
            sizes["v_means2d_abs"] = (C, N, 2)
        total = sum(int(torch.Size(s).numel()) for s in sizes.values())
        self.grad_flat = torch.empty(max(total, 1), **f32)
        self.g2, o = {}, 0
        for k, s in sizes.items():
            m = int(torch.Size(s).numel())
            self.g2[k] = self.grad_flat[o:o + m].view(s)
            o += m
        self.grad_rec = self.g2.pop("records", None)
        if self.records:   # the fields of the records, as strided views
            r = self.grad_rec
            self.g2.update(v_means2d=r[..., 0:2], v_conics=r[..., 2:5], v_colors=r[..., 5:8], v_opacities=r[..., 8])
        self.g2.setdefault("v_means2d_abs", None)
        sc = scene
        self.g3 = dict(v_means=torch.empty_like(sc["means"]), v_quats=torch.empty_like(sc["quats"]),
                       v_scales=torch.empty_like(sc["scales"]), v_opacities=torch.empty_like(sc["opacities"]),
                       v_sh=torch.empty_like(sc["sh"]))

    # -- stages -----------------------------------------------------------------
    def set_cameras(self, viewmats, Ks, copy=True):
        """The step's cameras ([C,4,4], [C,3,3] device tensors): copied into
        the pipeline's own slots (what a captured graph reads), or with
        ``copy=False`` used where they are (no launch; keep them alive and
        unchanged until the step has run)."""
        if copy:
            self.vm.copy_(viewmats)
            self.Ks.copy_(Ks)
            self.cam = (self.vm, self.Ks)
        else:
            self.cam = (viewmats.contiguous(), Ks.contiguous())

    def project(self):
        sc, pr = self.scene, self.proj
        L.gsr_project_fwd(self.p, self.C, self.N, self.W, self.H, sc["means"], sc["quats"], sc["scales"],
                          sc["opacities"], sc["sh"], *self.cam, pr["means2d"], pr["conics"], pr["radii"],
                          pr["depths"], pr["colors"], pr["comps"], stream=self.stream)

    def bin(self, slot=0):
        """Tile lists in depth order (no host wait); the true count goes to
        count slot ``slot``."""
        pr, sc = self.proj, self.scene
        cull = (pr["conics"], sc["opacities"], pr["comps"])
        L.gsr_bin_prepare(self.p, self.C, self.N, self.W, self.H, pr["means2d"], pr["radii"], pr["depths"], *cull,
                          self.totals[slot:slot + 1], self.ws_prep, sync=False, stream=self.stream)
        L.gsr_bin_finish(self.p, self.C, self.N, self.W, self.H, pr["means2d"], pr["radii"], pr["depths"], *cull,
                         self.capacity, self.ids, self.ranges, None, self.ws_prep, self.ws_fin, stream=self.stream)
        if self.order is not None:
            L.gsr_tile_order(self.T, self.ranges, self.order, self.ws_order, stream=self.stream)

    def rasterize_forward(self):
        pr, sc = self.proj, self.scene
        L.gsr_rasterize_fwd(self.p, self.C, self.N, 3, self.W, self.H, pr["means2d"], pr["conics"], pr["colors"],
                            pr["depths"], sc["opacities"], pr["comps"], None, self.ranges, self.ids, self.order,
                            self.image, self.alpha, self.final_T, self.last_ids, None, ws=self.ws_raster,
                            stream=self.stream)

    def zero_grads(self):
        L.gsr_fill_zero(self.grad_flat, stream=self.stream)

    def rasterize_backward(self, v_image, v_alpha=None):
        """The compositing backward alone: the records the forward packed are
        reused and the gradients (zeroed by ``zero_grads``) are added to."""
        pr, sc, g = self.proj, self.scene, self.g2
        g4 = self._grad_args()
        L.gsr_rasterize_bwd(self.p, self.C, self.N, 3, self.W, self.H, pr["means2d"], pr["conics"], pr["colors"],
                            pr["depths"], sc["opacities"], pr["comps"], None, self.ranges, self.ids, self.order,
                            self.image, self.final_T, self.last_ids, v_image, v_alpha, g4[0], g4[1], g4[2], None,
                            g4[3], g["v_means2d_abs"], ws=self.ws_raster,
                            flags=L.GSR_BWD_ACCUMULATE | L.GSR_BWD_PACKED, stream=self.stream)

    def _grad_args(self):
        """v_means2d, v_conics, v_colors, v_opacities as the library takes them: the records and three
        NULLs, or the four arrays."""
        g = self.g2
        if self.records:
            return self.grad_rec, None, None, None
        return g["v_means2d"], g["v_conics"], g["v_colors"], g["v_opacities"]

    def project_backward(self):
        sc, pr, g3 = self.scene, self.proj, self.g3
        g4 = self._grad_args()
        L.gsr_project_bwd(self.p, self.C, self.N, self.W, self.H, sc["means"], sc["quats"], sc["scales"],
                          sc["opacities"], sc["sh"], *self.cam, pr["radii"], pr["comps"], *g4, None,
                          g3["v_means"], g3["v_quats"], g3["v_scales"], g3["v_opacities"], g3["v_sh"],
                          stream=self.stream)

    def step(self, v_image, slot=0, v_alpha=None):
        """The whole forward + backward for the cameras set last."""
        self.project()
        self.bin(slot)
        self.rasterize_forward()
        self.zero_grads()
        self.rasterize_backward(v_image, v_alpha)
        self.project_backward()

    # -- after the fact -----------------------------------------------------------
    def counts(self):
        """True intersection counts of the slots (waits for the device)."""
        return [int(x) for x in self.totals.cpu()]

    def overflowed(self, slots=None):
        c = self.counts()
        return any(c[i] > self.capacity for i in (range(len(c)) if slots is None else slots))

    def ids_view(self, slot=0):
        """The sorted ids of the step that wrote ``slot`` (waits)."""
        M = self.counts()[slot]
        return self.ids[:min(M, self.capacity)]
