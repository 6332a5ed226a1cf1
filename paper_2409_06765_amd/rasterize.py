"""Differentiable tile rasterization on top of the C ABI.

``project`` / ``intersect`` / ``rasterize_forward`` / ``rasterize_backward`` /
``project_backward`` allocate outputs with torch and call the HIP library;
``RasterizeGaussians`` chains them in a ``torch.autograd.Function`` and
``rasterization`` mirrors the paper's 13-line example, returning
(image [C,H,W,3], alpha [C,H,W,1], meta).  The backward recomputes alphas
from the saved per-pixel last index and final transmittance instead of
keeping per-pixel lists.
"""
import math

import torch

from . import _lib as L


DEPTH_MODES = {"none": L.GSR_DEPTH_NONE, "accumulated": L.GSR_DEPTH_ACCUMULATED, "expected": L.GSR_DEPTH_EXPECTED}
RENDER_MODES = {"RGB": (True, "none"), "D": (False, "accumulated"), "ED": (False, "expected"),
                "RGB+D": (True, "accumulated"), "RGB+ED": (True, "expected")}


def make_params(sh_degree=-1, antialiased=False, render_depth="none", **kw):
    """Library parameters; ``render_depth`` is "none", "accumulated" or
    "expected" (a depth channel after the features)."""
    return L.default_params(sh_degree=int(sh_degree), antialiased=int(bool(antialiased)),
                            render_depth=DEPTH_MODES[render_depth] if isinstance(render_depth, str)
                            else int(render_depth), **kw)


def _with(p, **fields):
    q = L.gsr_params.from_buffer_copy(p)
    for k, v in fields.items():
        setattr(q, k, v)
    return q


def _dev(t):
    return t.device


def _sizes_per_cam(C, width, height):
    W = [int(width)] * C if isinstance(width, int) else [int(w) for w in width]
    H = [int(height)] * C if isinstance(height, int) else [int(h) for h in height]
    if len(W) != C or len(H) != C:
        raise ValueError("one width and height per camera")
    return W, H


def layout(W, H, tile=16):
    """Per-camera pixel offsets, tile offsets, total pixels and tiles."""
    pix_off, tile_off = [0], [0]
    for w, h in zip(W, H):
        pix_off.append(pix_off[-1] + w * h)
        tile_off.append(tile_off[-1] + ((w + tile - 1) // tile) * ((h + tile - 1) // tile))
    return pix_off, tile_off


def project(p, means, quats, scales, opacities, sh_or_colors, viewmats, Ks, W, H, stream=None):
    """Projection; ``sh_or_colors`` None (direct colours only) skips the colour
    output: the rasterizer then takes features of its own."""
    C, N = viewmats.shape[0], means.shape[0]
    d = _dev(means)
    f = dict(device=d, dtype=torch.float32)
    out = dict(means2d=torch.empty((C, N, 2), **f), conics=torch.empty((C, N, 3), **f),
               radii=torch.empty((C, N), device=d, dtype=torch.int32), depths=torch.empty((C, N), **f),
               colors=torch.empty((C, N, 3), **f) if sh_or_colors is not None else None,
               comps=torch.empty((C, N), **f) if p.antialiased else None,
               opacities=opacities)          # the binning's tile culling reads them
    L.gsr_project_fwd(p, C, N, W, H, means, quats, scales, opacities, sh_or_colors, viewmats, Ks,
                      out["means2d"], out["conics"], out["radii"], out["depths"], out["colors"], out["comps"],
                      stream=stream)
    return out


class Intersections(dict):
    """Result of ``intersect``.  With the binning route the intersection
    count M stays on the device while the lists are built in a buffer of a
    capacity chosen from earlier calls; reading ``M`` (or ``ids``/``keys``)
    waits only for the count's copy to host memory, and a count above the
    capacity rebuilds the lists (one extra synchronous pass, rare)."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self._pending = None          # (event, pinned count, capacity, shape key, rebuild) until resolved
        self.rebuilt = False

    def _resolve(self):
        if self._pending is None:
            return
        ev, pinned, cap, shape, rebuild = self._pending
        self._pending = None
        ev.synchronize()
        M = int(pinned[0])
        _CAPACITY.note(shape, M)
        if M > cap:
            dict.update(self, rebuild(M))
            self.rebuilt = True
        self._set_count(M)

    def _set_count(self, M):
        dict.__setitem__(self, "M", M)
        dict.__setitem__(self, "ids", self["ids_buf"][:M])
        if self.get("keys_buf") is not None:
            dict.__setitem__(self, "keys", self["keys_buf"][:M])

    def check(self):
        """Resolves the count; True when the lists had to be rebuilt, in
        which case work already launched on them must be launched again."""
        self._resolve()
        return self.rebuilt

    def __getitem__(self, k):
        if k in ("M", "ids", "keys"):
            self._resolve()
        return dict.__getitem__(self, k)


class _Capacity:
    """Intersection-buffer capacity per (device, cameras, Gaussians, image
    sizes): 1.25 x the largest count seen, at least 2^16."""

    def __init__(self):
        self.cap = {}

    def get(self, shape):
        return self.cap.get(shape, 0)

    def note(self, shape, M):
        if shape is not None:
            self.cap[shape] = max(self.cap.get(shape, 0), int(M * 1.25) + 1024, 1 << 16)


_CAPACITY = _Capacity()


def intersect(p, proj, W, H, method="bin", want_keys=False, stream=None, capacity=None, defer=False):
    """Per-tile depth-sorted lists.

    method="bin" (default): depth order of the projected Gaussians, then a
    stable sort of 32-bit tile keys (gsr_bin_prepare / gsr_bin_finish), with
    the tiles no pixel can see dropped when ``p.tile_cull`` is set.  The
    host does not wait for the intersection count: the lists are built in a
    buffer of ``capacity`` entries (default: from earlier calls of the same
    shape; the first call of a shape waits for the count) and the count is
    checked when M is read.  ``defer`` (with a capacity): no count check at
    all; the count stays in ``total_dev`` for the caller to compare with the
    capacity (what a captured graph needs).  method="keys64": count (waits for it), emit
    64-bit keys, stable radix sort, ranges of whole squares.  Without tile
    culling both give the same ids and ranges."""
    C, N = proj["radii"].shape
    d = proj["radii"].device
    _, tile_off = layout(W, H)
    total_tiles = tile_off[-1]
    total = torch.empty(1, device=d, dtype=torch.int64)
    ranges = torch.empty((max(total_tiles, 1), 2), device=d, dtype=torch.int32)
    key_bits = 32 + max(total_tiles - 1, 0).bit_length()
    if method == "bin":
        shape = (str(d), C, N, tuple(int(w) for w in W), tuple(int(h) for h in H), int(p.tile_cull))
        wsp = torch.empty(max(L.workspace_bytes(L.GSR_OP_BIN_PREPARE, C, N, 0), 1), device=d, dtype=torch.uint8)
        cap = int(capacity) if capacity is not None else _CAPACITY.get(shape)
        cull = (proj["conics"], proj.get("opacities"), proj.get("comps"))
        M_known = L.gsr_bin_prepare(p, C, N, W, H, proj["means2d"], proj["radii"], proj["depths"], *cull, total, wsp,
                                    sync=cap == 0, stream=stream)
        if M_known is not None:
            _CAPACITY.note(shape, M_known)
            cap = M_known

        def build(cap):
            ids = torch.empty(max(cap, 1), device=d, dtype=torch.int32)
            keys = torch.empty(max(cap, 1), device=d, dtype=torch.uint64) if want_keys else None
            wsf = torch.empty(max(L.workspace_bytes(L.GSR_OP_BIN_FINISH, C, N, cap), 1), device=d,
                              dtype=torch.uint8)
            L.gsr_bin_finish(p, C, N, W, H, proj["means2d"], proj["radii"], proj["depths"], *cull, cap, ids, ranges,
                             keys, wsp, wsf, stream=stream)
            return dict(ids_buf=ids, keys_buf=keys, order=tile_order(ranges, total_tiles, stream))

        out = Intersections(ranges=ranges, total_tiles=total_tiles, key_bits=key_bits, total_dev=total,
                            **build(cap))
        if M_known is not None:
            out._set_count(M_known)
            return out
        if defer:
            out["capacity"] = cap
            return out
        s = stream if stream is not None else torch.cuda.current_stream(d)
        pinned = torch.empty(1, dtype=torch.int64, pin_memory=True)
        with torch.cuda.stream(s):
            pinned.copy_(total, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)

        def rebuild(M):
            # the capacity was too small: wait for the stream, rebuild with the true count
            s.synchronize()
            return build(M)
        out._pending = (ev, pinned, cap, shape, rebuild)
        return out
    counts = torch.empty((C, N), device=d, dtype=torch.int32)
    offsets = torch.empty((C, N), device=d, dtype=torch.int64)
    ws = torch.empty(max(L.workspace_bytes(L.GSR_OP_INTERSECT_COUNT, C, N, 0), 1), device=d, dtype=torch.uint8)
    M = L.gsr_intersect_count(p, C, N, W, H, proj["means2d"], proj["radii"], counts, offsets, total, ws,
                              sync=True, stream=stream)
    keys = torch.empty(max(M, 1), device=d, dtype=torch.uint64)
    ids = torch.empty(max(M, 1), device=d, dtype=torch.int32)
    L.gsr_intersect_emit(p, C, N, W, H, proj["means2d"], proj["radii"], proj["depths"], offsets, M, keys, ids,
                         stream=stream)
    if M > 1:
        keys_alt = torch.empty_like(keys)
        ids_alt = torch.empty_like(ids)
        sws = torch.empty(max(L.workspace_bytes(L.GSR_OP_SORT, 0, 0, M), 1), device=d, dtype=torch.uint8)
        L.gsr_sort_pairs(M, key_bits, keys, ids, keys_alt, ids_alt, sws, stream=stream)
    L.gsr_tile_ranges(M, keys, total_tiles, ranges, stream=stream)
    # keys/ids are views of length M; the *_buf tensors (length max(M, 1)) are
    # what the library is handed, so a pointer is never NULL when M == 0
    return dict(counts=counts, offsets=offsets, M=M, keys=keys[:M], ids=ids[:M], ids_buf=ids, keys_buf=keys,
                ranges=ranges, total_tiles=total_tiles, key_bits=key_bits,
                order=tile_order(ranges, total_tiles, stream))


# Below this many tiles every compositing block of a launch runs at once on
# the 256 CUs, so the dispatch order changes nothing and is not computed.
ORDER_MIN_TILES = 1024


def tile_order(ranges, total_tiles, stream=None):
    """Launch order of the compositing blocks: tiles by list length, longest
    first (gsr_tile_order); None (tile id order) for fewer than
    ORDER_MIN_TILES tiles."""
    if total_tiles < ORDER_MIN_TILES:
        return None
    d = ranges.device
    order = torch.empty(max(total_tiles, 1), device=d, dtype=torch.int32)
    ws = torch.empty(max(L.workspace_bytes(L.GSR_OP_TILE_ORDER, 0, 0, 0), 1), device=d, dtype=torch.uint8)
    L.gsr_tile_order(total_tiles, ranges, order, ws, stream=stream)
    return order


def raster_workspace(C, N, device):
    return torch.empty(max(L.workspace_bytes(L.GSR_OP_RASTERIZE, C, N, 0), 1), device=device, dtype=torch.uint8)


def _features(p, proj, features):
    """(params, D, feature tensor) for the rasterizer: the projected colours
    [C,N,3] by default, else ``features`` [C,N,D] or [N,D] (shared by all
    cameras); D = 0 (a [..,0] tensor) renders the depth channel alone."""
    if features is None:
        if proj.get("colors") is None:
            raise ValueError("no projected colours: pass features")
        return _with(p, colors_shared=0), 3, proj["colors"]
    C, N = proj["radii"].shape
    if features.dim() == 2 and features.shape[0] == N:
        shared = 1
    elif features.dim() == 3 and tuple(features.shape[:2]) == (C, N):
        shared = 0
    else:
        raise ValueError(f"features must be [N,D] or [C,N,D] with N={N}, C={C}; got {tuple(features.shape)}")
    D = int(features.shape[-1])
    if not features.is_contiguous():
        raise ValueError("features must be contiguous")
    return _with(p, colors_shared=shared), D, (features if D > 0 else None)


def channels(p, D):
    """Channels of the rendered image: D features plus the depth channel."""
    return D + (1 if p.render_depth != L.GSR_DEPTH_NONE else 0)


def rasterize_forward(p, proj, opacities, isect, W, H, background=None, n_eval=False, features=None, stream=None):
    """Composite the sorted lists.  Returns image [P, Dt] (D feature channels,
    then depth when ``p.render_depth`` is set), alpha, final_T, last_ids, the
    optional per-pixel counts and the workspace holding the packed records."""
    C, N = proj["radii"].shape
    d = proj["radii"].device
    pf, D, feat = _features(p, proj, features)
    pix_off, _ = layout(W, H)
    P = pix_off[-1]
    f = dict(device=d, dtype=torch.float32)
    out = dict(image=torch.empty((P, channels(p, D)), **f), alpha=torch.empty(P, **f), final_T=torch.empty(P, **f),
               last_ids=torch.empty(P, device=d, dtype=torch.int32),
               n_eval=torch.empty((P, 5), device=d, dtype=torch.int32) if n_eval else None)
    # the workspace keeps the packed per-Gaussian records for the backward
    out["ws"] = raster_workspace(C, N, d)
    L.gsr_rasterize_fwd(pf, C, N, D, W, H, proj["means2d"], proj["conics"], feat, proj["depths"], opacities,
                        proj["comps"], background, isect["ranges"], isect["ids_buf"], isect.get("order"),
                        out["image"], out["alpha"], out["final_T"], out["last_ids"], out["n_eval"], ws=out["ws"],
                        stream=stream)
    return out


def grad_buffers(C, N, device, absgrad=False, D=3, shared=False, depth=False, zero=True, records=False):
    """Per-camera gradient buffers of the compositing backward, carved from
    one allocation (zeroed with one fill unless ``zero`` is False): v_colors
    is [N,D] for shared features, else [C,N,D]; v_depths [C,N] when depth is
    rendered.  ``records`` (plain RGB only): the four 2D gradients of each
    (camera, Gaussian) kept together in "grad_rec" [C,N,9] (the library's
    grad_records layout), with strided views of its fields under the usual
    names."""
    n = C * N
    if records:
        if D != 3 or shared or depth:
            raise ValueError("gradient records hold plain RGB only")
        G = L.GSR_GRAD_RECORD
        flat = (torch.zeros if zero else torch.empty)(n * G + (2 * n if absgrad else 0), device=device,
                                                      dtype=torch.float32)
        r = flat[:n * G].view(C, N, G)
        return dict(grad_rec=r, v_means2d=r[..., 0:2], v_conics=r[..., 2:5], v_colors=r[..., 5:8],
                    v_opacities=r[..., 8], v_depths=None,
                    v_means2d_abs=flat[n * G:].view(C, N, 2) if absgrad else None)
    nf = (N if shared else n) * D
    sizes = dict(v_means2d=2 * n, v_conics=3 * n, v_colors=nf, v_opacities=n, v_depths=n if depth else 0,
                 v_means2d_abs=2 * n if absgrad else 0)
    flat = (torch.zeros if zero else torch.empty)(sum(sizes.values()), device=device, dtype=torch.float32)
    shapes = dict(v_means2d=(C, N, 2), v_conics=(C, N, 3), v_colors=(N, D) if shared else (C, N, D),
                  v_opacities=(C, N), v_depths=(C, N), v_means2d_abs=(C, N, 2))
    out, o = {}, 0
    for k, m in sizes.items():
        out[k] = flat[o:o + m].view(shapes[k]) if (m or k == "v_colors") else None
        o += m
    return out


def rasterize_backward(p, proj, opacities, isect, W, H, fwd, v_image, v_alpha=None, background=None,
                       absgrad=False, grads=None, features=None, stream=None, overwrite=False, records=False):
    """Gradients of the compositing.  ``grads`` (from ``grad_buffers``) are
    added to; by default fresh zeroed buffers are used.  ``overwrite``: fresh
    uninitialised buffers that the library zeroes itself (no torch fill).
    The records the forward packed into its workspace are reused.
    ``records``: fresh buffers in the gradient-record layout (see
    ``grad_buffers``), which ``project_backward`` reads as they are."""
    C, N = proj["radii"].shape
    d = proj["radii"].device
    pf, D, feat = _features(p, proj, features)
    depth = p.render_depth != L.GSR_DEPTH_NONE
    if overwrite and grads is not None:
        raise ValueError("overwrite makes its own buffers")
    g = grad_buffers(C, N, d, absgrad, D, bool(pf.colors_shared), depth, zero=not overwrite, records=records) \
        if grads is None else grads
    if absgrad and g["v_means2d_abs"] is None:
        raise ValueError("absgrad needs grad buffers made with absgrad=True")
    ws = fwd.get("ws")
    flags = 0 if overwrite else L.GSR_BWD_ACCUMULATE
    if ws is None:
        ws = raster_workspace(C, N, d)
    else:
        flags |= L.GSR_BWD_PACKED
    rec = g.get("grad_rec")
    if rec is not None:
        pf = _with(pf, grad_records=1)
        g4 = (rec, None, None, None)
    else:
        g4 = (g["v_means2d"], g["v_conics"], g["v_colors"] if D > 0 else None, g["v_opacities"])
    L.gsr_rasterize_bwd(pf, C, N, D, W, H, proj["means2d"], proj["conics"], feat, proj["depths"], opacities,
                        proj["comps"], background, isect["ranges"], isect["ids_buf"], isect.get("order"), fwd["image"],
                        fwd["final_T"], fwd["last_ids"], v_image, v_alpha, g4[0], g4[1], g4[2],
                        g["v_depths"] if depth else None, g4[3], g["v_means2d_abs"] if absgrad else None, ws=ws,
                        flags=flags, stream=stream)
    return g


def project_backward(p, means, quats, scales, opacities, sh_or_colors, viewmats, Ks, W, H, proj, g2,
                     v_depths=None, viewmat_grad=False, stream=None):
    """Gradients of the projection; ``viewmat_grad`` adds "v_viewmats" [C,4,4].
    ``sh_or_colors`` None: the colours did not come from the projection (the
    rasterizer took features of its own), so none are differentiated here.
    The depth gradient is ``v_depths`` or, by default, the depth channel's."""
    C, N = viewmats.shape[0], means.shape[0]
    d = means.device
    colour = sh_or_colors is not None
    if v_depths is None:
        v_depths = g2.get("v_depths")
    out = dict(v_means=torch.empty_like(means), v_quats=torch.empty_like(quats), v_scales=torch.empty_like(scales),
               v_opacities=torch.empty_like(opacities), v_sh=torch.empty_like(sh_or_colors) if colour else None,
               v_viewmats=torch.empty((C, 4, 4), device=d, dtype=torch.float32) if viewmat_grad else None)
    ws = None
    if viewmat_grad:
        ws = torch.empty(max(L.workspace_bytes(L.GSR_OP_PROJECT_BWD, C, N, 0), 1), device=d, dtype=torch.uint8)
    rec = g2.get("grad_rec")
    if rec is not None:   # the gradient-record layout: one pointer, the three others NULL
        p = _with(p, grad_records=1)
        g4 = (rec, None, None, None)
    else:
        g4 = (g2["v_means2d"], g2["v_conics"], g2["v_colors"] if colour else None, g2["v_opacities"])
    L.gsr_project_bwd(p, C, N, W, H, means, quats, scales, opacities, sh_or_colors, viewmats, Ks, proj["radii"],
                      proj["comps"], *g4, v_depths, out["v_means"], out["v_quats"], out["v_scales"],
                      out["v_opacities"], out["v_sh"], v_viewmats=out["v_viewmats"], ws=ws, stream=stream)
    return out


class RasterizeGaussians(torch.autograd.Function):
    """(means, quats, scales, opacities, colors, viewmats) -> (image [P,Dt], alpha [P]).
    ``sh``: colors are SH coefficients [N,K,3] that the projection evaluates
    per view; otherwise features [N,D] or [C,N,D] composited as they are.
    Ks and background are constants."""

    @staticmethod
    def forward(ctx, means, quats, scales, opacities, colors, viewmats, Ks, background, p, W, H, absgrad, sh,
                meta):
        means, quats, scales, opacities, colors, viewmats = (t.contiguous() for t in
                                                             (means, quats, scales, opacities, colors, viewmats))
        feats = None if sh else colors
        proj = project(p, means, quats, scales, opacities, colors if sh else None, viewmats, Ks, W, H)
        isect = intersect(p, proj, W, H)
        fwd = rasterize_forward(p, proj, opacities, isect, W, H, background, features=feats)
        if isect.check():            # the list capacity was too small: composite the rebuilt lists
            fwd = rasterize_forward(p, proj, opacities, isect, W, H, background, features=feats)
        ctx.p, ctx.W, ctx.H, ctx.absgrad, ctx.sh = p, W, H, absgrad, sh
        ctx.proj, ctx.isect, ctx.fwd = proj, isect, fwd
        ctx.save_for_backward(means, quats, scales, opacities, colors, viewmats, Ks, background)
        ctx.meta = meta
        meta.update(radii=proj["radii"], means2d=proj["means2d"], depths=proj["depths"], conics=proj["conics"],
                    colors=proj["colors"] if sh else colors, n_intersections=isect["M"],
                    last_ids=fwd["last_ids"], final_T=fwd["final_T"])
        return fwd["image"], fwd["alpha"]

    @staticmethod
    def backward(ctx, v_image, v_alpha):
        means, quats, scales, opacities, colors, viewmats, Ks, background = ctx.saved_tensors
        p, W, H, sh = ctx.p, ctx.W, ctx.H, ctx.sh
        v_image = torch.zeros_like(ctx.fwd["image"]) if v_image is None else v_image.contiguous()
        v_alpha = None if v_alpha is None else v_alpha.contiguous()
        # colours from the projection's SH, plain RGB: the 2D gradients as records (fields as strided views)
        records = sh and p.render_depth == L.GSR_DEPTH_NONE and not p.colors_shared
        g2 = rasterize_backward(p, ctx.proj, opacities, ctx.isect, W, H, ctx.fwd, v_image, v_alpha, background,
                                absgrad=ctx.absgrad, features=None if sh else colors, records=records)
        # dL/d(2D means) per view, for densification (a contiguous copy when it is a field of the records)
        ctx.meta["means2d_grad"] = g2["v_means2d"].contiguous()
        ctx.meta["grads2d"] = g2                            # every compositing gradient, per view
        if ctx.absgrad:
            ctx.meta["means2d_absgrad"] = g2["v_means2d_abs"]
        want_vm = ctx.needs_input_grad[5]
        g3 = project_backward(p, means, quats, scales, opacities, colors if sh else None, viewmats, Ks, W, H,
                              ctx.proj, g2, viewmat_grad=want_vm)
        v_colors = g3["v_sh"] if sh else g2["v_colors"]
        return (g3["v_means"], g3["v_quats"], g3["v_scales"], g3["v_opacities"], v_colors,
                g3["v_viewmats"] if want_vm else None, None, None, None, None, None, None, None, None)


def rasterization(means, quats, scales, opacities, colors, viewmats, Ks, width, height, sh_degree=None,
                  background=None, absgrad=False, antialiased=False, render_mode="RGB", **params):
    """Render C views of N Gaussians (scales and opacities already activated).

    colors: SH coefficients [N,K,3] with K = (d+1)^2, evaluated per view
    (``sh_degree`` defaults to the largest degree K holds); or, with
    ``sh_degree`` None, features [N,D] (shared by all views) or [C,N,D]
    composited as they are (D <= 32; D = 3 is plain RGB).
    render_mode: "RGB" (the colours or features), "D" / "ED" (accumulated /
    expected depth alone), "RGB+D" / "RGB+ED" (features, then depth).
    background: [D] or [C,D] for the feature channels (depth has none).
    Returns (render [C,H,W,Dt], alpha [C,H,W,1], meta); views of different
    sizes are returned packed, as [P,Dt] and [P,1], when width/height are
    sequences.
    """
    C, N = viewmats.shape[0], means.shape[0]
    if render_mode not in RENDER_MODES:
        raise ValueError(f"render_mode must be one of {sorted(RENDER_MODES)}")
    want_feat, depth = RENDER_MODES[render_mode]
    colors = colors.float()
    if not want_feat:                                  # depth alone: no feature channels
        sh, deg, colors = False, -1, torch.zeros((N, 0), device=means.device, dtype=torch.float32)
    elif sh_degree is not None:
        sh, deg = True, int(sh_degree)
    elif colors.dim() == 3 and tuple(colors.shape[:2]) != (C, N):
        sh, deg = True, int(math.isqrt(colors.shape[1])) - 1
    else:
        sh, deg = False, -1
    p = make_params(sh_degree=deg, antialiased=antialiased, render_depth=depth, **params)
    W, H = _sizes_per_cam(C, width, height)
    D = 3 if sh else int(colors.shape[-1])
    bg = None
    if background is not None and D > 0:
        bg = background.to(torch.float32).reshape(-1, D).expand(C, D).contiguous()
    meta = dict(width=W, height=H, sh_degree=deg, render_mode=render_mode)
    image, alpha = RasterizeGaussians.apply(means.float(), quats.float(), scales.float(), opacities.float(), colors,
                                            viewmats.float().contiguous(), Ks.float().contiguous(), bg, p, W, H,
                                            absgrad, sh, meta)
    Dt = image.shape[-1]
    if len(set(W)) == 1 and len(set(H)) == 1:
        image = image.view(C, H[0], W[0], Dt)
        alpha = alpha.view(C, H[0], W[0], 1)
    else:
        alpha = alpha.view(-1, 1)
    return image, alpha, meta
