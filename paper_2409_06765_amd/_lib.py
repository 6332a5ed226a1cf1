"""ctypes binding of libgsraster.so (include/gsraster.h).

Argument marshalling only: every entry point keeps its C name and takes torch
tensors on the GPU (or None for a nullable pointer), host integer sequences for
the per-camera image sizes, and an optional torch stream.  All arithmetic runs
in the HIP library; there is no fallback.  torch is imported first so that the
library binds to the HIP runtime torch has already loaded.
"""
import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# GSR_LIB_VARIANT=san: the host-side sanitizer build (python -m paper_2409_06765_amd.build --sanitize)
LIB_PATH = os.path.join(_PKG, "libgsraster_san.so" if os.environ.get("GSR_LIB_VARIANT") == "san" else "libgsraster.so")

GSR_OK, GSR_EINVAL, GSR_EOVERFLOW, GSR_EWORKSPACE, GSR_EHIP = 0, 1, 2, 3, 4
GSR_OP_INTERSECT_COUNT, GSR_OP_SORT, GSR_OP_RASTERIZE, GSR_OP_BIN_PREPARE, GSR_OP_BIN_FINISH = 1, 2, 3, 4, 5
GSR_OP_PROJECT_BWD = 6
GSR_OP_TILE_ORDER = 7
GSR_OP_L1_LOSS, GSR_OP_DENSIFY_PLAN = 8, 9
GSR_ADAM_MAX_GROUPS, GSR_DENSIFY_MAX_COLUMNS = 8, 16
GSR_ACT_NONE, GSR_ACT_EXP, GSR_ACT_SIGMOID = 0, 1, 2
GSR_PRUNE, GSR_KEEP, GSR_CLONE, GSR_SPLIT = 0, 1, 2, 3
GSR_COLUMN_COPY, GSR_COLUMN_MEANS, GSR_COLUMN_LOG_SCALES, GSR_COLUMN_STATE = 0, 1, 2, 3
GSR_MAX_CAMERAS = 64
GSR_BWD_ACCUMULATE, GSR_BWD_PACKED = 1, 2
GSR_DEPTH_NONE, GSR_DEPTH_ACCUMULATED, GSR_DEPTH_EXPECTED = 0, 1, 2
ABI_VERSION = 9                 # the signatures below
_NAMES = {0: "GSR_OK", 1: "GSR_EINVAL", 2: "GSR_EOVERFLOW", 3: "GSR_EWORKSPACE", 4: "GSR_EHIP"}


class GsrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class gsr_params(ctypes.Structure):
    _fields_ = [("near_plane", ctypes.c_float), ("far_plane", ctypes.c_float), ("eps2d", ctypes.c_float),
                ("jac_clamp", ctypes.c_float), ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_min", ctypes.c_float), ("tile", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("antialiased", ctypes.c_int32), ("render_depth", ctypes.c_int32),
                ("colors_shared", ctypes.c_int32), ("tile_cull", ctypes.c_int32), ("grad_records", ctypes.c_int32)]
GSR_GRAD_RECORD = 9             # floats per (camera, Gaussian) in the grad_records layout


class gsr_adam_group(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("exp_avg", ctypes.c_void_p),
                ("exp_avg_sq", ctypes.c_void_p), ("activated", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("lr", ctypes.c_float), ("lr_rest", ctypes.c_float), ("row", ctypes.c_int32),
                ("row_first", ctypes.c_int32), ("activation", ctypes.c_int32), ("reg", ctypes.c_float)]


class gsr_densify_column(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("width", ctypes.c_int32),
                ("kind", ctypes.c_int32)]


_vp, _i, _i64, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
_f = ctypes.c_float
_P = ctypes.POINTER(gsr_params)
_SIGS = {
    "gsr_abi_version": ([], _i),
    "gsr_last_error": ([], ctypes.c_char_p),
    "gsr_default_params": ([_P], None),
    "gsr_workspace_bytes": ([_i, _i, _i, _i64], _sz),
    "gsr_project_fwd": ([_P, _i, _i, _vp, _vp] + [_vp] * 7 + [_vp] * 6 + [_vp], _i),
    "gsr_intersect_count": ([_P, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _i),
    "gsr_intersect_emit": ([_P, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp], _i),
    "gsr_sort_pairs": ([_i64, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _i),
    "gsr_sort_pairs_noalloc": ([_i64, _i, _vp, _vp, _vp, _vp, _vp], _i),
    "gsr_tile_ranges": ([_i64, _vp, ctypes.c_int32, _vp, _vp], _i),
    "gsr_bin_prepare": ([_P, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _i),
    "gsr_bin_finish": ([_P, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp, _sz,
                        _vp], _i),
    "gsr_tile_order": ([ctypes.c_int32, _vp, _vp, _vp, _sz, _vp], _i),
    "gsr_fill_zero": ([_vp, _sz, _vp], _i),
    "gsr_rasterize_fwd": ([_P, _i, _i, _i, _vp, _vp] + [_vp] * 10 + [_vp] * 5 + [_vp, _sz, _vp], _i),
    "gsr_rasterize_bwd": ([_P, _i, _i, _i, _vp, _vp] + [_vp] * 15 + [_vp] * 6 + [_vp, _sz, _i, _vp], _i),
    "gsr_project_bwd": ([_P, _i, _i, _vp, _vp] + [_vp] * 9 + [_vp] * 5 + [_vp] * 5 + [_vp, _vp, _sz, _vp], _i),
    "gsr_l1_loss": ([_i64, _vp, _vp, _f, _vp, _vp, _vp, _sz, _vp], _i),
    "gsr_activate": ([_i64, _vp, ctypes.c_int32, _vp, _vp], _i),
    "gsr_adam_step": ([_i, ctypes.POINTER(gsr_adam_group), ctypes.c_int32, _f, _f, _f, _vp], _i),
    "gsr_densify_stats": ([_i, _i, _vp, _vp, _vp, _vp, _f, _vp, _vp, _vp], _i),
    "gsr_densify_plan": ([_i, _vp, _vp, _vp, _vp, _f, _f, _f, _vp, _vp, _vp, _vp, _sz, _vp], _i),
    "gsr_densify_apply": ([_i, _vp, _vp, _vp, _vp, _vp, _f, _i, ctypes.POINTER(gsr_densify_column), _vp], _i),
    "gsr_opacity_reset": ([_i, _vp, _vp, _vp, _vp, _f, _vp], _i),
    "gsr_mcmc_noise": ([_i, _vp, _vp, _vp, _vp, _vp, _f, _f, _f, _vp], _i),
}

_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GsrError(GSR_EHIP, f"{LIB_PATH} is missing: build it with python -m paper_2409_06765_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        if L.gsr_abi_version() != ABI_VERSION:
            raise GsrError(GSR_EHIP, f"{LIB_PATH} has ABI version {L.gsr_abi_version()}, the binding expects "
                                     f"{ABI_VERSION}: rebuild it")
        _lib = L
    return _lib


def default_params(**overrides):
    p = gsr_params()
    lib().gsr_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown rasterizer parameter {k}")
        setattr(p, k, v)
    return p


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


_PINNED = threading.local()


def _host_count():
    """A pinned int64 the library copies a count into (a copy into pageable
    host memory goes through a staging buffer and waits much longer)."""
    t = getattr(_PINNED, "t", None)
    if t is None:
        t = _PINNED.t = torch.empty(1, dtype=torch.int64, pin_memory=True)
    t[0] = -1
    return t


def _sizes(xs):
    xs = [int(v) for v in xs]
    return (ctypes.c_int32 * max(len(xs), 1))(*xs)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc):
    if rc != GSR_OK:
        raise GsrError(rc, lib().gsr_last_error().decode(errors="replace"))


def abi_version():
    return lib().gsr_abi_version()


def workspace_bytes(op, C, N, M):
    return int(lib().gsr_workspace_bytes(op, C, N, M))


F32, I32, I64, U64 = torch.float32, torch.int32, torch.int64, torch.uint64


def gsr_project_fwd(p, C, N, W, H, means, quats, scales, opacities, sh_or_colors, viewmats, Ks,
                    means2d, conics, radii, depths, colors, compensations=None, stream=None):
    _check(lib().gsr_project_fwd(
        ctypes.byref(p), C, N, _sizes(W), _sizes(H), _ptr(means, F32, "means"), _ptr(quats, F32, "quats"),
        _ptr(scales, F32, "scales"), _ptr(opacities, F32, "opacities"), _ptr(sh_or_colors, F32, "sh_or_colors"),
        _ptr(viewmats, F32, "viewmats"), _ptr(Ks, F32, "Ks"), _ptr(means2d, F32, "means2d"),
        _ptr(conics, F32, "conics"), _ptr(radii, I32, "radii"), _ptr(depths, F32, "depths"),
        _ptr(colors, F32, "colors"), _ptr(compensations, F32, "compensations"), _stream(stream)))


def gsr_intersect_count(p, C, N, W, H, means2d, radii, tiles_per_gauss, offsets, total_dev, ws, sync=True,
                        stream=None):
    """Returns M when ``sync`` (the call then waits for the stream), else None."""
    host = _host_count() if sync else None
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().gsr_intersect_count(
        ctypes.byref(p), C, N, _sizes(W), _sizes(H), _ptr(means2d, F32, "means2d"), _ptr(radii, I32, "radii"),
        _ptr(tiles_per_gauss, I32, "tiles_per_gauss"), _ptr(offsets, I64, "offsets"), _ptr(total_dev, I64, "total"),
        ctypes.c_void_p(host.data_ptr()) if sync else None, _ptr(ws, None, "workspace"), ws_bytes, _stream(stream)))
    return int(host[0]) if sync else None


def gsr_intersect_emit(p, C, N, W, H, means2d, radii, depths, offsets, M_capacity, keys, ids, stream=None):
    _check(lib().gsr_intersect_emit(
        ctypes.byref(p), C, N, _sizes(W), _sizes(H), _ptr(means2d, F32, "means2d"), _ptr(radii, I32, "radii"),
        _ptr(depths, F32, "depths"), _ptr(offsets, I64, "offsets"), int(M_capacity), _ptr(keys, U64, "keys"),
        _ptr(ids, I32, "ids"), _stream(stream)))


def gsr_sort_pairs(M, key_bits, keys, ids, keys_alt, ids_alt, ws, stream=None):
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().gsr_sort_pairs(int(M), int(key_bits), _ptr(keys, U64, "keys"), _ptr(ids, I32, "ids"),
                                _ptr(keys_alt, U64, "keys_alt"), _ptr(ids_alt, I32, "ids_alt"),
                                _ptr(ws, None, "workspace"), ws_bytes, _stream(stream)))


GSR_SORT_NOALLOC_MAX_PAIRS = 1 << 25


def gsr_sort_pairs_noalloc(M, key_bits, keys, ids, keys_alt, ids_alt, stream=None):
    _check(lib().gsr_sort_pairs_noalloc(int(M), int(key_bits), _ptr(keys, U64, "keys"), _ptr(ids, I32, "ids"),
                                        _ptr(keys_alt, U64, "keys_alt"), _ptr(ids_alt, I32, "ids_alt"),
                                        _stream(stream)))


def gsr_tile_ranges(M, keys, total_tiles, ranges, stream=None):
    _check(lib().gsr_tile_ranges(int(M), _ptr(keys, U64, "keys"), int(total_tiles), _ptr(ranges, I32, "ranges"),
                                 _stream(stream)))


def gsr_bin_prepare(p, C, N, W, H, means2d, radii, depths, conics, opacities, compensations, total_dev, ws_prep,
                    sync=True, stream=None):
    """Returns M when ``sync`` (the call then waits for the stream), else None."""
    host = _host_count() if sync else None
    _check(lib().gsr_bin_prepare(
        ctypes.byref(p), C, N, _sizes(W), _sizes(H), _ptr(means2d, F32, "means2d"), _ptr(radii, I32, "radii"),
        _ptr(depths, F32, "depths"), _ptr(conics, F32, "conics"), _ptr(opacities, F32, "opacities"),
        _ptr(compensations, F32, "compensations"), _ptr(total_dev, I64, "total"),
        ctypes.c_void_p(host.data_ptr()) if sync else None, *_ws(ws_prep), _stream(stream)))
    return int(host[0]) if sync else None


def gsr_bin_finish(p, C, N, W, H, means2d, radii, depths, conics, opacities, compensations, M, ids, ranges, keys,
                   ws_prep, ws_fin, stream=None):
    _check(lib().gsr_bin_finish(
        ctypes.byref(p), C, N, _sizes(W), _sizes(H), _ptr(means2d, F32, "means2d"), _ptr(radii, I32, "radii"),
        _ptr(depths, F32, "depths"), _ptr(conics, F32, "conics"), _ptr(opacities, F32, "opacities"),
        _ptr(compensations, F32, "compensations"), int(M), _ptr(ids, I32, "ids"), _ptr(ranges, I32, "ranges"),
        _ptr(keys, U64, "keys"), *_ws(ws_prep), *_ws(ws_fin), _stream(stream)))


def _ws(ws):
    return (_ptr(ws, None, "workspace"), ws.numel() * ws.element_size()) if ws is not None else (None, 0)


def gsr_tile_order(total_tiles, ranges, order, ws, stream=None):
    _check(lib().gsr_tile_order(int(total_tiles), _ptr(ranges, I32, "ranges"), _ptr(order, I32, "order"), *_ws(ws),
                                _stream(stream)))


def gsr_fill_zero(t, stream=None):
    """Zeroes the whole of tensor ``t`` (contiguous, on the GPU) with the
    library's fill kernel."""
    _check(lib().gsr_fill_zero(_ptr(t, None, "tensor"), t.numel() * t.element_size(), _stream(stream)))


def gsr_rasterize_fwd(p, C, N, D, W, H, means2d, conics, colors, depths, opacities, compensations, background,
                      ranges, ids, tile_order, image, alpha, final_T, last_ids, n_eval=None, ws=None, stream=None):
    _check(lib().gsr_rasterize_fwd(
        ctypes.byref(p), C, N, D, _sizes(W), _sizes(H), _ptr(means2d, F32, "means2d"), _ptr(conics, F32, "conics"),
        _ptr(colors, F32, "colors"), _ptr(depths, F32, "depths"), _ptr(opacities, F32, "opacities"),
        _ptr(compensations, F32, "compensations"), _ptr(background, F32, "background"),
        _ptr(ranges, I32, "ranges"), _ptr(ids, I32, "ids"), _ptr(tile_order, I32, "tile_order"),
        _ptr(image, F32, "image"), _ptr(alpha, F32, "alpha"),
        _ptr(final_T, F32, "final_T"), _ptr(last_ids, I32, "last_ids"), _ptr(n_eval, I32, "n_eval"), *_ws(ws),
        _stream(stream)))


def gsr_rasterize_bwd(p, C, N, D, W, H, means2d, conics, colors, depths, opacities, compensations, background,
                      ranges, ids, tile_order, image, final_T, last_ids, v_image, v_alpha, v_means2d, v_conics,
                      v_colors, v_depths, v_opacities, v_means2d_abs=None, ws=None, flags=0, stream=None):
    _check(lib().gsr_rasterize_bwd(
        ctypes.byref(p), C, N, D, _sizes(W), _sizes(H), _ptr(means2d, F32, "means2d"), _ptr(conics, F32, "conics"),
        _ptr(colors, F32, "colors"), _ptr(depths, F32, "depths"), _ptr(opacities, F32, "opacities"),
        _ptr(compensations, F32, "compensations"), _ptr(background, F32, "background"),
        _ptr(ranges, I32, "ranges"), _ptr(ids, I32, "ids"), _ptr(tile_order, I32, "tile_order"),
        _ptr(image, F32, "image"),
        _ptr(final_T, F32, "final_T"), _ptr(last_ids, I32, "last_ids"), _ptr(v_image, F32, "v_image"),
        _ptr(v_alpha, F32, "v_alpha"), _ptr(v_means2d, F32, "v_means2d"), _ptr(v_conics, F32, "v_conics"),
        _ptr(v_colors, F32, "v_colors"), _ptr(v_depths, F32, "v_depths"), _ptr(v_opacities, F32, "v_opacities"),
        _ptr(v_means2d_abs, F32, "v_means2d_abs"), *_ws(ws), int(flags), _stream(stream)))


def gsr_project_bwd(p, C, N, W, H, means, quats, scales, opacities, sh_or_colors, viewmats, Ks, radii,
                    compensations, v_means2d, v_conics, v_colors, v_opacities_cn, v_depths, v_means, v_quats,
                    v_scales, v_opacities, v_sh_or_colors, v_viewmats=None, ws=None, stream=None):
    _check(lib().gsr_project_bwd(
        ctypes.byref(p), C, N, _sizes(W), _sizes(H), _ptr(means, F32, "means"), _ptr(quats, F32, "quats"),
        _ptr(scales, F32, "scales"), _ptr(opacities, F32, "opacities"), _ptr(sh_or_colors, F32, "sh_or_colors"),
        _ptr(viewmats, F32, "viewmats"), _ptr(Ks, F32, "Ks"), _ptr(radii, I32, "radii"),
        _ptr(compensations, F32, "compensations"), _ptr(v_means2d, F32, "v_means2d"),
        _ptr(v_conics, F32, "v_conics"), _ptr(v_colors, F32, "v_colors"),
        _ptr(v_opacities_cn, F32, "v_opacities_cn"), _ptr(v_depths, F32, "v_depths"),
        _ptr(v_means, F32, "v_means"), _ptr(v_quats, F32, "v_quats"), _ptr(v_scales, F32, "v_scales"),
        _ptr(v_opacities, F32, "v_opacities"), _ptr(v_sh_or_colors, F32, "v_sh_or_colors"),
        _ptr(v_viewmats, F32, "v_viewmats"), *_ws(ws), _stream(stream)))


# ---- training-loop steps ----------------------------------------------------------
def gsr_l1_loss(image, target, scale, v_image, loss, ws, stream=None):
    n = image.numel()
    if target.numel() != n or v_image.numel() != n:
        raise ValueError("image, target and v_image must have the same number of elements")
    _check(lib().gsr_l1_loss(n, _ptr(image, F32, "image"), _ptr(target, F32, "target"), float(scale),
                             _ptr(v_image, F32, "v_image"), _ptr(loss, F32, "loss"), *_ws(ws), _stream(stream)))


def gsr_activate(raw, activation, out, stream=None):
    if raw.numel() != out.numel():
        raise ValueError("raw and out must have the same number of elements")
    _check(lib().gsr_activate(raw.numel(), _ptr(raw, F32, "raw"), int(activation), _ptr(out, F32, "out"),
                              _stream(stream)))


def gsr_adam_step(groups, step, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """groups: dicts with param, grad, exp_avg, exp_avg_sq (tensors of one
    size), optional activated, lr, lr_rest, row, row_first, activation, reg."""
    arr = (gsr_adam_group * max(len(groups), 1))()
    keep = []
    for i, g in enumerate(groups):
        n = g["param"].numel()
        for k in ("grad", "exp_avg", "exp_avg_sq", "activated"):
            if g.get(k) is not None and g[k].numel() != n:
                raise ValueError(f"group {i}: {k} has {g[k].numel()} elements, param {n}")
        e = arr[i]
        e.param, e.grad = _ptr(g["param"], F32, "param"), _ptr(g["grad"], F32, "grad")
        e.exp_avg, e.exp_avg_sq = _ptr(g["exp_avg"], F32, "exp_avg"), _ptr(g["exp_avg_sq"], F32, "exp_avg_sq")
        e.activated = _ptr(g.get("activated"), F32, "activated")
        e.n = n
        e.lr = float(g["lr"])
        e.lr_rest = float(g.get("lr_rest", g["lr"]))
        e.row, e.row_first = int(g.get("row", 0)), int(g.get("row_first", 0))
        e.activation, e.reg = int(g.get("activation", GSR_ACT_NONE)), float(g.get("reg", 0.0))
        keep.append(g)
    _check(lib().gsr_adam_step(len(groups), arr, int(step), float(beta1), float(beta2), float(eps), _stream(stream)))


def gsr_densify_stats(C, N, W, H, radii, v_means2d, scale, grad_accum, count, stream=None):
    _check(lib().gsr_densify_stats(C, N, _sizes(W), _sizes(H), _ptr(radii, I32, "radii"),
                                   _ptr(v_means2d, F32, "v_means2d"), float(scale), _ptr(grad_accum, F32, "grad_accum"),
                                   _ptr(count, I32, "count"), _stream(stream)))


def gsr_densify_plan(N, grad_accum, count, scales, opacities, grad_threshold, scale_threshold, prune_opacity,
                     action, offsets, ws, sync=True, stream=None):
    """Returns the new count when ``sync`` (the call then waits)."""
    host = _host_count() if sync else None
    _check(lib().gsr_densify_plan(N, _ptr(grad_accum, F32, "grad_accum"), _ptr(count, I32, "count"),
                                  _ptr(scales, F32, "scales"), _ptr(opacities, F32, "opacities"),
                                  float(grad_threshold), float(scale_threshold), float(prune_opacity),
                                  _ptr(action, I32, "action"), _ptr(offsets, I64, "offsets"),
                                  ctypes.c_void_p(host.data_ptr()) if sync else None, *_ws(ws), _stream(stream)))
    return int(host[0]) if sync else None


def gsr_densify_apply(N, action, offsets, quats, log_scales, split_normals, split_shrink, columns, stream=None):
    """columns: (src, dst, kind) triples; the width is src.numel() / N."""
    arr = (gsr_densify_column * max(len(columns), 1))()
    for i, (src, dst, kind) in enumerate(columns):
        w = src.numel() // N if N > 0 else 1
        arr[i].src, arr[i].dst = _ptr(src, F32, "src"), _ptr(dst, F32, "dst")
        arr[i].width, arr[i].kind = int(w), int(kind)
    _check(lib().gsr_densify_apply(N, _ptr(action, I32, "action"), _ptr(offsets, I64, "offsets"),
                                   _ptr(quats, F32, "quats"), _ptr(log_scales, F32, "log_scales"),
                                   _ptr(split_normals, F32, "split_normals"), float(split_shrink), len(columns), arr,
                                   _stream(stream)))


def gsr_opacity_reset(N, logits, exp_avg, exp_avg_sq, opacities, max_opacity, stream=None):
    _check(lib().gsr_opacity_reset(N, _ptr(logits, F32, "logits"), _ptr(exp_avg, F32, "exp_avg"),
                                   _ptr(exp_avg_sq, F32, "exp_avg_sq"), _ptr(opacities, F32, "opacities"),
                                   float(max_opacity), _stream(stream)))


def gsr_mcmc_noise(N, means, quats, scales, opacities, normals, coeff, k=100.0, t=0.005, stream=None):
    _check(lib().gsr_mcmc_noise(N, _ptr(means, F32, "means"), _ptr(quats, F32, "quats"), _ptr(scales, F32, "scales"),
                                _ptr(opacities, F32, "opacities"), _ptr(normals, F32, "normals"), float(coeff),
                                float(k), float(t), _stream(stream)))
