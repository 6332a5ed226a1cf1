"""CPU oracle for the differentiable tile rasterizer of gsplat (arXiv 2409.06765).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path never does.  It
shares no code with the HIP library.

``Oracle(np.float32)`` wraps the C oracle built in the kernels' precision,
which is the precision in which every floating-point decision that fixes an
integer (radius, tile rectangle, depth key bits, skip/stop) is taken.
``Oracle(np.float64)`` is the same source in double precision, used by the
pins (invariants, closed forms, finite differences).

Rasterization outputs carry per-pixel ``flags`` (FLAG_* bits: a decision
within the error bound of an accurate float32 implementation, so that one may
take it the other way) and ``margin`` (the smallest |ln(value / threshold)|
over the pixel's skip, clamp and stop decisions).

Images are packed per camera: pixel (c, y, x) lives at ``pix_off[c] + y*W_c + x``
of a flat [P, 3] / [P] array; for cameras of equal size that is [C, H, W, ...].
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


@dataclass
class OracleParams:
    """Rasterizer constants.  Thresholds are float32-representable so that the
    single- and double-precision builds compare against the same numbers."""
    near_plane: float = float(np.float32(0.01))
    far_plane: float = float("inf")
    eps2d: float = float(np.float32(0.3))
    jac_clamp: float = float(np.float32(1.3))
    alpha_min: float = float(np.float32(1.0) / np.float32(255.0))
    alpha_max: float = float(np.float32(0.99))
    T_min: float = float(np.float32(1e-4))
    tile: int = 16
    sh_degree: int = -1
    antialiased: int = 0


class _CParams(ctypes.Structure):
    _fields_ = [("near_plane", ctypes.c_double), ("far_plane", ctypes.c_double),
                ("eps2d", ctypes.c_double), ("jac_clamp", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("T_min", ctypes.c_double), ("tile", ctypes.c_int),
                ("sh_degree", ctypes.c_int), ("antialiased", ctypes.c_int)]


def build(force=False):
    """Compile both precisions with the oracle's own Makefile."""
    args = ["make", "-s", "-C", _HERE]
    if force:
        args.insert(1, "-B")
    subprocess.check_call(args)


_LIBS = {}


def _load(kind):
    """The oracle build of one precision; GSORACLE_VARIANT=asan loads the
    sanitizer build (make -C oracle asan) instead."""
    if kind in _LIBS:
        return _LIBS[kind]
    variant = os.environ.get("GSORACLE_VARIANT", "")
    suffix = "_asan" if variant == "asan" else ""
    path = os.path.join(_HERE, f"libgsoracle_{kind}{suffix}.so")
    src = os.path.join(_HERE, "gsoracle.c")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        subprocess.check_call(["make", "-s", "-C", _HERE] + (["asan"] if suffix else []))
    lib = ctypes.CDLL(path)
    lib.orc_intersect_count.restype = ctypes.c_int64
    _LIBS[kind] = lib
    return lib


class _Keep:
    """Pointer maker that holds every array it hands out, so temporaries made
    by dtype conversion stay alive until the C call has returned."""

    def __init__(self):
        self.arrays = []

    def __call__(self, a):
        if a is None:
            return None
        assert a.flags["C_CONTIGUOUS"], "oracle inputs must be contiguous"
        self.arrays.append(a)
        return ctypes.c_void_p(a.ctypes.data)


def _nch(proj):
    """Feature channels D of the projected colours [C, N, D]."""
    return int(np.asarray(proj["colors"]).shape[-1])


def _ints(xs):
    a = np.ascontiguousarray(np.asarray(xs, dtype=np.int32))
    return a


# Per-pixel decision flags of the compositing (one bit per kind of decision
# that lies within an accurate float32 implementation's error bound).
FLAG_SIGN, FLAG_SKIP, FLAG_CLAMP, FLAG_STOP = 1, 2, 4, 8


def set_threads(n):
    """Threads of the oracle's loops over tiles (both precisions; 1 by
    default).  For timing on every host core and for whole-frame tests;
    forward results do not depend on it."""
    for kind in ("f32", "f64"):
        _load(kind).orc_set_threads(int(n))


def get_threads():
    return int(_load("f32").orc_get_threads())


def camera_layout(W, H, tile=16):
    """Per-camera pixel and tile offsets of the packed layout."""
    W = np.asarray(W, dtype=np.int64)
    H = np.asarray(H, dtype=np.int64)
    TX = (W + tile - 1) // tile
    TY = (H + tile - 1) // tile
    pix_off = np.concatenate([[0], np.cumsum(W * H)])
    tile_off = np.concatenate([[0], np.cumsum(TX * TY)])
    return pix_off, tile_off, TX, TY


class Oracle:
    def __init__(self, dtype=np.float32):
        self.dtype = np.dtype(dtype)
        self.lib = _load("f32" if self.dtype == np.float32 else "f64")

    # -- helpers ---------------------------------------------------------
    def _abs_buf(self, out, C, N, want):
        if not want:
            return None
        out["_abs"] = np.zeros((C, N, 6 + out["v_colors"].shape[-1]), self.dtype)
        return out["_abs"]

    def _absgrad_buf(self, out, C, N, want):
        if not want:
            return None
        out["v_means2d_abs"] = np.zeros((C, N, 2), self.dtype)
        return out["v_means2d_abs"]

    @staticmethod
    def _split_abs(out, C, N):
        a = out.pop("_abs", None)
        if a is not None:
            out.update(abs_v_means2d=a[..., 0:2], abs_v_conics=a[..., 2:5], abs_v_opacities=a[..., 5],
                       abs_v_colors=a[..., 6:])
        return out

    def _r(self, a):
        return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=self.dtype))

    def _cp(self, P):
        return ctypes.byref(_CParams(P.near_plane, P.far_plane, P.eps2d, P.jac_clamp, P.alpha_min,
                                     P.alpha_max, P.T_min, P.tile, P.sh_degree, P.antialiased))

    @staticmethod
    def _whc(viewmats, W, H):
        C = viewmats.shape[0]
        W = _ints(np.broadcast_to(np.asarray(W), (C,)))
        H = _ints(np.broadcast_to(np.asarray(H), (C,)))
        return C, W, H

    # -- Projection of Gaussians -----------------------------------------
    def project(self, P, means, quats, scales, opacities, sh_or_colors, viewmats, Ks, W, H):
        _p = _Keep()
        means, quats, scales, opacities = map(self._r, (means, quats, scales, opacities))
        shc, viewmats, Ks = map(self._r, (sh_or_colors, viewmats, Ks))
        N = means.shape[0]
        C, Wa, Ha = self._whc(viewmats, W, H)
        dt = self.dtype
        out = dict(means2d=np.zeros((C, N, 2), dt), conics=np.zeros((C, N, 3), dt),
                   radii=np.zeros((C, N), np.int32), depths=np.zeros((C, N), dt),
                   colors=np.zeros((C, N, 3), dt), comps=np.zeros((C, N), dt))
        self.lib.orc_project(self._cp(P), C, N, _p(Wa), _p(Ha), _p(means), _p(quats), _p(scales),
                             _p(opacities), _p(shc), _p(viewmats), _p(Ks), _p(out["means2d"]),
                             _p(out["conics"]), _p(out["radii"]), _p(out["depths"]), _p(out["colors"]),
                             _p(out["comps"]))
        return out

    def project_bwd(self, P, means, quats, scales, opacities, sh_or_colors, viewmats, Ks, W, H,
                    v_means2d, v_conics, v_colors, v_opacities_cn, v_depths=None, viewmat_grad=False):
        """viewmat_grad: also return "v_viewmats" [C,4,4], the gradient with
        respect to the world-to-camera matrices (last row zero)."""
        _p = _Keep()
        means, quats, scales, opacities = map(self._r, (means, quats, scales, opacities))
        shc, viewmats, Ks = map(self._r, (sh_or_colors, viewmats, Ks))
        v_means2d, v_conics, v_colors, v_opacities_cn, v_depths = map(
            self._r, (v_means2d, v_conics, v_colors, v_opacities_cn, v_depths))
        N = means.shape[0]
        C, Wa, Ha = self._whc(viewmats, W, H)
        dt = self.dtype
        out = dict(v_means=np.zeros((N, 3), dt), v_quats=np.zeros((N, 4), dt),
                   v_scales=np.zeros((N, 3), dt), v_opacities=np.zeros((N,), dt),
                   v_sh=np.zeros(shc.shape, dt))
        self.lib.orc_project_bwd(self._cp(P), C, N, _p(Wa), _p(Ha), _p(means), _p(quats), _p(scales),
                                 _p(opacities), _p(shc), _p(viewmats), _p(Ks), _p(v_means2d), _p(v_conics),
                                 _p(v_colors), _p(v_opacities_cn), _p(v_depths), _p(out["v_means"]),
                                 _p(out["v_quats"]), _p(out["v_scales"]), _p(out["v_opacities"]),
                                 _p(out["v_sh"]), _p(self._viewmat_buf(out, C, viewmat_grad)))
        return out

    def _viewmat_buf(self, out, C, want):
        if not want:
            return None
        out["v_viewmats"] = np.zeros((C, 4, 4), self.dtype)
        return out["v_viewmats"]

    # -- tile binning and depth sort ---------------------------------------
    def intersect(self, P, proj, W, H, sort=True):
        _p = _Keep()
        means2d, depths = self._r(proj["means2d"]), self._r(proj["depths"])
        radii = np.ascontiguousarray(proj["radii"], dtype=np.int32)
        C, N = radii.shape
        Wa = _ints(np.broadcast_to(np.asarray(W), (C,)))
        Ha = _ints(np.broadcast_to(np.asarray(H), (C,)))
        counts = np.zeros((C, N), np.int32)
        offsets = np.zeros((C, N), np.int64)
        cp = self._cp(P)
        M = int(self.lib.orc_intersect_count(cp, C, N, _p(Wa), _p(Ha), _p(means2d), _p(radii),
                                             _p(counts), _p(offsets)))
        keys = np.zeros(max(M, 1), np.uint64)
        ids = np.zeros(max(M, 1), np.int32)
        self.lib.orc_intersect_emit(cp, C, N, _p(Wa), _p(Ha), _p(means2d), _p(radii), _p(depths),
                                    _p(offsets), _p(keys), _p(ids))
        keys, ids = keys[:M].copy(), ids[:M].copy()
        out = dict(counts=counts, offsets=offsets, M=M, keys_emitted=keys.copy(), ids_emitted=ids.copy())
        _, tile_off, _, _ = camera_layout(Wa, Ha, P.tile)
        total_tiles = int(tile_off[-1])
        if sort:
            self.lib.orc_sort_pairs(ctypes.c_int64(M), _p(keys), _p(ids))
            ranges = np.zeros((total_tiles, 2), np.int32)
            self.lib.orc_tile_ranges(ctypes.c_int64(M), _p(keys), total_tiles, _p(ranges))
            out.update(keys=keys, ids=ids, ranges=ranges)
        return out

    # -- Rasterization of Gaussians ----------------------------------------
    def _pixbufs(self, Wa, Ha, D=3):
        npix = int(np.sum(Wa.astype(np.int64) * Ha))
        dt = self.dtype
        return dict(image=np.zeros((npix, D), dt), alpha=np.zeros(npix, dt), final_T=np.zeros(npix, dt),
                    n_eval=np.zeros(npix, np.int32), n_comp=np.zeros(npix, np.int32),
                    flags=np.zeros(npix, np.uint8),
                    trace=np.zeros(npix, np.uint32), margin=np.full(npix, np.inf))

    def rasterize_fwd(self, P, proj, opacities, ranges, ids, W, H, background=None, tile_mask=None):
        _p = _Keep()
        C, N = proj["radii"].shape
        Wa = _ints(np.broadcast_to(np.asarray(W), (C,)))
        Ha = _ints(np.broadcast_to(np.asarray(H), (C,)))
        out = self._pixbufs(Wa, Ha, _nch(proj))
        out["last_ids"] = np.full(out["alpha"].shape, -1, np.int32)
        comps = self._r(proj["comps"]) if P.antialiased else None
        tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
        self.lib.orc_rasterize_fwd(self._cp(P), C, N, _nch(proj), _p(Wa), _p(Ha), _p(self._r(proj["means2d"])),
                                   _p(self._r(proj["conics"])), _p(self._r(proj["colors"])),
                                   _p(self._r(opacities)), _p(comps), _p(self._r(background)),
                                   _p(np.ascontiguousarray(ranges, np.int32)), _p(np.ascontiguousarray(ids, np.int32)),
                                   _p(tm), _p(out["image"]), _p(out["alpha"]), _p(out["final_T"]),
                                   _p(out["last_ids"]), _p(out["n_eval"]), _p(out["n_comp"]), _p(out["flags"]),
                                   _p(out["trace"]), _p(out["margin"]))
        return out

    def rasterize_bwd(self, P, proj, opacities, ranges, ids, W, H, final_T, last_ids, v_image,
                      v_alpha=None, background=None, tile_mask=None, abs_sums=False, absgrad=False):
        """abs_sums: also return "abs_<name>", per gradient element the sum of
        the magnitudes of its terms (the scale of float32 summation error).
        absgrad: also return "v_means2d_abs", per Gaussian the sum over
        pixels of the absolute values of their mean-gradient contributions."""
        _p = _Keep()
        C, N = proj["radii"].shape
        Wa = _ints(np.broadcast_to(np.asarray(W), (C,)))
        Ha = _ints(np.broadcast_to(np.asarray(H), (C,)))
        dt = self.dtype
        out = dict(v_means2d=np.zeros((C, N, 2), dt), v_conics=np.zeros((C, N, 3), dt),
                   v_colors=np.zeros((C, N, _nch(proj)), dt), v_opacities=np.zeros((C, N), dt))
        comps = self._r(proj["comps"]) if P.antialiased else None
        tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
        self.lib.orc_rasterize_bwd(self._cp(P), C, N, _nch(proj), _p(Wa), _p(Ha), _p(self._r(proj["means2d"])),
                                   _p(self._r(proj["conics"])), _p(self._r(proj["colors"])),
                                   _p(self._r(opacities)), _p(comps), _p(self._r(background)),
                                   _p(np.ascontiguousarray(ranges, np.int32)), _p(np.ascontiguousarray(ids, np.int32)),
                                   _p(tm), _p(self._r(final_T)), _p(np.ascontiguousarray(last_ids, np.int32)),
                                   _p(self._r(v_image)), _p(self._r(v_alpha)), _p(out["v_means2d"]),
                                   _p(out["v_conics"]), _p(out["v_colors"]), _p(out["v_opacities"]),
                                   _p(self._abs_buf(out, C, N, abs_sums)), _p(self._absgrad_buf(out, C, N, absgrad)))
        return self._split_abs(out, C, N)

    # -- N-D features and depth rendering -----------------------------------
    def _channels(self, proj, features, depth):
        """The per-Gaussian channels the definitions composite: the features
        ([C,N,D], or [N,D] shared by every camera; None = the projected
        colours), then the depth z (accumulated or expected depth), then a
        channel of ones for expected depth, whose composite is the sum of
        alpha T (Depth rendering appendix).  Returns (channels [C,N,D+e], D,
        shared, e)."""
        C, N = proj["radii"].shape
        F = proj["colors"] if features is None else features
        F = np.asarray(F, dtype=self.dtype)
        shared = F.ndim == 2
        F = np.broadcast_to(F, (C, N, F.shape[-1])) if shared else F
        D = F.shape[-1]
        if depth not in ("none", "accumulated", "expected"):
            raise ValueError(depth)
        extra = []
        if depth != "none":
            extra.append(np.asarray(proj["depths"], self.dtype)[..., None])
        if depth == "expected":
            extra.append(np.ones((C, N, 1), self.dtype))
        return np.ascontiguousarray(np.concatenate([F] + extra, axis=-1)), D, shared, len(extra)

    @staticmethod
    def _bg_channels(background, C, D, e):
        if background is None:
            return None
        bg = np.asarray(background, dtype=np.float64).reshape(C, D)
        return np.concatenate([bg, np.zeros((C, e))], axis=1)    # depth has no background

    def channels_fwd(self, P, proj, opacities, ranges, ids, W, H, features=None, depth="none",
                     background=None):
        """Compositing of D feature channels, plus the depth channel:
        "accumulated" is the sum of z alpha T; "expected" divides it by the
        sum of alpha T (0 where nothing is composited).  Returns the
        rasterize_fwd outputs with image [P, D (+1)], and "weight" (the sum of
        alpha T, composited as a channel of ones) for expected depth."""
        C, N = proj["radii"].shape
        ch, D, shared, e = self._channels(proj, features, depth)
        out = self.rasterize_fwd(P, dict(proj, colors=ch), opacities, ranges, ids, W, H,
                                 background=self._bg_channels(background, C, D, e))
        if depth == "expected":
            A, Wt = out["image"][:, D], out["image"][:, D + 1]
            pos = Wt > 0
            E = np.zeros_like(A)
            E[pos] = A[pos] / Wt[pos]
            out["image"] = np.ascontiguousarray(np.concatenate([out["image"][:, :D], E[:, None]], axis=1))
            out["weight"] = Wt
        return out

    def channels_bwd(self, P, proj, opacities, ranges, ids, W, H, fwd, v_image, v_alpha=None, features=None,
                     depth="none", background=None, abs_sums=False, absgrad=False):
        """Gradients of channels_fwd.  Expected depth E = A / Wt by the
        quotient rule: dL/dA = v_E / Wt, dL/dWt = -v_E E / Wt (both 0 where
        Wt = 0), composited back through the depth and ones channels.
        v_colors has the features' shape (summed over cameras when they are
        shared); "v_depths" [C,N] is the depth channel's gradient."""
        C, N = proj["radii"].shape
        ch, D, shared, e = self._channels(proj, features, depth)
        v_image = np.asarray(v_image, dtype=np.float64).reshape(-1, D + (1 if depth != "none" else 0))
        parts = [v_image[:, :D]]
        if depth == "accumulated":
            parts.append(v_image[:, D:D + 1])
        elif depth == "expected":
            Wt = np.asarray(fwd["weight"], np.float64)
            E = np.asarray(fwd["image"], np.float64)[:, D]
            vE = v_image[:, D]
            pos = Wt > 0
            vA, vW = np.zeros_like(vE), np.zeros_like(vE)
            vA[pos] = vE[pos] / Wt[pos]
            vW[pos] = -vE[pos] * E[pos] / Wt[pos]
            parts += [vA[:, None], vW[:, None]]
        g = self.rasterize_bwd(P, dict(proj, colors=ch), opacities, ranges, ids, W, H, fwd["final_T"],
                               fwd["last_ids"], np.concatenate(parts, axis=1), v_alpha,
                               background=self._bg_channels(background, C, D, e), abs_sums=abs_sums, absgrad=absgrad)
        vc = g["v_colors"]
        if depth != "none":
            g["v_depths"] = np.ascontiguousarray(vc[..., D])
        g["v_colors"] = vc[..., :D].sum(axis=0) if shared else np.ascontiguousarray(vc[..., :D])
        if "abs_v_colors" in g:
            a = g["abs_v_colors"]
            if depth != "none":
                g["abs_v_depths"] = np.ascontiguousarray(a[..., D])
            g["abs_v_colors"] = a[..., :D].sum(axis=0) if shared else np.ascontiguousarray(a[..., :D])
        return g

    # -- the plain definition, tile by tile ---------------------------------
    def render_tiles_fwd(self, P, proj, opacities, tiles, W, H, background=None, untiled=False):
        """``tiles``: int array [T, 3] of (camera, tile x, tile y)."""
        _p = _Keep()
        C, N = proj["radii"].shape
        Wa = _ints(np.broadcast_to(np.asarray(W), (C,)))
        Ha = _ints(np.broadcast_to(np.asarray(H), (C,)))
        tiles = np.ascontiguousarray(np.asarray(tiles, dtype=np.int32).reshape(-1, 3))
        out = self._pixbufs(Wa, Ha, _nch(proj))
        out["last_gid"] = np.full(out["alpha"].shape, -1, np.int32)
        out["last_pos"] = np.full(out["alpha"].shape, -1, np.int32)
        out["list_len"] = np.zeros(tiles.shape[0], np.int32)
        comps = self._r(proj["comps"]) if P.antialiased else None
        self.lib.orc_render_tiles_fwd(self._cp(P), C, N, _nch(proj), _p(Wa), _p(Ha), _p(self._r(proj["means2d"])),
                                      _p(self._r(proj["conics"])), _p(self._r(proj["colors"])),
                                      _p(self._r(opacities)), _p(comps),
                                      _p(np.ascontiguousarray(proj["radii"], np.int32)),
                                      _p(self._r(proj["depths"])), _p(self._r(background)),
                                      tiles.shape[0], _p(tiles), int(bool(untiled)), _p(out["image"]),
                                      _p(out["alpha"]), _p(out["final_T"]), _p(out["last_gid"]),
                                      _p(out["last_pos"]), _p(out["n_eval"]), _p(out["n_comp"]),
                                      _p(out["flags"]), _p(out["trace"]), _p(out["list_len"]), _p(out["margin"]))
        return out

    def render_tiles_bwd(self, P, proj, opacities, tiles, W, H, v_image, v_alpha=None, background=None,
                         abs_sums=False, absgrad=False):
        _p = _Keep()
        C, N = proj["radii"].shape
        Wa = _ints(np.broadcast_to(np.asarray(W), (C,)))
        Ha = _ints(np.broadcast_to(np.asarray(H), (C,)))
        tiles = np.ascontiguousarray(np.asarray(tiles, dtype=np.int32).reshape(-1, 3))
        dt = self.dtype
        out = dict(v_means2d=np.zeros((C, N, 2), dt), v_conics=np.zeros((C, N, 3), dt),
                   v_colors=np.zeros((C, N, _nch(proj)), dt), v_opacities=np.zeros((C, N), dt))
        comps = self._r(proj["comps"]) if P.antialiased else None
        self.lib.orc_render_tiles_bwd(self._cp(P), C, N, _nch(proj), _p(Wa), _p(Ha), _p(self._r(proj["means2d"])),
                                      _p(self._r(proj["conics"])), _p(self._r(proj["colors"])),
                                      _p(self._r(opacities)), _p(comps),
                                      _p(np.ascontiguousarray(proj["radii"], np.int32)),
                                      _p(self._r(proj["depths"])), _p(self._r(background)),
                                      tiles.shape[0], _p(tiles), _p(self._r(v_image)), _p(self._r(v_alpha)),
                                      _p(out["v_means2d"]), _p(out["v_conics"]), _p(out["v_colors"]),
                                      _p(out["v_opacities"]), _p(self._abs_buf(out, C, N, abs_sums)),
                                      _p(self._absgrad_buf(out, C, N, absgrad)))
        return self._split_abs(out, C, N)

    def tile_list(self, P, proj, W, H, c, tx, ty):
        """The definition's per-tile list (ids in depth-bits, id order)."""
        _p = _Keep()
        C, N = proj["radii"].shape
        Wa = _ints(np.broadcast_to(np.asarray(W), (C,)))
        Ha = _ints(np.broadcast_to(np.asarray(H), (C,)))
        out = np.zeros(max(N, 1), np.int32)
        n = self.lib.orc_tile_list(self._cp(P), C, N, _p(Wa), _p(Ha), _p(self._r(proj["means2d"])),
                                   _p(np.ascontiguousarray(proj["radii"], np.int32)), _p(self._r(proj["depths"])),
                                   int(c), int(tx), int(ty), _p(out))
        return out[:n].copy()

    # -- pins support --------------------------------------------------------
    def cov3d(self, q, s):
        _p = _Keep()
        q, s = self._r(q), self._r(s)
        Sig = np.zeros(9, self.dtype)
        R = np.zeros(9, self.dtype)
        self.lib.orc_cov3d(_p(q), _p(s), _p(Sig), _p(R))
        return Sig.reshape(3, 3), R.reshape(3, 3)

    def sh_basis(self, nk, direction):
        _p = _Keep()
        d = np.ascontiguousarray(np.asarray(direction, dtype=np.float64))
        Y = np.zeros(nk, np.float64)
        dY = np.zeros(3 * nk, np.float64)
        self.lib.orc_sh_basis(nk, _p(d), _p(Y), _p(dY))
        return Y, dY.reshape(nk, 3)

    # -- whole pipeline -------------------------------------------------------
    def forward(self, P, scene, cams, background=None):
        """Projection, binning, sort, ranges and tiled rasterization."""
        proj = self.project(P, scene["means"], scene["quats"], scene["scales"], scene["opacities"],
                            scene["sh"], cams["viewmats"], cams["Ks"], cams["W"], cams["H"])
        isect = self.intersect(P, proj, cams["W"], cams["H"])
        ras = self.rasterize_fwd(P, proj, scene["opacities"], isect["ranges"], isect["ids"], cams["W"],
                                 cams["H"], background=background)
        return proj, isect, ras

    def backward(self, P, scene, cams, proj, isect, ras, v_image, v_alpha=None, background=None):
        g2 = self.rasterize_bwd(P, proj, scene["opacities"], isect["ranges"], isect["ids"], cams["W"],
                                cams["H"], ras["final_T"], ras["last_ids"], v_image, v_alpha, background)
        g3 = self.project_bwd(P, scene["means"], scene["quats"], scene["scales"], scene["opacities"],
                              scene["sh"], cams["viewmats"], cams["Ks"], cams["W"], cams["H"],
                              g2["v_means2d"], g2["v_conics"], g2["v_colors"], g2["v_opacities"])
        return g2, g3
