"""The C-ABI library loads on a host without a GPU, exports every entry
point include/gsraster.h declares, and rejects bad arguments before touching
the device (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsraster.h")
LIB = os.path.join(ROOT, "paper_2409_06765_amd", "libgsraster.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libgsraster.so is not built (python -m paper_2409_06765_amd.build)")
    from paper_2409_06765_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported(L):
    syms = declared_symbols()
    assert len(syms) >= 12
    lib = L.lib()
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L._SIGS), "binding and header disagree"


def test_version_and_defaults(L):
    hdr = open(HEADER).read()
    assert L.abi_version() == int(re.search(r"#define GSR_ABI_VERSION (\d+)", hdr).group(1)) == L.ABI_VERSION
    p = L.default_params()
    assert p.tile == 16 and p.sh_degree == -1 and p.antialiased == 0
    import numpy as np
    assert np.float32(p.alpha_min) == np.float32(1.0) / np.float32(255.0)
    assert np.float32(p.alpha_max) == np.float32(0.99)
    assert np.float32(p.T_min) == np.float32(1e-4)
    assert np.float32(p.near_plane) == np.float32(0.01) and p.far_plane == float("inf")
    assert np.float32(p.eps2d) == np.float32(0.3) and np.float32(p.jac_clamp) == np.float32(1.3)


def test_defaults_match_the_oracle_constants(L):
    from oracle import OracleParams
    import numpy as np
    p, o = L.default_params(), OracleParams()
    for k in ("near_plane", "eps2d", "jac_clamp", "alpha_min", "alpha_max", "T_min"):
        assert np.float32(getattr(p, k)) == np.float32(getattr(o, k)), k


def test_workspace_sizes(L):
    assert L.workspace_bytes(L.GSR_OP_INTERSECT_COUNT, 1, 10_000, 0) >= 8 * (10_000 // 1024)
    assert L.workspace_bytes(L.GSR_OP_SORT, 0, 0, 5_000_000) >= 256 * 4 * (5_000_000 // 2048)
    assert L.workspace_bytes(99, 1, 1, 1) == 0


def _call_project(L, p, C=1, N=4, W=(64,), H=(64,), null_means=False):
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    Wa = (ctypes.c_int32 * max(C, 1))(*W)
    Ha = (ctypes.c_int32 * max(C, 1))(*H)
    args = [None if null_means else fake] + [fake] * 6 + [fake] * 5 + [None]
    return lib.gsr_project_fwd(ctypes.byref(p) if p is not None else None, C, N, Wa, Ha, *args, None)


def test_argument_validation_happens_before_any_launch(L):
    p = L.default_params()
    assert _call_project(L, None) == L.GSR_EINVAL
    assert "params" in L.lib().gsr_last_error().decode()
    bad = L.default_params(tile=8)
    assert _call_project(L, bad) == L.GSR_EINVAL
    bad = L.default_params(sh_degree=4)
    assert _call_project(L, bad) == L.GSR_EINVAL
    bad = L.default_params(alpha_max=1.5)
    assert _call_project(L, bad) == L.GSR_EINVAL
    assert _call_project(L, p, C=65, W=[64] * 65, H=[64] * 65) == L.GSR_EINVAL
    assert _call_project(L, p, N=-1) == L.GSR_EINVAL
    assert _call_project(L, p, W=(0,)) == L.GSR_EINVAL
    assert _call_project(L, p, H=(20000,)) == L.GSR_EINVAL
    assert _call_project(L, p, null_means=True) == L.GSR_EINVAL
    assert "means" in L.lib().gsr_last_error().decode()
    # empty problems are valid no-ops
    assert _call_project(L, p, N=0) == L.GSR_OK


def test_sort_and_workspace_validation(L):
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    assert lib.gsr_sort_pairs(-1, 40, fake, fake, fake, fake, fake, 1 << 20, None) == L.GSR_EINVAL
    assert lib.gsr_sort_pairs(100, 65, fake, fake, fake, fake, fake, 1 << 20, None) == L.GSR_EINVAL
    assert lib.gsr_sort_pairs(100_000, 40, fake, fake, fake, fake, fake, 16, None) == L.GSR_EWORKSPACE
    assert lib.gsr_sort_pairs(1, 40, None, None, None, None, None, 0, None) == L.GSR_OK
    # the scratch-free sort checks its size limit before it looks up its device array
    assert lib.gsr_sort_pairs_noalloc((1 << 25) + 1, 40, fake, fake, fake, fake, None) == L.GSR_EINVAL
    assert "0..33554432" in lib.gsr_last_error().decode()
    assert lib.gsr_sort_pairs_noalloc(100, 0, fake, fake, fake, fake, None) == L.GSR_EINVAL
    assert lib.gsr_sort_pairs_noalloc(1, 40, None, None, None, None, None) == L.GSR_OK
    p = L.default_params()
    W = (ctypes.c_int32 * 1)(64)
    assert lib.gsr_intersect_count(ctypes.byref(p), 1, 5000, W, W, fake, fake, fake, fake, fake, None, fake, 8,
                                   None) == L.GSR_EWORKSPACE
    assert lib.gsr_intersect_emit(ctypes.byref(p), 1, 10, W, W, fake, fake, fake, fake, -5, fake, fake,
                                  None) == L.GSR_EINVAL
    # the fill kernel's entry point: whole aligned words only, empty is a no-op
    assert lib.gsr_fill_zero(fake, 6, None) == L.GSR_EINVAL
    assert lib.gsr_fill_zero(ctypes.c_void_p(0x1002), 8, None) == L.GSR_EINVAL
    assert lib.gsr_fill_zero(None, 8, None) == L.GSR_EINVAL
    assert lib.gsr_fill_zero(None, 0, None) == L.GSR_OK


def test_training_entry_points_reject_bad_arguments(L):
    """The training-loop calls validate before any launch (fake pointers are
    never dereferenced)."""
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.workspace_bytes(L.GSR_OP_L1_LOSS, 0, 0, 10) >= 8
    assert L.workspace_bytes(L.GSR_OP_DENSIFY_PLAN, 0, 1_000_000, 0) >= 4_000_000
    # L1: negative n, aliasing, small workspace
    assert lib.gsr_l1_loss(-1, fake, fake, 1.0, fake, fake, fake, 1 << 20, None) == L.GSR_EINVAL
    assert lib.gsr_l1_loss(8, fake, fake, 1.0, fake, fake, fake, 1 << 20, None) == L.GSR_EINVAL
    assert lib.gsr_l1_loss(8, fake, ctypes.c_void_p(0x2000), 1.0, ctypes.c_void_p(0x3000), fake, fake, 8,
                           None) == L.GSR_EWORKSPACE
    # Adam: group count, step, betas, reg without an activation
    g = (L.gsr_adam_group * 1)()
    g[0].param = g[0].grad = g[0].exp_avg = g[0].exp_avg_sq = 0x1000
    g[0].n, g[0].lr = 4, 0.1
    assert lib.gsr_adam_step(L.GSR_ADAM_MAX_GROUPS + 1, g, 1, 0.9, 0.999, 1e-15, None) == L.GSR_EINVAL
    assert lib.gsr_adam_step(1, g, 0, 0.9, 0.999, 1e-15, None) == L.GSR_EINVAL
    assert lib.gsr_adam_step(1, g, 1, 1.0, 0.999, 1e-15, None) == L.GSR_EINVAL
    g[0].reg = 0.5
    assert lib.gsr_adam_step(1, g, 1, 0.9, 0.999, 1e-15, None) == L.GSR_EINVAL
    assert "reg" in lib.gsr_last_error().decode()
    g[0].reg, g[0].activation = 0.0, 7
    assert lib.gsr_adam_step(1, g, 1, 0.9, 0.999, 1e-15, None) == L.GSR_EINVAL
    g[0].activation, g[0].grad = L.GSR_ACT_EXP, None
    assert lib.gsr_adam_step(1, g, 1, 0.9, 0.999, 1e-15, None) == L.GSR_EINVAL
    # plan: N range, NaN thresholds, workspace
    assert lib.gsr_densify_plan(-1, fake, fake, fake, fake, 2e-4, 0.01, 0.005, fake, fake, None, fake, 1 << 30,
                                None) == L.GSR_EINVAL
    assert lib.gsr_densify_plan(4, fake, fake, fake, fake, float("nan"), 0.01, 0.005, fake, fake, None, fake,
                                1 << 30, None) == L.GSR_EINVAL
    assert lib.gsr_densify_plan(4096, fake, fake, fake, fake, 2e-4, 0.01, 0.005, fake, fake, None, fake, 16,
                                None) == L.GSR_EWORKSPACE
    # apply: column kinds, widths, aliasing, split inputs
    cols = (L.gsr_densify_column * 2)()
    cols[0].src, cols[0].dst, cols[0].width, cols[0].kind = 0x1000, 0x2000, 3, L.GSR_COLUMN_MEANS
    cols[1].src, cols[1].dst, cols[1].width, cols[1].kind = 0x3000, 0x4000, 2, L.GSR_COLUMN_LOG_SCALES
    assert lib.gsr_densify_apply(4, fake, fake, fake, fake, fake, 1.6, 2, cols, None) == L.GSR_EINVAL
    cols[1].width = 3
    assert lib.gsr_densify_apply(4, fake, fake, None, fake, fake, 1.6, 2, cols, None) == L.GSR_EINVAL
    assert lib.gsr_densify_apply(4, fake, fake, fake, fake, fake, 0.0, 2, cols, None) == L.GSR_EINVAL
    cols[1].kind = 9
    assert lib.gsr_densify_apply(4, fake, fake, fake, fake, fake, 1.6, 2, cols, None) == L.GSR_EINVAL
    cols[1].kind, cols[1].dst = L.GSR_COLUMN_COPY, 0x3000
    assert lib.gsr_densify_apply(4, fake, fake, fake, fake, fake, 1.6, 2, cols, None) == L.GSR_EINVAL
    assert lib.gsr_densify_apply(4, fake, fake, fake, fake, fake, 1.6, L.GSR_DENSIFY_MAX_COLUMNS + 1, cols,
                                 None) == L.GSR_EINVAL
    # opacity reset and MCMC noise
    assert lib.gsr_opacity_reset(4, fake, fake, fake, None, 1.0, None) == L.GSR_EINVAL
    assert lib.gsr_opacity_reset(4, fake, None, fake, None, 0.01, None) == L.GSR_EINVAL
    assert lib.gsr_mcmc_noise(4, fake, fake, fake, fake, None, 1.0, 100.0, 0.005, None) == L.GSR_EINVAL
    assert lib.gsr_mcmc_noise(4, fake, fake, fake, fake, fake, float("inf"), 100.0, 0.005, None) == L.GSR_EINVAL
    # zero sizes are no-ops
    assert lib.gsr_opacity_reset(0, None, None, None, None, 0.01, None) == L.GSR_OK
    assert lib.gsr_mcmc_noise(0, None, None, None, None, None, 1.0, 100.0, 0.005, None) == L.GSR_OK
    assert lib.gsr_densify_apply(0, None, None, None, None, None, 1.6, 0, None, None) == L.GSR_OK


def test_grad_records_layout_is_validated(L):
    """params.grad_records: 0 or 1; only plain RGB (D = 3, no depth channel, colours per camera); the
    three other gradient pointers NULL.  All rejected before anything is enqueued (fake pointers)."""
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    W = (ctypes.c_int32 * 1)(64)

    def bwd(p, D=3, v_conics=None, v_colors=None, v_opac=None):
        # p, C, N, D, W, H; means2d conics colors depths opacities comps background; ranges ids order;
        # image final_T last_ids; v_image v_alpha; v_means2d v_conics v_colors v_depths v_opac v_abs; ws flags
        return lib.gsr_rasterize_bwd(ctypes.byref(p), 1, 8, D, W, W, fake, fake, fake, fake, fake, None, None,
                                     fake, fake, None, None, fake, fake, fake, None, fake, v_conics, v_colors,
                                     fake if p.render_depth else None, v_opac, None, fake, 1 << 30, 0, None)

    def pbwd(p, v_conics=None, v_colors=None, v_opac=None):
        return lib.gsr_project_bwd(ctypes.byref(p), 1, 8, W, W, fake, fake, fake, fake, fake, fake, fake, fake,
                                   None, fake, v_conics, v_colors, v_opac, None, fake, fake, fake, fake, fake,
                                   None, None, 0, None)

    assert bwd(L.default_params(grad_records=2)) == L.GSR_EINVAL
    assert "grad_records" in lib.gsr_last_error().decode()
    rec = L.default_params(grad_records=1, sh_degree=3)
    assert bwd(rec, D=4) == L.GSR_EINVAL
    assert bwd(L.default_params(grad_records=1, render_depth=1), D=3) == L.GSR_EINVAL
    assert bwd(L.default_params(grad_records=1, colors_shared=1)) == L.GSR_EINVAL
    assert bwd(rec, v_conics=fake) == L.GSR_EINVAL
    assert "NULL" in lib.gsr_last_error().decode()
    assert bwd(rec, v_colors=fake) == L.GSR_EINVAL
    assert bwd(rec, v_opac=fake) == L.GSR_EINVAL
    assert pbwd(rec, v_conics=fake) == L.GSR_EINVAL
    assert pbwd(rec, v_opac=fake) == L.GSR_EINVAL
    assert pbwd(L.default_params(grad_records=1, colors_shared=1)) == L.GSR_EINVAL
    # the four-array layout still needs its arrays
    assert bwd(L.default_params(sh_degree=3)) == L.GSR_EINVAL
    assert pbwd(L.default_params(sh_degree=3)) == L.GSR_EINVAL
