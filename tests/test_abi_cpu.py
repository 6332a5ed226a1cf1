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
    p = L.default_params()
    W = (ctypes.c_int32 * 1)(64)
    assert lib.gsr_intersect_count(ctypes.byref(p), 1, 5000, W, W, fake, fake, fake, fake, fake, None, fake, 8,
                                   None) == L.GSR_EWORKSPACE
    assert lib.gsr_intersect_emit(ctypes.byref(p), 1, 10, W, W, fake, fake, fake, fake, -5, fake, fake,
                                  None) == L.GSR_EINVAL
