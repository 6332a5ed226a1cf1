"""gsr_sort_pairs_noalloc (the sort without a workspace argument, for callers
that cannot allocate) against gsr_sort_pairs, through the C ABI: two calls
in a row on one device, the second smaller, each bit for bit equal to the
workspace entry point's result and to numpy's stable argsort."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _pairs(M, key_bits, dups, seed):
    g = np.random.default_rng(seed)
    mask = np.uint64((1 << key_bits) - 1) if key_bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    base = g.integers(0, 2 ** 63, size=max(M // dups, 1), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    keys = (base[g.integers(0, base.size, M)] & mask).astype(np.uint64)
    return keys, g.permutation(M).astype(np.int32)


def _sort_both(M, key_bits, dups, seed):
    from paper_2409_06765_amd import _lib as L
    print(f"[no-alloc] M={M} key_bits={key_bits}", flush=True)
    keys, ids = _pairs(M, key_bits, dups, seed)
    order = np.argsort(keys, kind="stable")
    out = []
    for noalloc in (False, True):
        dk, di = torch.from_numpy(keys).cuda(), torch.from_numpy(ids).cuda()
        ka, ia = torch.empty_like(dk), torch.empty_like(di)
        if noalloc:
            L.gsr_sort_pairs_noalloc(M, key_bits, dk, di, ka, ia)
        else:
            ws = torch.empty(max(L.workspace_bytes(L.GSR_OP_SORT, 0, 0, M), 1), dtype=torch.uint8, device="cuda")
            L.gsr_sort_pairs(M, key_bits, dk, di, ka, ia, ws)
        torch.cuda.synchronize()
        out.append((dk.cpu().numpy(), di.cpu().numpy()))
    (k0, i0), (k1, i1) = out
    np.testing.assert_array_equal(k1, k0)
    np.testing.assert_array_equal(i1, i0)
    np.testing.assert_array_equal(k1, keys[order])
    np.testing.assert_array_equal(i1, ids[order])


def test_noalloc_sort_matches_the_workspace_sort_twice():
    # the first call fills the static histograms of a large problem; the second, smaller one must not
    # see any of them (every slot it reads it writes first)
    _sort_both(3_000_017, 45, 7, seed=1)
    _sort_both(70_001, 64, 3, seed=2)


def test_noalloc_sort_rejects_sizes_beyond_its_maximum():
    from paper_2409_06765_amd import _lib as L
    x = torch.empty(2, dtype=torch.uint64, device="cuda")
    y = torch.empty(2, dtype=torch.int32, device="cuda")
    with pytest.raises(L.GsrError) as e:
        L.gsr_sort_pairs_noalloc(L.GSR_SORT_NOALLOC_MAX_PAIRS + 1, 40, x, y, x, y)
    assert e.value.code == L.GSR_EINVAL
