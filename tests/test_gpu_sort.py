"""The library's stable radix sort (field pull-back order, deterministic
adjoint grouping) against numpy's stable sort: every key and value equal,
equal keys in input order, on ragged sizes around the 4096-pair tile."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    from paper_2406_16360_amd import mirres   # fails loudly if libmirres.so is missing
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return mirres


def _keys(rng, n, kind):
    if kind == "uniform":
        return rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    if kind == "few":            # heavy duplicates: stability decides the value order
        return rng.choice(np.array([3, 0x00FF00FF, 0xFFFFFFFF, 7 << 24, 12345], np.uint32), size=n)
    # the two key shapes the library sorts: 30-bit Morton codes or record
    # words, with the empty marker 0xFFFFFFFF
    k = rng.integers(0, 2**30, size=n, dtype=np.uint64).astype(np.uint32)
    k[rng.random(n) < 0.2] = 0xFFFFFFFF
    return k


@pytest.mark.parametrize("n", [1, 7, 4095, 4096, 4097, 100003, 3 * (1 << 20) + 17])
@pytest.mark.parametrize("kind", ["uniform", "few", "morton"])
def test_sort_matches_stable_sort(mr, n, kind):
    rng = np.random.default_rng(n * 31 + len(kind))
    keys = _keys(rng, n, kind)
    vals = np.arange(n, dtype=np.uint32) ^ np.uint32(0x5A5A5A5A)
    ko, vo = mr.sort_pairs(torch.from_numpy(keys.view(np.int32)).cuda(), torch.from_numpy(vals.view(np.int32)).cuda())
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(ko.cpu().numpy().view(np.uint32), keys[order])
    assert np.array_equal(vo.cpu().numpy().view(np.uint32), vals[order])


def test_sort_rejects_bad_arguments(mr):
    lib = mr.lib()
    k = torch.zeros(16, dtype=torch.int32, device="cuda")
    v = torch.zeros(16, dtype=torch.int32, device="cuda")
    o = torch.zeros(16, dtype=torch.int32, device="cuda")
    need = int(lib.mrs_sort_pairs_tmp_bytes(16))
    tmp = torch.zeros(need, dtype=torch.uint8, device="cuda")
    st = lib.mrs_sort_pairs_u32(k.data_ptr(), k.data_ptr(), v.data_ptr(), o.data_ptr(), 16, tmp.data_ptr(), need, None)
    assert st == mr.MRS_EINVAL and b"must not be the inputs" in lib.mrs_last_error()
    st = lib.mrs_sort_pairs_u32(k.data_ptr(), o.data_ptr(), v.data_ptr(), tmp.data_ptr(), 16, tmp.data_ptr(), need - 1,
                                None)
    assert st == mr.MRS_EINVAL and b"scratch" in lib.mrs_last_error()
    st = lib.mrs_sort_pairs_u32(k.data_ptr(), o.data_ptr(), v.data_ptr(), o.data_ptr(), -1, tmp.data_ptr(), need, None)
    assert st == mr.MRS_EINVAL
    with pytest.raises(ValueError):
        mr.sort_pairs(k, torch.zeros(15, dtype=torch.int32, device="cuda"))
