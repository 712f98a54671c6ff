"""The allocation-free denoiser forward (mrs_denoise_noalloc, for callers that
cannot allocate device memory) against mrs_denoise with its workspace, both
called through the C ABI on the same seeded inputs: two calls in a row, the
second on a smaller input, then the host-side rejections."""
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


class V:
    def __init__(self, w, h):
        self.w, self.h, self.spp = w, h, 1
        self.c2w = np.eye(4, dtype=np.float32)
        self.fov_y_deg = 40.0


def _inputs(seed, views):
    """Seeded colour, unit normals and positions with flat regions and edges."""
    rng = np.random.default_rng(seed)
    n = sum(v.w * v.h for v in views)
    c = rng.lognormal(0.0, 1.0, (n, 3)).astype(np.float32)
    nrm = rng.normal(size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    region = rng.integers(0, 3, (n, 1))
    nrm = np.where(region == 0, np.array([[0.0, 0.0, 1.0]]), nrm).astype(np.float32)
    pos = (rng.random((n, 3)) * 0.2 + region * 0.5).astype(np.float32)
    t = lambda a: torch.tensor(a, device="cuda")
    return t(c), t(nrm), t(pos)


def _compare(mr, views, levels, seed):
    c, n, x = _inputs(seed, views)
    sig = dict(sigma_rt=0.8, sigma_n=0.4, sigma_x=0.3)
    ref = mr.Denoiser(views, n, x, levels=levels, **sig).forward(c)
    out = torch.full_like(c, float("nan"))
    mr.denoise_noalloc(views, c, n, x, out, levels=levels, **sig)
    torch.cuda.synchronize()
    diff = (out - ref).abs().max().item()
    print(f"   noalloc {[(v.w, v.h) for v in views]} L={levels}: max |diff| {diff:.3e}", flush=True)
    # the same kernel on the same inputs: identical floats
    assert torch.equal(out, ref)


def test_noalloc_matches_workspace_denoise_twice(mr):
    _compare(mr, [V(37, 29), V(64, 48), V(20, 33)], 3, 21)
    _compare(mr, [V(16, 12)], 2, 22)     # second call, smaller input: the scratch keeps the first's contents
    _compare(mr, [V(5, 3), V(1, 1)], 1, 23)


def test_noalloc_largest_view_that_fits(mr):
    # 1664 x 1680 = 2,795,520 pixels: 24 bytes each at three levels, just under 64 MiB
    _compare(mr, [V(1664, 1680)], 3, 24)


def test_noalloc_rejects_on_the_host(mr):
    lib = mr.lib()
    views = [V(2048, 1400)]            # 2,867,200 pixels: 68.8 MB of scratch at three levels
    vs, npix, _ = mr.views_struct(views)
    bufs = [torch.zeros((npix, 3), device="cuda") for _ in range(4)]
    params = mr._DenoiseParams(3, 1.0, 0.5, 0.5)
    st = lib.mrs_denoise_noalloc(C.addressof(vs), 1, C.byref(params), *[b.data_ptr() for b in bufs], None)
    assert st == mr.MRS_EOVERFLOW
    assert b"scratch" in lib.mrs_last_error()
    # two levels need half of that: it fits
    params2 = mr._DenoiseParams(2, 1.0, 0.5, 0.5)
    assert lib.mrs_denoise_noalloc(C.addressof(vs), 1, C.byref(params2), *[b.data_ptr() for b in bufs], None) == 0
    # output over the input
    st = lib.mrs_denoise_noalloc(C.addressof(vs), 1, C.byref(params2), bufs[0].data_ptr(), bufs[1].data_ptr(),
                                 bufs[2].data_ptr(), bufs[0].data_ptr(), None)
    assert st == mr.MRS_EINVAL
    torch.cuda.synchronize()
