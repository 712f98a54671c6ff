"""GPU parity of the denoiser row: G-buffer, EAWT forward and its adjoint
against the FP64 reference (oracle/denoise.py) on the same seeded inputs."""
import numpy as np
import pytest
import torch

from paper_2406_16360_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    from paper_2406_16360_amd import mirres   # fails loudly if libmirres.so is missing
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return mirres


@pytest.fixture(scope="module")
def dn():
    from oracle import denoise
    return denoise


class V:
    def __init__(self, w, h):
        self.w, self.h, self.spp = w, h, 1
        self.c2w = np.eye(4, dtype=np.float32)
        self.fov_y_deg = 40.0


def _buffers(seed, views):
    """Seeded colour with flat patches and edges, normals and positions of a
    few planes, so the edge-stopping weights span their whole range."""
    rng = np.random.default_rng(seed)
    cs, ns, xs = [], [], []
    for v in views:
        yy, xx = np.mgrid[0:v.h, 0:v.w]
        region = ((xx * 3) // max(v.w, 1) + 2 * ((yy * 2) // max(v.h, 1))) % 4
        base = np.array([[0.2, 0.4, 0.9], [1.5, 0.3, 0.2], [0.6, 0.6, 0.6], [3.0, 2.0, 0.1]])[region]
        c = base + rng.normal(scale=0.3, size=base.shape) * rng.random((v.h, v.w, 1))
        nrm = np.array([[0, 0, 1.0], [0, 1.0, 0], [0.6, 0, 0.8], [-0.8, 0.6, 0]])[region]
        pos = np.stack([xx / v.w, yy / v.h, region * 0.3], -1) + rng.normal(scale=0.01, size=(v.h, v.w, 3))
        cs.append(c.reshape(-1, 3)); ns.append(nrm.reshape(-1, 3)); xs.append(pos.reshape(-1, 3))
    f = lambda a: np.concatenate(a).astype(np.float32)
    return f(cs), f(ns), f(xs)


VIEW_SETS = {
    "uneven": [V(37, 29), V(64, 48), V(20, 33)],
    "tiny": [V(1, 1), V(3, 2), V(2, 7), V(16, 1)],     # views smaller than a tile or an apron
    "full": [V(800, 800), V(333, 517)],                # the rendered views' size, and a ragged one
}


@pytest.mark.parametrize("vset", list(VIEW_SETS))
@pytest.mark.parametrize("levels", [1, 3])
def test_denoise_forward_and_adjoint(mr, dn, vset, levels):
    views = VIEW_SETS[vset]
    c, n, x = _buffers(11, views)
    sig = dict(s_rt=0.7, s_n=0.5, s_x=0.3)
    ref = dn.denoise(c, n, x, views, levels=levels, **sig)
    den = mr.Denoiser(views, torch.tensor(n, device="cuda"), torch.tensor(x, device="cuda"), levels=levels,
                      sigma_rt=sig["s_rt"], sigma_n=sig["s_n"], sigma_x=sig["s_x"])
    out = den.forward(torch.tensor(c, device="cuda")).cpu().numpy()
    err = np.abs(out - ref) / (np.abs(ref) + 1e-3)
    print(f"   forward {vset} L={levels}: max rel err {err.max():.2e}")
    assert err.max() < 2e-5
    g = np.random.default_rng(12).normal(size=c.shape).astype(np.float32)
    gref = dn.denoise_grad(c, n, x, g, views, levels=levels, **sig)
    gout = den.backward(torch.tensor(g, device="cuda")).cpu().numpy()
    scale = np.abs(gref).max()
    gerr = np.abs(gout - gref) / scale
    print(f"   adjoint {vset} L={levels}: max err / max |grad| {gerr.max():.2e}")
    assert gerr.max() < 1e-4


def test_denoise_autograd(mr, dn):
    views = VIEW_SETS["uneven"]
    c, n, x = _buffers(13, views)
    den = mr.Denoiser(views, torch.tensor(n, device="cuda"), torch.tensor(x, device="cuda"))
    ct = torch.tensor(c, device="cuda", requires_grad=True)
    w = torch.tensor(np.random.default_rng(14).random(c.shape).astype(np.float32), device="cuda")
    (mr.denoise_autograd(ct, den) * w).sum().backward()
    gref = dn.denoise_grad(c, n, x, w.cpu().numpy(), views)
    assert np.abs(ct.grad.cpu().numpy() - gref).max() < 1e-4 * np.abs(gref).max()


def test_gbuffer_matches_oracle(mr):
    from oracle import denoise as odn
    from oracle.oracle import Oracle
    w = synth.config1()
    views = w.views[:2]
    sc = mr.GpuScene.from_synth(w.scene)
    pos, nrm = mr.gbuffer(sc, views)
    pos, nrm = pos.cpu().numpy(), nrm.cpu().numpy()
    opos, onrm, oid = odn.gbuffer(Oracle(w.scene), w.scene, views)
    ghit = np.abs(nrm).sum(1) > 0
    ohit = oid >= 0
    assert np.mean(ghit == ohit) >= 0.999
    both = ghit & ohit
    same_face = np.abs((nrm[both] * onrm[both]).sum(1)) > 0.99999
    assert same_face.mean() >= 0.995
    d = np.linalg.norm(pos[both] - opos[both], axis=1) / np.maximum(1e-3, np.linalg.norm(opos[both], axis=1))
    assert np.quantile(d[same_face], 0.999) < 1e-5
    np.testing.assert_allclose(np.linalg.norm(nrm[ghit], axis=1), 1.0, atol=1e-5)
    assert np.all(pos[~ghit] == 0) and np.all(nrm[~ghit] == 0)


def test_denoise_rejects_bad_parameters(mr):
    views = [V(8, 8)]
    z = torch.zeros((64, 3), device="cuda")
    with pytest.raises(mr.MirresError):
        mr.Denoiser(views, z, z, levels=4)
    with pytest.raises(mr.MirresError):
        mr.Denoiser(views, z, z, sigma_rt=0.0)


def test_denoise_autograd_refuses_a_stale_workspace(mr):
    """Two differentiable denoises through one Denoiser: the first one's
    backward would read the second one's levels, so it raises."""
    views = VIEW_SETS["uneven"]
    c, n, x = _buffers(15, views)
    den = mr.Denoiser(views, torch.tensor(n, device="cuda"), torch.tensor(x, device="cuda"))
    ct = torch.tensor(c, device="cuda", requires_grad=True)
    a = mr.denoise_autograd(ct, den)
    b = mr.denoise_autograd(ct * 2.0, den)
    with pytest.raises(RuntimeError, match="another forward"):
        a.sum().backward()
    # the latest call still differentiates
    ct.grad = None
    b2 = mr.denoise_autograd(ct, den)
    b2.sum().backward()
    assert torch.isfinite(ct.grad).all()
    del b
