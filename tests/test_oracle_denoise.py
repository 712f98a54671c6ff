"""Pins of the FP64 denoiser reference (oracle/denoise.py) against what the
definition fixes independently of its code: finite differences, the plain
B3 a-trous convolution it reduces to without edge-stopping, invariants of the
normalised weights, the separation each edge-stopping term enforces, and the
pinhole camera of the G-buffer."""
import numpy as np
import pytest

from oracle import denoise as dn
from paper_2406_16360_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


class V:
    def __init__(self, w, h, c2w=None, fov=40.0):
        self.w, self.h = w, h
        self.c2w = np.eye(4) if c2w is None else c2w
        self.fov_y_deg = fov


def _rand_buffers(rng, views):
    P = sum(v.w * v.h for v in views)
    c = rng.random((P, 3)) * 2
    n = rng.normal(size=(P, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    x = rng.normal(size=(P, 3)) * 0.3
    return c, n, x


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    views = [V(7, 6), V(4, 5)]
    c, n, x = _rand_buffers(rng, views)
    g = rng.normal(size=c.shape)
    kw = dict(levels=3, s_rt=0.8, s_n=0.7, s_x=0.6)
    grad = dn.denoise_grad(c, n, x, g, views, **kw)
    h = 1e-6
    for idx in [(0, 0), (5, 1), (17, 2), (41, 0), (45, 2), (61, 1)]:
        cp, cm = c.copy(), c.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = ((dn.denoise(cp, n, x, views, **kw) - dn.denoise(cm, n, x, views, **kw)) * g).sum() / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-7 + 1e-6 * abs(fd), (idx, fd, grad[idx])


def _atrous_convolution(img, levels):
    """Plain separable B3 a-trous smoothing with numpy.convolve (no weights,
    no boundary handling: valid only away from the borders)."""
    k = np.array([1, 4, 6, 4, 1], np.float64) / 16
    out = img.copy()
    for i in range(levels):
        s = 2 ** i
        kd = np.zeros(4 * s + 1)
        kd[::s] = k
        out = np.apply_along_axis(lambda r: np.convolve(r, kd, mode="same"), 0, out)
        out = np.apply_along_axis(lambda r: np.convolve(r, kd, mode="same"), 1, out)
    return out


def test_without_edge_stopping_is_the_b3_atrous_convolution():
    rng = np.random.default_rng(1)
    views = [V(40, 36)]
    c, n, x = _rand_buffers(rng, views)
    out = dn.denoise(c, n, x, views, levels=3, s_rt=1e12, s_n=1e12, s_x=1e12).reshape(36, 40, 3)
    ref = _atrous_convolution(c.reshape(36, 40, 3), 3)
    m = 2 * (1 + 2 + 4)                      # the interior the three levels reach from
    np.testing.assert_allclose(out[m:-m, m:-m], ref[m:-m, m:-m], rtol=1e-12, atol=1e-12)


def test_constant_colour_is_unchanged():
    rng = np.random.default_rng(2)
    views = [V(9, 8), V(5, 3)]
    _, n, x = _rand_buffers(rng, views)
    c = np.tile(np.array([[0.3, 1.7, 0.05]]), (n.shape[0], 1))
    out = dn.denoise(c, n, x, views, levels=3, s_rt=0.2, s_n=0.3, s_x=0.4)
    np.testing.assert_allclose(out, c, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("term", ["normal", "position", "colour"])
def test_each_edge_stopping_term_separates_regions(term):
    """Left and right halves differ strongly in one buffer only; with that
    buffer's sigma small, the left half's result ignores the right half's
    colours, and with all sigmas large it does not."""
    rng = np.random.default_rng(3)
    v = V(12, 10)
    P = v.w * v.h
    n = np.tile([[0.0, 0.0, 1.0]], (P, 1))
    x = np.zeros((P, 3))
    c = rng.random((P, 3)) * 0.1 + 0.5
    right = (np.arange(P) % v.w) >= v.w // 2
    s = dict(s_rt=1e6, s_n=1e6, s_x=1e6)
    if term == "normal":
        n[right] = [1.0, 0.0, 0.0]
        s["s_n"] = 0.05
    elif term == "position":
        x[right] = [0.0, 0.0, 5.0]
        s["s_x"] = 0.05
    else:
        c[right] += 20.0
        s["s_rt"] = 0.05
    c2 = c.copy()
    c2[right] += 3.0 if term != "colour" else 7.0
    a = dn.denoise(c, n, x, [v], levels=3, **s)
    b = dn.denoise(c2, n, x, [v], levels=3, **s)
    np.testing.assert_allclose(a[~right], b[~right], rtol=0, atol=1e-12)
    loose = dict(s_rt=1e6, s_n=1e6, s_x=1e6)
    a = dn.denoise(c, n, x, [v], levels=3, **loose)
    b = dn.denoise(c2, n, x, [v], levels=3, **loose)
    assert np.abs(a[~right] - b[~right]).max() > 1e-3


def test_views_are_filtered_independently():
    rng = np.random.default_rng(4)
    views = [V(6, 5), V(8, 4)]
    c, n, x = _rand_buffers(rng, views)
    both = dn.denoise(c, n, x, views)
    first = dn.denoise(c[:30], n[:30], x[:30], views[:1])
    np.testing.assert_array_equal(both[:30], first)


def test_pixel_center_camera():
    """Odd-sized view: the centre pixel looks down -z of the camera; the
    rays through the centres of the top and bottom rows span the vertical
    field of view less one pixel."""
    c2w = synth.look_at(np.array([0.0, 1.0, 3.0]))
    v = V(41, 31, np.asarray(c2w), fov=50.0)
    o, d = dn.pixel_center_rays(v)
    R = np.asarray(c2w, np.float64).reshape(4, 4)[:3, :3]
    np.testing.assert_allclose(d[15 * 41 + 20], -R[:, 2], atol=1e-12)
    top, bottom = d[0 * 41 + 20], d[30 * 41 + 20]
    ang = np.arccos(np.clip(top @ bottom, -1, 1))
    th = np.tan(np.deg2rad(25.0))
    expect = 2 * np.arctan(th * (31 - 1) / 31)
    assert abs(ang - expect) < 1e-12
    np.testing.assert_allclose(o, np.broadcast_to(np.asarray(c2w, np.float64).reshape(4, 4)[:3, 3], o.shape))
