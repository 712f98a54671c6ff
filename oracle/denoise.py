"""FP64 reference of the edge-avoiding a-trous wavelet denoiser and of its
G-buffer (the paper's "Denoiser" paragraph in Appendix A, after Dammertz et
al., "Edge-avoiding a-trous wavelet transform for fast global illumination
filtering", HPG 2010).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's CPU
baseline leg, never by the GPU product path.

Definition (one view, pixels p, q on its grid):
  level i = 0, 1, 2 filters c_i into c_{i+1} with the B3-spline taps
  h = (1, 4, 6, 4, 1) / 16 in x and in y, spaced 2^i pixels apart;
      a(p, q)   = h(dx) h(dy) w_rt w_n w_x
      w_rt      = exp(-|c_i(p) - c_i(q)|^2 / s_rt^2)   (colour of the level's input)
      w_n       = exp(-|n(p) - n(q)|^2 / s_n^2)         (normal buffer)
      w_x       = exp(-|x(p) - x(q)|^2 / s_x^2)         (position buffer)
      k(p)      = sum_q a(p, q)
      c_{i+1}(p) = sum_q a(p, q) c_i(q) / k(p)
  Taps outside the view are left out of both sums.
The gradient is reverse-mode differentiation of exactly this computation
(torch autograd on the CPU, float64); nothing is held fixed.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import torch

B3 = (1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16)


def _shift(a: torch.Tensor, oy: int, ox: int) -> Tuple[torch.Tensor, torch.Tensor]:
    """a[y + oy, x + ox] for every (y, x), and a mask of where that pixel exists."""
    H, W = a.shape[:2]
    out = torch.zeros_like(a)
    valid = torch.zeros((H, W), dtype=torch.bool)
    ys, ye = max(0, -oy), min(H, H - oy)
    xs, xe = max(0, -ox), min(W, W - ox)
    if ys < ye and xs < xe:
        out[ys:ye, xs:xe] = a[ys + oy:ye + oy, xs + ox:xe + ox]
        valid[ys:ye, xs:xe] = True
    return out, valid


def eawt_level(c: torch.Tensor, n: torch.Tensor, x: torch.Tensor, stride: int, s_rt: float, s_n: float,
               s_x: float) -> Tuple[torch.Tensor, torch.Tensor]:
    """One a-trous level on one view: c, n, x are [H, W, 3].  Returns c_{i+1}
    and the normalisation k."""
    num = torch.zeros_like(c)
    k = torch.zeros(c.shape[:2], dtype=c.dtype)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            cq, valid = _shift(c, dy * stride, dx * stride)
            nq, _ = _shift(n, dy * stride, dx * stride)
            xq, _ = _shift(x, dy * stride, dx * stride)
            w_rt = torch.exp(-((c - cq) ** 2).sum(-1) / s_rt ** 2)
            w_n = torch.exp(-((n - nq) ** 2).sum(-1) / s_n ** 2)
            w_x = torch.exp(-((x - xq) ** 2).sum(-1) / s_x ** 2)
            a = B3[dy + 2] * B3[dx + 2] * w_rt * w_n * w_x * valid
            num = num + a[..., None] * cq
            k = k + a
    return num / k[..., None], k


def eawt(c0: torch.Tensor, n: torch.Tensor, x: torch.Tensor, levels: int = 3, s_rt: float = 1.0,
         s_n: float = 0.5, s_x: float = 0.5) -> torch.Tensor:
    """All levels on one view ([H, W, 3] tensors)."""
    c = c0
    for i in range(levels):
        c, _ = eawt_level(c, n, x, 2 ** i, s_rt, s_n, s_x)
    return c


def _views(img: np.ndarray, views: Sequence) -> List[np.ndarray]:
    out, off = [], 0
    for v in views:
        out.append(img[off:off + v.w * v.h].reshape(v.h, v.w, 3))
        off += v.w * v.h
    return out


def denoise(color: np.ndarray, normal: np.ndarray, position: np.ndarray, views: Sequence, levels: int = 3,
            s_rt: float = 1.0, s_n: float = 0.5, s_x: float = 0.5) -> np.ndarray:
    """Packed images [sum_v W_v H_v, 3] (views in order, rows top to bottom)."""
    res = []
    for c, n, x in zip(_views(color, views), _views(normal, views), _views(position, views)):
        t = lambda a: torch.tensor(np.asarray(a, np.float64))
        res.append(eawt(t(c), t(n), t(x), levels, s_rt, s_n, s_x).numpy().reshape(-1, 3))
    return np.concatenate(res, 0)


def denoise_grad(color: np.ndarray, normal: np.ndarray, position: np.ndarray, grad_out: np.ndarray,
                 views: Sequence, levels: int = 3, s_rt: float = 1.0, s_n: float = 0.5,
                 s_x: float = 0.5) -> np.ndarray:
    """d(sum grad_out . denoise(color)) / d color, by autograd of the forward."""
    res = []
    for c, n, x, g in zip(_views(color, views), _views(normal, views), _views(position, views),
                          _views(grad_out, views)):
        ct = torch.tensor(np.asarray(c, np.float64), requires_grad=True)
        out = eawt(ct, torch.tensor(np.asarray(n, np.float64)), torch.tensor(np.asarray(x, np.float64)), levels,
                   s_rt, s_n, s_x)
        (gc,) = torch.autograd.grad(out, ct, torch.tensor(np.asarray(g, np.float64)))
        res.append(gc.numpy().reshape(-1, 3))
    return np.concatenate(res, 0)


# ---------------------------------------------------------------- G-buffer
def pixel_center_rays(view) -> Tuple[np.ndarray, np.ndarray]:
    """Pinhole rays through the pixel centres of one view, in float64: the
    camera of the renderer with the sub-pixel offset fixed at (1/2, 1/2)."""
    c2w = np.asarray(view.c2w, np.float64).reshape(4, 4)
    th = np.tan(np.deg2rad(view.fov_y_deg) / 2)
    aspect = view.w / view.h
    ys, xs = np.mgrid[0:view.h, 0:view.w]
    nx = 2.0 * (xs + 0.5) / view.w - 1.0
    ny = 1.0 - 2.0 * (ys + 0.5) / view.h
    dc = np.stack([nx * th * aspect, ny * th, -np.ones_like(nx)], -1).reshape(-1, 3)
    d = dc @ c2w[:3, :3].T
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(c2w[:3, 3], d.shape).copy()
    return o, d


def gbuffer(orc, scene, views) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Position o + t d and unit geometric normal facing the camera of the
    closest hit at every pixel centre (zeros where the ray misses), with the
    hit face id (-1 on a miss).  orc is an oracle.Oracle over `scene`."""
    pos, nrm, ids = [], [], []
    P = np.asarray(scene.pos, np.float64)
    F = np.asarray(scene.faces, np.int64)
    for v in views:
        o, d = pixel_center_rays(v)
        prim, t, _, _ = orc.trace(o, d)
        hit = prim >= 0
        x = np.zeros_like(o)
        nn = np.zeros_like(o)
        x[hit] = o[hit] + t[hit, None] * d[hit]
        f = F[prim[hit]]
        g = np.cross(P[f[:, 1]] - P[f[:, 0]], P[f[:, 2]] - P[f[:, 0]])
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        g[(g * d[hit]).sum(1) > 0] *= -1.0
        nn[hit] = g
        pos.append(x)
        nrm.append(nn)
        ids.append(prim)
    return np.concatenate(pos), np.concatenate(nrm), np.concatenate(ids)
