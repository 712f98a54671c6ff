"""Inverse-rendering loop over the differentiable path tracer.

Materials (albedo, roughness, metallic textures) and the HDR environment map
are optimised with Adam against target images rendered from seeded
ground-truth materials, the intrinsic-decomposition part of the paper's
second stage (Sec. 3 "Intrinsic decomposition", loss Eq. loss_pbr).  The
geometry is fixed (vertex optimisation through visibility is not part of
this path).  Each step renders with a fresh Philox seed, so the L2 gradient
is not correlated with the noise of the image it is computed from.

    python -m paper_2406_16360_amd.inverse --steps 200     # the full 1M-tri, 100x800^2 workload
    python -m paper_2406_16360_amd.inverse --small         # a reduced run

With --ckpt PATH the loop saves the textures, the env, Adam's state, the step
and the seen-texel masks every --ckpt-every steps (torch.save of tensors and
numbers only, loaded back with weights_only=True); --resume continues from
PATH.  With deterministic gradients (--deterministic) a resumed run gives the
same bits as an uninterrupted one.
"""
from __future__ import annotations

import argparse
import copy
import json
import time

import torch

from . import mirres, synth


def _rmse(a: torch.Tensor, b: torch.Tensor, mask: torch.Tensor | None = None) -> float:
    d = (a - b).pow(2)
    if mask is not None:                                     # texels some step has seen (nonzero gradient)
        d = d[mask]                                          # (H, W) mask over (H, W) or (H, W, 3)
    return float(d.mean().sqrt()) if d.numel() else float("nan")


def run(n_views=100, res=800, spp=2, target_spp=256, steps=200, lr=1e-2, rows=500, cols=1000, tex_res=4096,
        env_hw=(512, 1024), bounces=5, ris_m=32, log_every=10, seed=5, fixed_env=False, ckpt=None, ckpt_every=0,
        resume=False, deterministic=False):
    w = synth.config5(n_views=n_views, res=res, rows=rows, cols=cols, tex_res=tex_res, env_hw=env_hw)
    for v in w.views:
        v.spp = spp
    opts = mirres.RenderOptions.from_any(w.opts)
    opts.bounces, opts.ris_m, opts.ris_m_brdf = bounces, ris_m, ris_m // 2
    opts.deterministic = int(bool(deterministic))
    gt = mirres.GpuScene.from_synth(w.scene)
    t0 = time.perf_counter()
    targets = []
    topts = copy.copy(opts)
    topts.seed = 0x9E37 + seed
    for v in w.views:                                       # per view: 800^2 x 256 spp fits one call
        tv = copy.copy(v)
        tv.spp = target_spp
        targets.append(mirres.render(gt, [tv], topts))
    target = torch.cat(targets)
    torch.cuda.synchronize()
    t_target = time.perf_counter() - t0
    albedo = torch.full_like(gt.albedo, 0.5).requires_grad_(True)
    rough = torch.full_like(gt.rough, 0.5).requires_grad_(True)
    metal = torch.full_like(gt.metal, 0.5).requires_grad_(True)
    if fixed_env:                                            # ablation: the lighting is known
        env = gt.env.clone()
    else:
        env = torch.full_like(gt.env, float(gt.env.mean())).requires_grad_(True)
    params = [albedo, rough, metal, env]
    init = [p.detach().clone() for p in params]
    optim = torch.optim.Adam([p for p in params if p.requires_grad], lr=lr)
    npix = target.shape[0]
    # Texels that received a gradient in some step: the error over them says
    # how well the observed part of each texture is recovered; texels no view
    # reaches keep their initial value and only dilute the whole-texture RMSE.
    seen = [torch.zeros(p.shape[:2], dtype=torch.bool, device=p.device) for p in params]
    names = ("albedo", "rough", "metal", "env")
    truth = (gt.albedo, gt.rough, gt.metal, gt.env)

    def errors():
        e = {k: _rmse(p.detach(), t) for k, p, t in zip(names, params, truth)}
        e.update({k + "_seen": _rmse(p.detach(), t, m) for k, p, t, m in zip(names, params, truth, seen)})
        e.update({k + "_seen_frac": float(m.float().mean()) for k, m in zip(names, seen)})
        return e

    log = [{"step": 0, **errors()}]
    start = 0
    if resume:
        st = torch.load(ckpt, map_location=albedo.device, weights_only=True)
        with torch.no_grad():
            for p, v in zip(params, st["params"]):
                p.copy_(v)
            for m, v in zip(seen, st["seen"]):
                m.copy_(v)
        optim.load_state_dict(st["optim"])
        start, log = int(st["step"]), list(st["log"])

    def save(step):
        torch.save({"params": [p.detach() for p in params], "seen": seen, "optim": optim.state_dict(),
                    "step": step, "log": log}, ckpt)

    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for it in range(start, steps):
        o = copy.copy(opts)
        o.seed = 1000 + it
        img = mirres.render_autograd(gt, w.views, o, albedo=albedo, rough=rough, metal=metal, env=env)
        loss = (img - target).pow(2).sum() / npix
        optim.zero_grad(set_to_none=False)
        loss.backward()
        with torch.no_grad():
            for m, p in zip(seen, params):
                if p.grad is None:
                    continue
                g = p.grad != 0
                m |= g.any(-1) if g.dim() == 3 else g
        optim.step()
        with torch.no_grad():                                # keep parameters in their valid ranges
            albedo.clamp_(0.0, 1.0)
            rough.clamp_(0.05, 1.0)
            metal.clamp_(0.0, 1.0)
            env.clamp_(min=0.0)
        if (it + 1) % log_every == 0 or it + 1 == steps:
            rec = {"step": it + 1, "loss": float(loss.detach()), **errors(), "s": time.perf_counter() - t1}
            log.append(rec)
            print(json.dumps(rec), flush=True)
        if ckpt and ckpt_every and ((it + 1) % ckpt_every == 0 or it + 1 == steps):
            save(it + 1)
    torch.cuda.synchronize()
    dt = max(time.perf_counter() - t1, 1e-9)
    done = steps - start
    # step 0 over the texels the run ended up seeing (the mask is empty before the first step)
    log[0].update({k + "_seen": _rmse(p, t, m) for k, p, t, m in zip(names, init, truth, seen)})
    S = sum(v.w * v.h * v.spp for v in w.views)
    return {"workload": w.name, "triangles": w.scene.nf, "views": n_views, "res": res, "spp": spp,
            "target_spp": target_spp, "bounces": bounces, "ris_m": ris_m, "steps": steps, "lr": lr,
            "env_optimised": not fixed_env,
            "steps_per_s": done / dt, "samples_per_s": done * S / dt, "target_render_s": t_target,
            "initial": log[0], "final": log[-1], "params": [p.detach() for p in params]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--views", type=int, default=100)
    ap.add_argument("--res", type=int, default=800)
    ap.add_argument("--target-spp", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--spp", type=int, default=2)
    ap.add_argument("--fixed-env", action="store_true", help="hold the environment map at the ground truth")
    ap.add_argument("--ckpt", default=None, help="checkpoint file")
    ap.add_argument("--ckpt-every", type=int, default=0, help="save the checkpoint every K steps")
    ap.add_argument("--resume", action="store_true", help="continue from --ckpt")
    ap.add_argument("--deterministic", action="store_true", help="bitwise reproducible gradients (slower)")
    ap.add_argument("--small", action="store_true", help="8 views of 256^2, 100k triangles, 1024^2 textures")
    a = ap.parse_args()
    if a.resume and not a.ckpt:
        ap.error("--resume needs --ckpt")
    kw = dict(fixed_env=a.fixed_env, ckpt=a.ckpt, ckpt_every=a.ckpt_every, resume=a.resume,
              deterministic=a.deterministic)
    if a.small:
        res = run(n_views=8, res=256, spp=a.spp, target_spp=64, steps=a.steps, lr=a.lr, rows=158, cols=316,
                  tex_res=1024, env_hw=(128, 256), **kw)
    else:
        res = run(n_views=a.views, res=a.res, spp=a.spp, target_spp=a.target_spp, steps=a.steps, lr=a.lr, **kw)
    res.pop("params")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
