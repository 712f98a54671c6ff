#!/usr/bin/env python3
"""Throughput of the differentiable RIS path tracer on one MI355X.

One step = one optimisation step of the texture/env inverse problem on the
differentiation workload: render 8 views of 800x800 at 4 spp over a ~300k
triangle displaced mesh with 2048^2 fp32 textures and a 512x256 HDR env
(3 bounces, RIS M = 32), L2 loss against a target rendered from seeded
ground-truth materials, then the adjoint replay that scatters dL/dtexel and
dL/denv-texel.  value = path samples per second of that fwd+bwd step.

--workload reuse runs the same step as a sequence of frames with spatial and
temporal reservoir reuse at the primary vertices (5 neighbours in a 61 x 61
pixel window, history capped at 20 M); each step's reservoirs feed the next.

--workload field runs the same step with the materials from the paper's
neural material field F_m (16-level hash grid, 2^19 slots per level,
resolutions 16..2048, 2-layer MLP with 32 hidden units) instead of textures,
differentiating the field's table and weights.

--workload c5 is the inverse-rendering workload's step (100 views of 800x800,
2 spp, 5 bounces, 1M triangles, 4096^2 textures); c2 the single-view plain
forward workload (run it with --mode fwd); c1 the tiny workload as graph
replays of plans; c4 the 64 uneven views as one persistent graph-replayed
plan (fwd+bwd, beside the batched forward and 64 separate launches).
--mode fwd times the forward alone; --tape off makes the adjoint re-render
instead of reading the per-vertex tape.

Also reported (one JSON line):
  roofline      the dominant kernel's algorithmic bytes per second (counts
                from the FP64 oracle's own SAH BVH on a seeded subset of the
                same samples, bytes per unit as in kernel_bytes below) over
                its HIP-event-timed duration, against the 8 TB/s HBM3E peak;
                per kernel, the counter-measured HBM rate beside it when the
                committed FETCH_SIZE/WRITE_SIZE traffic matches the sources;
  cpu_baseline  the FP64 oracle, as it stands, on a bounded seeded subset of
                the same samples, on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd path samples/s at 800x800, 3 bounces, RIS M=32; % of HBM roofline"
HBM_PEAK_GBPS = 8000.0

# algorithmic bytes per unit (gather model): BVH node 32 B, triangle 36 B,
# hit re-read 36 B (indices + uv), material fetch 80 B (bilinear: 4 texels x
# 20 B) or 60 B (per-vertex), RIS candidate 20 B (env radiance 12 + pdf
# entries 8), pixel 12 B, adjoint gradient RMW 3x the material fetch, env
# gradient RMW 24 B, vertex record 32 B written + read.
NODE_B, TRI_B, HIT_B, CAND_B, PIX_B, ENVG_B, VREC_B = 32, 36, 36, 20, 12, 24, 64
# material field, per point: hit or tape record 16 B, triangle 36 B, 16
# levels x 8 corners x 8 B of table entries, output 16 B; the pull-back adds
# the read-modify-write of the same 128 entries; the output kept on the tape
# for the backward is 16 B more per hit
FIELD_B = 16 + 36 + 128 * 8 + 16
FIELD_BWD_B = FIELD_B + 2 * 128 * 8
FIELD_TAPE_B = 16


def kernel_bytes(cnt, n, spp, tex, field=False, reuse_k=0, ris_m=32):
    """Per-sample algorithmic bytes attributed to each kernel class."""
    tmat = 16 if field else (80 if tex else 60)
    per = {k: v / n for k, v in cnt.items()}
    primary = 1.0 - per["primary_miss"]
    kb = {
        "trace_closest": NODE_B * per["closest_nodes"] + TRI_B * per["closest_tris"],
        "trace_shadow": NODE_B * per["shadow_nodes"] + TRI_B * per["shadow_tris"],
        "shade": per["hits"] * (HIT_B + tmat) + per["candidates"] * CAND_B,
        "resolve": PIX_B / spp,
        "adjoint": PIX_B / spp + per["hits"] * (HIT_B + (2 if field else 3) * tmat) + per["nee_visible"] * ENVG_B
                   + per["hits"] * VREC_B,
    }
    if field:
        kb["field_eval"] = per["hits"] * FIELD_B              # the forward pass (the tape keeps its output)
        kb["shade"] += per["hits"] * FIELD_TAPE_B            # that output written to the tape
        kb["field_backward"] = per["hits"] * FIELD_BWD_B
    if reuse_k:
        # one more camera ray per sample, the initial RIS at its primary vertex,
        # and the merges: (2 + k) 32-byte records read, 3 written, the
        # primary hit and material re-read per pass
        ray = kb["trace_closest"] / max(per["closest_rays"], 1e-9)
        kb["reuse"] = (ray + 16 + primary * (3 * (HIT_B + tmat) + ris_m * CAND_B + (2 + reuse_k) * 32 + 3 * 32))
    return kb


# sources the default step's kernels are compiled from (the BVH builder
# included: its tree sets the traversal traffic); reuse.h, denoise.hip and
# field.hip hold kernels the default step never launches
DIGEST_EXCLUDE = {"reuse.h", "denoise.hip", "field.hip", "roofs.hip"}


def source_digest():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2406_16360_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")) and f not in DIGEST_EXCLUDE:
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None if the kernel sources changed since it was taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


def make_workload(name):
    from paper_2406_16360_amd import synth
    if name == "c3":
        return synth.config3()
    if name == "reuse":
        w = synth.config3()
        w.opts.reuse_spatial, w.opts.reuse_radius, w.opts.reuse_temporal, w.opts.reuse_m_cap = 5, 30, 1, 20
        w.name = "c3_reuse_" + w.name[3:]
        return w
    if name == "field":
        w = synth.config3()
        w.scene = synth.with_field(w.scene, np.random.default_rng(3003))
        w.name = "c3_field_" + w.name[3:]
        return w
    if name == "c2":
        return synth.config2()
    if name == "c1":
        return synth.config1()
    if name == "c5":
        return synth.config5()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, seconds, nthreads):
    """The FP64 oracle on a bounded seeded subset of the same samples (render
    + gradient), plus its traversal counters for the roofline model and the
    number of samples they cover."""
    from oracle.oracle import Oracle
    from paper_2406_16360_amd import synth
    orc = Oracle(w.scene)
    probe = synth.sample_items(w, 40000, 12345)   # large enough to amortise thread start-up
    t0 = time.perf_counter()
    orc.render(w.views, w.opts, probe, nthreads=nthreads)
    orc.grad(w.views, w.opts, probe, np.ones((len(probe), 3)), nthreads=nthreads)
    per = (time.perf_counter() - t0) / len(probe)
    n = int(min(max(seconds / max(per, 1e-9), 4000), 16_000_000))
    items = synth.sample_items(w, n, 2024)
    n = len(items)                                  # a small workload has fewer samples than the budget
    dl = np.random.default_rng(7).random((n, 3))
    t0 = time.perf_counter()
    _, _, cnt = orc.render(w.views, w.opts, items, nthreads=nthreads, counters=True)
    orc.grad(w.views, w.opts, items, dl, nthreads=nthreads)
    dt = time.perf_counter() - t0
    # one thread on a share of the same samples, for the per-core rate
    n1 = max(n // max(nthreads, 1), 1000)
    t0 = time.perf_counter()
    orc.render(w.views, w.opts, items[:n1], nthreads=1)
    orc.grad(w.views, w.opts, items[:n1], dl[:n1], nthreads=1)
    cpu_baseline.one_thread = n1 / (time.perf_counter() - t0)
    if getattr(w.opts, "reuse_spatial", 0) or getattr(w.opts, "reuse_temporal", 0):
        # the per-kernel byte model takes the path's own traversal counts: the
        # oracle's reuse re-traces each neighbour's camera ray per sample
        import copy
        plain = copy.deepcopy(w.opts)
        plain.reuse_spatial, plain.reuse_temporal = 0, 0
        _, _, cnt = orc.render(w.views, plain, probe, nthreads=nthreads, counters=True)
        return n / dt, n, dt, cnt, len(probe)
    return n / dt, n, dt, cnt, n


def roofline_from(prof, kb, S, steps, workload):
    """Dominant kernel's algorithmic GB/s from HIP-event kernel times, and per
    kernel the algorithmic rate beside the counter-measured HBM rate (the
    committed FETCH_SIZE/WRITE_SIZE traffic per launch over the same launch
    time) when the counters match the current sources."""
    kern = {}
    for name, (launches, ms) in prof.items():
        if name in kb:
            per_step_ms = ms / steps
            k = {"ms_per_step": per_step_ms, "launches_per_step": launches / steps,
                 "alg_bytes_per_sample": kb[name],
                 "alg_GBps": S * kb[name] / (per_step_ms * 1e-3) / 1e9}
            traffic = load_traffic(name, workload)
            if traffic is not None and launches:
                hbm = traffic / (per_step_ms * steps / launches * 1e-3) / 1e9
                k.update(hbm_counter_GBps=hbm, hbm_counter_frac=hbm / HBM_PEAK_GBPS)
            kern[name] = k
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    d = kern[dom]
    launches = d["launches_per_step"]
    roof = {"bound": "hbm", "kernel": dom, "achieved": d["alg_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": d["alg_GBps"] / HBM_PEAK_GBPS, "traffic": load_traffic(dom, workload),
            "alg_bytes_per_launch": S * kb[dom] / launches, "avg_launch_ms": d["ms_per_step"] / launches}
    if "hbm_counter_frac" in d:
        roof["hbm_counter_frac"] = d["hbm_counter_frac"]
    return roof, kern


def _timed(args, fn):
    """Seconds per call of fn over args.steps calls after args.warmup."""
    import torch
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / args.steps


def _gt_target_scene(mirres, synth, sc, dev):
    """Ground-truth materials the L2 target is rendered from: a second seeded
    texture set, or the vertex materials in reverse order."""
    import torch
    rng = np.random.default_rng(9000)
    if sc.mat_mode == mirres.MAT_TEXTURE:
        ga, gr_, gm = synth.noise_textures(sc.rough.shape[0], rng)
        return sc.with_params(albedo=torch.tensor(ga, device=dev), rough=torch.tensor(gr_, device=dev),
                              metal=torch.tensor(gm, device=dev))
    return sc.with_params(vmat=sc.vmat.flip(0).contiguous())


def _plan_step(plan, target):
    """One optimisation step on a graph-replayed plan: forward, dL/dI of the
    L2 loss into the bound grad image, zeroed gradients, backward."""
    import torch
    img = plan.forward()
    torch.sub(img, target, out=plan.grad_image)
    plan.grad_image.mul_(2.0)
    plan.zero_grad()
    plan.backward()


def bench_batched(args):
    """Config 4: 64 views of uneven size (256^2..1024^2) and spp (1..16) over the
    300k-triangle mesh as one persistent pool captured in hipGraphs, with
    autotuned pool/workgroup sizes.  value = fwd+bwd samples/s of the batched
    plan (forward, L2 gradient, adjoint); beside it the batched forward alone
    and 64 separate forward launches (one eager mrs_render per view)."""
    import torch
    from paper_2406_16360_amd import autotune, mirres, synth
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = synth.config4()
    S = w.samples
    print(f"# workload {w.name}: {S} samples/pass, {w.scene.nf} triangles", file=sys.stderr, flush=True)
    sc = mirres.GpuScene.from_synth(w.scene)
    opts = mirres.RenderOptions.from_any(w.opts)
    tune = autotune.autotune(sc, w.views, opts, reps=2, verbose=True, cache=None)
    opts.pool, opts.block = tune["pool"], tune["block"]
    target = mirres.render(_gt_target_scene(mirres, synth, sc, dev), w.views, opts).clone()
    plan = mirres.Plan(sc, w.views, opts, use_graph=True)
    t_batched = _timed(args, plan.forward)
    del plan
    # the fwd+bwd plan gets sizes tuned for the forward and backward together
    gtune = autotune.autotune(sc, w.views, opts, reps=2, verbose=True, cache=None, with_grad=True)
    gopts = mirres.RenderOptions(**{**opts.__dict__, "pool": gtune["pool"], "block": gtune["block"]})
    gplan = mirres.Plan(sc, w.views, gopts, with_grad=True, use_graph=True)
    t_fwdbwd = _timed(args, lambda: _plan_step(gplan, target))
    keeps_tape = gplan.info()[1]
    del gplan
    plain_opts = mirres.RenderOptions.from_any(w.opts)
    t_plain = _timed(args, lambda: [mirres.render(sc, [v], plain_opts) for v in w.views])
    # per-kernel times from eager fwd+bwd steps with the tuned sizes
    mirres.profile_begin()
    for _ in range(2):
        img, tape = mirres.render(sc, w.views, gopts, keep_tape=True)
        mirres.render_backward(sc, w.views, gopts, 2.0 * (img - target), tape=tape)
    torch.cuda.synchronize()
    prof = mirres.profile_end()
    cpu, roof, extra = None, None, {}
    if not args.no_cpu_baseline:
        ncores = len(os.sched_getaffinity(0))
        v, nsub, dt, cnt, ncnt = cpu_baseline(w, args.cpu_seconds, ncores)
        cpu = {"value": v, "unit": "samples/s", "cores": ncores, "kind": "oracle",
               "sample": f"{nsub} seeded samples of {w.name} (render + gradient) in {dt:.1f}s",
               "value_1_thread": cpu_baseline.one_thread}
        kb = kernel_bytes(cnt, ncnt, S / sum(v.w * v.h for v in w.views), True)
        roof, kern = roofline_from(prof, kb, S, 2, "c4")
        extra = {"path_alg_bytes_per_sample": sum(kb.values()), "kernels": kern}
    out = {"metric": "fwd+bwd path samples/s, 64 uneven views in one persistent graph-replayed plan",
           "value": S / t_fwdbwd, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t_fwdbwd * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "views": len(w.views), "samples_per_step": S, "bounces": w.opts.bounces,
                      "ris_m": w.opts.ris_m, "triangles": w.scene.nf, "pool": gopts.pool, "block": gopts.block,
                      "tape": keeps_tape, "forward_pool": opts.pool, "forward_block": opts.block},
           "forward_batched": {"value": S / t_batched, "ms_per_step": t_batched * 1e3},
           "forward_64_plain_launches": {"value": S / t_plain, "ms_per_step": t_plain * 1e3},
           "batched_forward_speedup": t_plain / t_batched, "autotune": tune["table"],
           "autotune_fwdbwd": gtune["table"],
           "roofline": roof, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_graph_small(args):
    """Config 1 (16,384 samples per step) cannot fill 256 CUs in one launch, so
    its fwd+bwd step runs as graph replays of plans with distinct seeds (8
    plans in rotation): value = samples/s over args.steps replays.  The
    per-kernel roofline comes from eager steps (graph replays are not timed
    per kernel)."""
    import copy
    import torch
    from paper_2406_16360_amd import mirres, synth
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = synth.config1()
    S = w.samples
    print(f"# workload {w.name}: {S} samples/step, {w.scene.nf} triangles", file=sys.stderr, flush=True)
    sc = mirres.GpuScene.from_synth(w.scene)
    opts = mirres.RenderOptions.from_any(w.opts)
    target = mirres.render(_gt_target_scene(mirres, synth, sc, dev), w.views, opts).clone()
    plans = []
    for j in range(8):
        o = copy.copy(opts)
        o.seed = w.opts.seed + 7919 * j
        plans.append(mirres.Plan(sc, w.views, o, with_grad=True, use_graph=True))
    turn = [0]

    def step():
        _plan_step(plans[turn[0] % len(plans)], target)
        turn[0] += 1

    t_step = _timed(args, step)
    mirres.profile_begin()
    steps_prof = 20
    for _ in range(steps_prof):
        img, tape = mirres.render(sc, w.views, opts, keep_tape=True)
        mirres.render_backward(sc, w.views, opts, 2.0 * (img - target), tape=tape)
    torch.cuda.synchronize()
    prof = mirres.profile_end()
    cpu, roof, extra = None, None, {}
    if not args.no_cpu_baseline:
        ncores = len(os.sched_getaffinity(0))
        v, nsub, dt, cnt, ncnt = cpu_baseline(w, args.cpu_seconds, ncores)
        cpu = {"value": v, "unit": "samples/s", "cores": ncores, "kind": "oracle",
               "sample": f"{nsub} seeded samples of {w.name} (render + gradient) in {dt:.1f}s",
               "value_1_thread": cpu_baseline.one_thread}
        kb = kernel_bytes(cnt, ncnt, w.views[0].spp, False)
        roof, kern = roofline_from(prof, kb, S, steps_prof, "c1")
        extra = {"path_alg_bytes_per_sample": sum(kb.values()), "kernels": kern}
    out = {"metric": "fwd+bwd path samples/s, config 1 as graph replays", "value": S / t_step,
           "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "samples_per_step": S, "bounces": w.opts.bounces, "ris_m": w.opts.ris_m,
                      "triangles": w.scene.nf, "plans_in_rotation": len(plans)},
           "roofline": roof, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_bvh(args):
    """Per-iteration acceleration-structure update: full builds (LBVH, PLOC)
    and a refit after the vertices move, over the 300k- and 1M-triangle meshes
    of configs 3 and 5 (median of `steps` timed runs after `warmup`)."""
    import torch
    from paper_2406_16360_amd import mirres, synth
    torch.cuda.set_device(0)
    out = {}
    for name, w in (("c3_300k_tris", synth.config3()), ("c5_1m_tris", synth.config5())):
        pos = torch.tensor(w.scene.pos, device="cuda")
        faces = torch.tensor(w.scene.faces, device="cuda")
        moved = pos + 0.01 * torch.randn(pos.shape, device="cuda", generator=torch.Generator("cuda").manual_seed(1))

        def timed(fn):
            for _ in range(args.warmup):
                fn()
            ts = []
            for _ in range(args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            return float(np.median(ts))

        rec = {"triangles": int(faces.shape[0])}
        for bname, b in (("lbvh", mirres.BVH_LBVH), ("ploc", mirres.BVH_PLOC)):
            rec[f"build_{bname}_ms"] = timed(lambda: mirres.build_bvh(pos, faces, builder=b))
            bvh = mirres.build_bvh(pos, faces, builder=b)
            rec[f"refit_{bname}_ms"] = timed(lambda: bvh.refit(moved))
            rec[f"depth_{bname}"] = bvh.info()[2]
        out[name] = rec
        print(f"# {name}: {rec}", file=sys.stderr, flush=True)
    c5 = out["c5_1m_tris"]
    line = {"metric": "BVH refit ms (1M triangles), per optimisation iteration", "value": c5["refit_ploc_ms"],
            "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": c5["refit_ploc_ms"],
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "bvh_build_refit", **{k: v for k, v in out.items()}}}
    print(json.dumps(line), flush=True)


def bench_denoise(args):
    """The denoiser row at the differentiation workload's image size (8 views
    of 800x800): G-buffer, three a-trous levels forward and their adjoint.
    value = pixels per second of one forward + adjoint; roofline against the
    algorithmic bytes (per pixel and level: forward reads colour, normal and
    position and writes colour and weight sum, 52 B; the adjoint reads those
    plus dL/dout and the weight sum and writes dL/dc, 76 B)."""
    import torch
    from paper_2406_16360_amd import mirres, synth
    torch.cuda.set_device(0)
    w = synth.config3()
    sc = mirres.GpuScene.from_synth(w.scene)
    pos, nrm = mirres.gbuffer(sc, w.views)
    img = mirres.render(sc, w.views, mirres.RenderOptions.from_any(w.opts))
    den = mirres.Denoiser(w.views, nrm, pos, levels=3)
    g = torch.randn_like(img)
    npix = img.shape[0]

    def step():
        den.forward(img)
        den.backward(g)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        den.forward(img)
    ev[1].record()
    for _ in range(args.steps):
        den.backward(g)
    ev[2].record()
    torch.cuda.synchronize()
    f_ms = ev[0].elapsed_time(ev[1]) / args.steps
    b_ms = ev[1].elapsed_time(ev[2]) / args.steps
    ms = f_ms + b_ms
    L = 3
    f_gbps = npix * L * 52 / (f_ms * 1e-3) / 1e9
    b_gbps = npix * L * 76 / (b_ms * 1e-3) / 1e9
    dom = ("adjoint", b_gbps, b_ms, 76) if b_ms >= f_ms else ("forward", f_gbps, f_ms, 52)
    line = {"metric": "denoiser fwd+adjoint pixels/s, 3 a-trous levels, 8 x 800x800", "value": npix / (ms * 1e-3),
            "unit": "pixels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "denoise_8x800x800_3levels", "pixels": npix, "forward_ms": f_ms, "adjoint_ms": b_ms},
            "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": dom[1], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": dom[1] / HBM_PEAK_GBPS, "traffic": None,
                         "alg_bytes_per_launch": npix * dom[3], "avg_launch_ms": dom[2] / (L * len(w.views))},
            "forward_roofline_frac": f_gbps / HBM_PEAK_GBPS, "adjoint_roofline_frac": b_gbps / HBM_PEAK_GBPS}
    if not args.no_cpu_baseline:
        from oracle import denoise as odn
        v0 = w.views[0]
        rng = np.random.default_rng(9)   # seeded buffers of one view's shape
        c, n, x, gg = (rng.random((v0.w * v0.h, 3)) for _ in range(4))
        t0 = time.perf_counter()
        odn.denoise(c, n, x, [v0])
        odn.denoise_grad(c, n, x, gg, [v0])
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": v0.w * v0.h / dt, "unit": "pixels/s", "cores": torch.get_num_threads(),
                                "kind": "oracle", "sample": f"one 800x800 view, forward + autograd adjoint, {dt:.1f}s"}
    print(json.dumps(line), flush=True)


def bench_roofs(args):
    """Measured memory ceilings: streaming HBM read and copy over 4 GiB, and
    independent random gathers of 16- and 64-byte records from tables of
    4 MiB (L2), 32 MiB (the config-3 BVH and triangles), 192 MiB (memory-side
    cache) and 4 GiB (HBM)."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2406_16360_amd", "libmrsroofs.so"))
    lib.mrs_roofs_stream.restype = C.c_int
    lib.mrs_roofs_stream.argtypes = [C.c_uint64, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.mrs_roofs_gather.restype = C.c_int
    lib.mrs_roofs_gather.argtypes = [C.c_uint64, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    rd, cp = C.c_double(), C.c_double()
    if lib.mrs_roofs_stream(4 << 30, 5, C.byref(rd), C.byref(cp)) != 0:
        raise SystemExit("stream measurement failed")
    gather = {}
    for tb, label in ((4 << 20, "4MiB"), (32 << 20, "32MiB"), (192 << 20, "192MiB"), (4 << 30, "4GiB")):
        for rb in (16, 64):
            g, r = C.c_double(), C.c_double()
            if lib.mrs_roofs_gather(tb, rb, 3, C.byref(g), C.byref(r)) != 0:
                raise SystemExit("gather measurement failed")
            gather[f"{label}_{rb}B"] = {"GBps": g.value, "Grecords_per_s": r.value}
            print(f"# gather {label} {rb} B records: {g.value:.0f} GB/s, {r.value:.1f} G records/s",
                  file=sys.stderr, flush=True)
    line = {"metric": "measured memory ceilings", "value": rd.value, "unit": "GB/s", "n_gpus": 1,
            "steps": 5, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "roofs"}, "hbm_read_GBps": rd.value, "hbm_copy_GBps": cp.value,
            "hbm_peak_GBps": HBM_PEAK_GBPS, "random_gather": gather}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3",
                    choices=["c1", "c2", "c3", "c4", "c5", "bvh", "denoise", "field", "reuse", "roofs"])
    ap.add_argument("--mode", default="fwdbwd", choices=["fwdbwd", "fwd"])
    ap.add_argument("--tape", default="on", choices=["auto", "on", "off"])
    ap.add_argument("--pool", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: there is no multi-GPU path here (each GPU would render its own "
              "share of the views). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        bench_batched(args)
        return
    if args.workload == "c1":
        bench_graph_small(args)
        return
    if args.workload == "roofs":
        bench_roofs(args)
        return
    if args.workload == "bvh":
        bench_bvh(args)
        return
    if args.workload == "denoise":
        bench_denoise(args)
        return

    import torch
    from paper_2406_16360_amd import mirres, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = make_workload(args.workload)
    print(f"# workload {w.name}: {w.samples} samples/step, {w.scene.nf} triangles", file=sys.stderr, flush=True)
    sc = mirres.GpuScene.from_synth(w.scene)
    opts = mirres.RenderOptions.from_any(w.opts)
    opts.tape_mode = {"auto": mirres.TAPE_AUTO, "on": mirres.TAPE_ON, "off": mirres.TAPE_OFF}[args.tape]
    opts.pool, opts.block = args.pool, args.block
    tex = sc.mat_mode == mirres.MAT_TEXTURE
    field = sc.mat_mode == mirres.MAT_FIELD

    # target rendered from seeded ground-truth materials (a second texture set or field)
    if field:
        f2 = synth.with_field(w.scene, np.random.default_rng(9000)).field
        gt = mirres.GpuScene(sc.pos, sc.faces, sc.env, bvh=sc.bvh, field=mirres.Field.from_synth(f2))
    else:
        gt = _gt_target_scene(mirres, synth, sc, dev)
    reuse = opts.reuse_spatial > 0 or opts.reuse_temporal
    res = [torch.zeros((w.samples, 8), device=dev), torch.zeros((w.samples, 8), device=dev)] if reuse else None
    frame = [0]
    target = mirres.render(gt, w.views, opts).clone() if not reuse else \
        mirres.render(gt, w.views, opts, reservoir_out=res[1]).clone()
    grads = sc.zero_grads()

    def step():
        kw = {}
        if reuse:   # this frame's reservoirs become the next frame's history; a new seed per frame
            frame[0] += 1
            opts.seed = w.opts.seed + frame[0]
            kw = dict(reservoir_prev=res[frame[0] % 2 ^ 1], reservoir_out=res[frame[0] % 2])
        if args.mode == "fwd":
            mirres.render(sc, w.views, opts, **kw)
            return
        img, tape = mirres.render(sc, w.views, opts, keep_tape=True, **kw)
        dimg = 2.0 * (img - target)                    # d/dI of the L2 loss sum (I - I_ref)^2
        for g in grads.values():
            g.zero_()
        mirres.render_backward(sc, w.views, opts, dimg, tape=tape, grads=grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mirres.profile_begin()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = mirres.profile_end()
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = wall * 1e3 / args.steps
    S = w.samples
    value = S * args.steps / wall
    print(f"# wall {wall:.3f}s events {gpu_ms:.1f}ms kernels {json.dumps(prof)}", file=sys.stderr, flush=True)

    # CPU baseline (oracle) and the roofline model from its counters
    cpu = None
    cnt = None
    nsub = 0
    if not args.no_cpu_baseline:
        ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        v, nsub, dt, cnt, ncnt = cpu_baseline(w, args.cpu_seconds, ncores)
        cpu = {"value": v, "unit": "samples/s", "cores": ncores, "kind": "oracle",
               "sample": f"{nsub} seeded samples of {w.name} (render + gradient) in {dt:.1f}s",
               "value_1_thread": cpu_baseline.one_thread}
        if args.mode == "fwd":
            cpu["sample"] += "; value counts render + gradient per sample"
    roof = None
    extra = {}
    if cnt is not None:
        kb = kernel_bytes(cnt, ncnt, w.views[0].spp, tex, field, w.opts.reuse_spatial if reuse else 0, w.opts.ris_m)
        if args.mode == "fwd":
            kb.pop("adjoint")
            kb.pop("field_backward", None)
        balg = sum(kb.values())
        roof, kern = roofline_from(prof, kb, S, args.steps, args.workload)
        # the whole path's algorithmic bytes per second: a gather rate (much
        # of it served from L2 and the memory-side cache), not an HBM fraction
        extra = {"path_alg": {"alg_bytes_per_sample": balg, "alg_GBps": value * balg / 1e9,
                              "counts_per_sample": {k: v / ncnt for k, v in cnt.items()}},
                 "kernels": kern}
    out = {"metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "views": len(w.views), "width": w.views[0].w, "height": w.views[0].h,
                      "spp": w.views[0].spp, "samples_per_step": S, "bounces": w.opts.bounces,
                      "ris_m": w.opts.ris_m, "ris_m_brdf": w.opts.ris_m_brdf, "triangles": w.scene.nf,
                      "mode": args.mode, "tape": args.tape, "pool": args.pool, "block": args.block},
           "roofline": roof, "cpu_baseline": cpu, "gpu_event_ms": gpu_ms}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
