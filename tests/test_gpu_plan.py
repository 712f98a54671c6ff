"""Plans: persistent batched launch captured in a hipGraph, replayed.

Every graph replay is checked against the eager result of the same call,
with eager torch work and synchronisations between replays."""
import copy

import numpy as np
import pytest
import torch

from paper_2406_16360_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr():
    from paper_2406_16360_amd import mirres
    return mirres


def _uneven_views(n=6, seed=5, lo=16, hi=72):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        s = int(rng.integers(lo, hi + 1))
        out.append(synth.View(c2w=synth.orbit(3.0, rng.uniform(5, 60), rng.uniform(0, 6.28)), fov_y_deg=40.0,
                              w=s, h=s, spp=int(rng.integers(1, 5))))
    return out


def _scene():
    rng = np.random.default_rng(77)
    return synth._displaced_scene(40, 80, 64, (16, 32), rng)


def test_graph_forward_replays_match_eager(mr):
    sc = mr.GpuScene.from_synth(_scene())
    views = _uneven_views()
    opts = mr.RenderOptions(bounces=3, ris_m=8, ris_m_brdf=4, rr_start=2, seed=21, pool=3000)
    ref = mr.render(sc, views, opts)
    plan = mr.Plan(sc, views, opts, use_graph=True)
    assert plan.info()[2]
    for rep in range(4):
        img = plan.forward().clone()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(img, ref), rep
        del junk


def test_graph_sees_in_place_parameter_updates(mr):
    sc = mr.GpuScene.from_synth(_scene())
    views = _uneven_views(3)
    opts = mr.RenderOptions(bounces=2, ris_m=8, ris_m_brdf=4, seed=3)
    plan = mr.Plan(sc, views, opts, use_graph=True)
    a = plan.forward().clone()
    sc.albedo.mul_(0.5)                 # in place: the graph reads the new values
    sc.env.mul_(2.0)
    b = plan.forward().clone()
    ref = mr.render(sc, views, opts)
    assert torch.equal(b, ref) and not torch.equal(a, b)


@pytest.mark.parametrize("tape_mode", [0, 2])
def test_graph_backward_matches_eager(mr, tape_mode):
    sc = mr.GpuScene.from_synth(_scene())
    views = _uneven_views(4, seed=9)
    opts = mr.RenderOptions(bounces=3, ris_m=8, ris_m_brdf=4, seed=8, tape_mode=tape_mode)
    plan = mr.Plan(sc, views, opts, with_grad=True, use_graph=True)
    assert plan.info()[1] == (tape_mode == 0)
    img = plan.forward()
    gi = torch.rand_like(img)
    plan.grad_image.copy_(gi)
    for rep in range(3):
        plan.zero_grad()
        plan.forward()
        g = {k: v.clone() for k, v in plan.backward().items()}
        torch.cuda.synchronize()
        ref_img, tape = mr.render(sc, views, opts, keep_tape=True)
        ref = mr.render_backward(sc, views, opts, gi, tape=tape)
        assert torch.equal(plan.image, ref_img)
        for k in ref:
            rms = ref[k].pow(2).mean().sqrt().item()
            assert (g[k] - ref[k]).abs().max().item() <= 1e-4 * rms, (rep, k)


def test_eager_plan_without_graph(mr):
    sc = mr.GpuScene.from_synth(_scene())
    views = _uneven_views(2, seed=1)
    opts = mr.RenderOptions(bounces=2, ris_m=4, ris_m_brdf=2, seed=4)
    plan = mr.Plan(sc, views, opts, use_graph=False)
    assert torch.equal(plan.forward(), mr.render(sc, views, opts))


def test_plan_debug_outputs_and_errors(mr):
    sc = mr.GpuScene.from_synth(_scene())
    views = _uneven_views(2, seed=2)
    opts = mr.RenderOptions(bounces=2, ris_m=4, ris_m_brdf=2, seed=4)
    plan = mr.Plan(sc, views, opts, use_graph=True, debug=True)
    plan.forward()
    img, rgb, h = mr.render(sc, views, opts, debug=True)
    assert torch.equal(plan.dbg_rgb, rgb) and torch.equal(plan.dbg_hash, h)
    with pytest.raises(mr.MirresError):
        plan.backward()                  # created without gradient buffers


def test_autotune_small(mr, tmp_path):
    from paper_2406_16360_amd import autotune
    sc = mr.GpuScene.from_synth(_scene())
    views = _uneven_views(3, seed=3)
    opts = mr.RenderOptions(bounces=2, ris_m=4, ris_m_brdf=2, seed=4)
    cache = str(tmp_path / "tune.json")
    res = autotune.autotune(sc, views, opts, pools=(1 << 12, 1 << 14), blocks=(64, 256), reps=2, cache=cache)
    assert res["pool"] in (1 << 12, 1 << 14) and res["block"] in (64, 256) and len(res["table"]) >= 2
    again = autotune.autotune(sc, views, opts, pools=(1 << 16,), blocks=(128,), cache=cache)
    assert again["pool"] == res["pool"]              # served from the cache
    tuned = copy.copy(opts)
    tuned.pool, tuned.block = res["pool"], res["block"]
    assert torch.equal(mr.render(sc, views, tuned), mr.render(sc, views, opts))
    # forward + backward plans are tuned under their own key
    g = autotune.autotune(sc, views, opts, pools=(1 << 12, 1 << 14), blocks=(64,), reps=2, cache=cache,
                          with_grad=True)
    assert g["pool"] in (1 << 12, 1 << 14) and len(g["table"]) == 2
