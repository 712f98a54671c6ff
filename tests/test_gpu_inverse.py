"""The inverse-rendering loop (Adam over textures and env through the
autograd Function) reduces the material and lighting error on a small
instance of the config-5 workload."""
import pytest

pytestmark = pytest.mark.gpu


def test_inverse_loop_reduces_error():
    from paper_2406_16360_amd import inverse
    res = inverse.run(n_views=6, res=64, spp=2, target_spp=32, steps=40, lr=3e-2, rows=40, cols=80, tex_res=32,
                      env_hw=(16, 32), bounces=3, ris_m=8, log_every=20)
    a, b = res["initial"], res["final"]
    assert b["albedo"] < a["albedo"] and b["env"] < a["env"], (a, b)
    assert res["steps_per_s"] > 0


def test_checkpoint_resume_matches_uninterrupted(tmp_path):
    """With deterministic gradients, 4 steps in one go and 2 + 2 steps
    through a checkpoint end with the same bits in every parameter."""
    import torch
    from paper_2406_16360_amd import inverse
    kw = dict(n_views=2, res=32, spp=2, target_spp=8, lr=3e-2, rows=20, cols=40, tex_res=16, env_hw=(8, 16),
              bounces=2, ris_m=4, log_every=2, deterministic=True)
    ck = str(tmp_path / "ck.pt")
    a = inverse.run(steps=4, **kw)
    inverse.run(steps=2, ckpt=ck, ckpt_every=2, **kw)
    c = inverse.run(steps=4, ckpt=ck, resume=True, **kw)
    for x, y in zip(a["params"], c["params"]):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))
    assert c["final"]["step"] == 4 and a["final"]["loss"] == c["final"]["loss"]
