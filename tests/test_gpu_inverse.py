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
