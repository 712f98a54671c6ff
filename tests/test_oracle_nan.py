"""Pins of the oracle's reading for inputs that are not numbers (the paper
is silent): a material value that is NaN after interpolation takes the lower
end of its clamp range and passes no derivative; a NaN env channel is
radiance 0 with no derivative, like a negative one."""
import copy

import numpy as np

from paper_2406_16360_amd import synth


def _small_c1():
    w = synth.config1()
    w.views[0].w, w.views[0].h = 24, 20
    return w


def _render(oracle_lib, scene, w, items):
    return oracle_lib.Oracle(scene).render(w.views, w.opts, items)


def test_nan_roughness_renders_at_the_lower_bound(oracle_lib):
    w = _small_c1()
    items = synth.all_items(w)
    a = copy.deepcopy(w.scene)
    a.vmat[:, 3] = np.nan
    b = copy.deepcopy(w.scene)
    b.vmat[:, 3] = 0.0          # below the range: clamps to its lower end, 0.05
    ra, ha = _render(oracle_lib, a, w, items)
    rb, hb = _render(oracle_lib, b, w, items)
    assert np.array_equal(ra, rb) and np.array_equal(ha, hb)
    g = oracle_lib.Oracle(a).grad(w.views, w.opts, items, np.ones((len(items), 3)))
    assert np.all(g["vmat"][:, 3] == 0.0)
    assert np.all(np.isfinite(g["vmat"])) and np.all(np.isfinite(g["env"]))
    assert np.abs(g["vmat"][:, :3]).sum() > 0


def test_nan_albedo_channel_renders_as_zero(oracle_lib):
    w = _small_c1()
    items = synth.all_items(w)
    a = copy.deepcopy(w.scene)
    a.vmat[:, 1] = np.nan
    b = copy.deepcopy(w.scene)
    b.vmat[:, 1] = 0.0
    ra, ha = _render(oracle_lib, a, w, items)
    rb, hb = _render(oracle_lib, b, w, items)
    assert np.array_equal(ra, rb) and np.array_equal(ha, hb)
    g = oracle_lib.Oracle(a).grad(w.views, w.opts, items, np.ones((len(items), 3)))
    assert np.all(g["vmat"][:, 1] == 0.0) and np.all(np.isfinite(g["vmat"]))


def test_nan_env_channel_is_zero_radiance(oracle_lib):
    w = _small_c1()
    items = synth.all_items(w)
    rng = np.random.default_rng(7)
    mask = rng.random(w.scene.env.shape) < 0.15
    a = copy.deepcopy(w.scene)
    a.env[mask] = np.nan
    b = copy.deepcopy(w.scene)
    b.env[mask] = 0.0
    ra, ha = _render(oracle_lib, a, w, items)
    rb, hb = _render(oracle_lib, b, w, items)
    assert np.array_equal(ra, rb) and np.array_equal(ha, hb)
    dl = np.ones((len(items), 3))
    ga = oracle_lib.Oracle(a).grad(w.views, w.opts, items, dl)
    gb = oracle_lib.Oracle(b).grad(w.views, w.opts, items, dl)
    assert np.all(ga["env"][mask] == 0.0) and np.all(np.isfinite(ga["env"]))
    # away from the NaN channels the gradients are those of the zeroed map
    # (up to the order in which the oracle's threads add samples)
    assert np.allclose(ga["env"][~mask], gb["env"][~mask], rtol=1e-12, atol=0)
    assert np.allclose(ga["vmat"], gb["vmat"], rtol=1e-12, atol=1e-300)
    # a zero channel still passes its derivative (closed interval), so some differ
    assert np.any(gb["env"][mask] != 0.0)
