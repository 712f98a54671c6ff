"""Pins of the oracle's gradient: the detached-sampling derivative of the
path functional (the adjoint of Sec. 4.2's path tracer; the paper's choice
of detaching indirect rays is the grad_mode=1 variant).  Pinned by central
finite differences of the frozen functional and by closed forms."""
import copy

import numpy as np
import pytest

from paper_2406_16360_amd import synth


def _perturbed(scene, field, idx, delta):
    sc = copy.copy(scene)
    arr = getattr(scene, field).copy()
    flat = arr.reshape(-1)
    old = np.float64(flat[idx])
    flat[idx] = np.float32(old + delta)
    setattr(sc, field, arr)
    return sc, np.float64(flat[idx]) - old


def _dense_grads(o, wl, item):
    """d C_c / d theta for the three channels of one sample."""
    out = []
    for c in range(3):
        dl = np.zeros((1, 3)); dl[0, c] = 1.0
        out.append(o.grad(wl.views, wl.opts, np.array([item]), dl))
    return out


def _fd_check(oracle_lib, wl, items, fields, h=2.0 ** -11, rtol=2e-4, max_params=40, one_sided=False):
    o = oracle_lib.Oracle(wl.scene)
    checked = 0
    for item in items:
        g = _dense_grads(o, wl, item)
        for field in fields:
            key = field if field != "vmat" else "vmat"
            dense = np.stack([g[c][key].reshape(-1) for c in range(3)], 0)    # [3, P]
            nz = np.nonzero(np.abs(dense).sum(0))[0]
            for idx in nz[:max_params]:
                sp, dp = _perturbed(wl.scene, field, idx, h)
                cp = o.frozen(oracle_lib.Oracle(sp, use_bvh=False), wl.views, wl.opts, item)
                if one_sided:
                    c0 = o.frozen(o, wl.views, wl.opts, item)
                    fd = (cp - c0) / dp
                else:
                    sm, dm = _perturbed(wl.scene, field, idx, -h)
                    cm = o.frozen(oracle_lib.Oracle(sm, use_bvh=False), wl.views, wl.opts, item)
                    fd = (cp - cm) / (dp - dm)
                an = dense[:, idx]
                scale = np.abs(an).max() + 1e-12
                assert np.all(np.abs(fd - an) <= rtol * scale), (field, idx, fd, an)
                checked += 1
    return checked


def _c1_interior():
    w = synth.config1()
    rng = np.random.default_rng(4)
    # metallic strictly inside (0, 1) so central differences do not straddle the clamp
    w.scene.vmat[:, 4] = rng.uniform(0.2, 0.8, w.scene.vmat.shape[0]).astype(np.float32)
    return w


def test_fd_vertex_materials_full(oracle_lib):
    w = _c1_interior()
    items = synth.sample_items(w, 6, 3)
    assert _fd_check(oracle_lib, w, items, ["vmat", "env"]) > 50


def test_fd_vertex_materials_primary(oracle_lib):
    w = _c1_interior()
    w.opts.grad_mode = 1
    items = synth.sample_items(w, 6, 8)
    assert _fd_check(oracle_lib, w, items, ["vmat", "env"]) > 20


def _tex_workload(tex_res=16):
    rng = np.random.default_rng(12)
    pos, faces, uv = synth.displaced_latlong_sphere(12, 24, 0.2, rng)
    box = synth.ground_box(-1.45, -1.25, 4.0)
    pos, faces, uv = synth.merge([(pos, faces, uv), box])
    albedo, rough, metal = synth.noise_textures(tex_res, rng)
    metal = (0.2 + 0.6 * metal).astype(np.float32)
    env = synth.hdr_env(8, 16, rng, [(20.0, 10.0)])
    sc = synth.Scene(pos=pos, faces=faces, env=env, mat_mode=1, uv=uv, albedo=albedo, rough=rough, metal=metal)
    v = synth.View(c2w=synth.orbit(3.0, 25.0, 0.7), fov_y_deg=40.0, w=16, h=16, spp=2)
    return synth.Workload("t", sc, [v], synth.Options(bounces=3, ris_m=8, ris_m_brdf=4, seed=5))


def test_fd_textures(oracle_lib):
    w = _tex_workload()
    items = synth.sample_items(w, 5, 1)
    assert _fd_check(oracle_lib, w, items, ["albedo", "rough", "metal", "env"], max_params=16) > 40


def test_fd_zero_albedo_channel(oracle_lib):
    """A Lambert vertex with an exactly-zero albedo channel makes that channel
    of the continuation weight zero; the derivative through it is still the
    frozen functional's (one-sided difference at the clamp's lower end)."""
    w = _c1_interior()
    w.scene.vmat[:, 0] = 0.0
    w.opts.brdf = 0
    items = synth.sample_items(w, 5, 2)
    assert _fd_check(oracle_lib, w, items, ["vmat"], one_sided=True, rtol=2e-3) > 20


def test_closed_form_plane(oracle_lib):
    """Plane under constant L with cosine candidates: C = (1 - mu) a L, so
    dC_c/da_c = (1 - mu) L summed over the vertex weights, dC_c/dmu = -a_c L,
    and the env derivative sums to (1 - mu) a_c."""
    a = np.array([0.3, 0.5, 0.7], np.float32)
    L = 2.0
    sc = synth.plane_scene(tuple(a), L)
    mu = np.float32(0.25)
    sc.vmat[:, 4] = mu
    o = oracle_lib.Oracle(sc)
    v = synth.View(c2w=synth.look_at([0.0, 3.0, 2.0]), fov_y_deg=40.0, w=8, h=8, spp=1)
    wl = synth.Workload("p", sc, [v], synth.Options(bounces=2, ris_m=4, ris_m_brdf=4, brdf=0, seed=1))
    for item in synth.sample_items(wl, 5, 0):
        for c in range(3):
            dl = np.zeros((1, 3)); dl[0, c] = 1.0
            g = o.grad(wl.views, wl.opts, np.array([item]), dl)
            da = g["vmat"][:, c].sum()
            dmu = g["vmat"][:, 4].sum()
            denv = g["env"][..., c].sum()
            assert abs(da - (1 - float(mu)) * L) < 1e-9
            assert abs(dmu + float(a[c]) * L) < 1e-9
            assert abs(denv - (1 - float(mu)) * float(a[c])) < 1e-9
            assert np.abs(g["vmat"][:, 3]).max() < 1e-12   # Lambert: no roughness dependence


def test_primary_equals_full_on_single_vertex_paths(oracle_lib):
    sc = synth.furnace_scene(1.0)
    sc.vmat[:, :3] = np.array([0.4, 0.6, 0.8], np.float32)
    o = oracle_lib.Oracle(sc)
    v = synth.View(c2w=synth.look_at([0.0, 0.5, 3.0]), fov_y_deg=40.0, w=8, h=8, spp=1)
    items = synth.all_items(synth.Workload("f", sc, [v], synth.Options()))
    dl = np.random.default_rng(0).random((items.shape[0], 3))
    ga = o.grad([v], synth.Options(bounces=3, ris_m=8, ris_m_brdf=4, grad_mode=0), items, dl)
    gb = o.grad([v], synth.Options(bounces=3, ris_m=8, ris_m_brdf=4, grad_mode=1), items, dl)
    for k in ga:
        assert np.allclose(ga[k], gb[k], rtol=1e-12, atol=1e-15)
