"""Pins of the oracle's environment-map proposal (Sec. 4.1: candidates drawn
from a distribution proportional to L_env, on the 256x512 HDR map of
Sec. 3 "Intrinsic decomposition")."""
import numpy as np
from scipy import stats

from paper_2406_16360_amd import synth


def _env_oracle(oracle_lib, eh=16, ew=32, seed=3):
    rng = np.random.default_rng(seed)
    env = synth.hdr_env(eh, ew, rng, [(30.0, 10.0)])
    sc = synth.plane_scene()
    sc.env = env
    return oracle_lib.Oracle(sc, use_bvh=False), env


def _dir(theta, phi):
    return np.array([np.sin(theta) * np.sin(phi), np.cos(theta), -np.sin(theta) * np.cos(phi)])


def test_pdf_integrates_to_one(oracle_lib):
    o, _ = _env_oracle(oracle_lib)
    # midpoint quadrature over (theta, phi): dw = sin(theta) dtheta dphi
    nt, npf = 640, 1280
    th = (np.arange(nt) + 0.5) * np.pi / nt
    ph = (np.arange(npf) + 0.5) * 2 * np.pi / npf - np.pi
    tot = 0.0
    for t in th:
        s = np.sin(t)
        tot += sum(o.env_pdf(_dir(t, p)) for p in ph[::1]) * s
    tot *= (np.pi / nt) * (2 * np.pi / npf)
    assert abs(tot - 1.0) < 2e-3


def test_sampler_matches_pdf_chi2(oracle_lib):
    o, env = _env_oracle(oracle_lib, eh=8, ew=16)
    rng = np.random.default_rng(11)
    n = 40000
    counts = np.zeros(8 * 16)
    w = env.clip(min=0).mean(-1) * np.sin(np.pi * (np.arange(8) + 0.5) / 8)[:, None]
    expect = (w / w.sum()).reshape(-1) * n
    for u0, u1 in rng.random((n, 2)):
        ok, d, pdf, tex = o.env_sample(u0, u1)
        assert ok
        counts[tex] += 1
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert stats.chi2.sf(chi2, df=8 * 16 - 1) > 1e-3


def test_sample_consistency(oracle_lib):
    """The sampled texel equals the texel looked up from the sampled
    direction, and the density returned with the sample equals the density
    evaluated from the direction."""
    o, _ = _env_oracle(oracle_lib)
    rng = np.random.default_rng(5)
    for u0, u1 in rng.random((2000, 2)):
        ok, d, pdf, tex = o.env_sample(u0, u1)
        t2, _ = o.env_lookup(d)
        assert t2 == tex
        assert abs(o.env_pdf(d) - pdf) <= 1e-7 * pdf  # sqrt(1 - y^2) vs sin(theta) near the poles


def test_lookup_axes(oracle_lib):
    """Equirectangular convention: +y is row 0, -z is the centre column."""
    o, env = _env_oracle(oracle_lib, eh=16, ew=32)
    t, rgb = o.env_lookup([0, 1, 0])
    assert t // 32 == 0
    t, _ = o.env_lookup([0, -1, 0])
    assert t // 32 == 15
    t, rgb = o.env_lookup([0, 0, -1])        # theta = pi/2, phi = 0 -> u = 1/2
    assert t == 8 * 32 + 16
    assert np.allclose(rgb, np.maximum(env[8, 16], 0))
    t, _ = o.env_lookup([1, 0, 0])            # phi = pi/2 -> u = 3/4
    assert t == 8 * 32 + 24
