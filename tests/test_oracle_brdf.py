"""Pins of the oracle's BRDF (Disney-style albedo + roughness (+ metallic),
Sec. 3 "Intrinsic decomposition") and its sampler (GGX visible-normal
importance sampling cited in Sec. 4.2, mixed with cosine sampling)."""
import numpy as np
import pytest
from scipy import integrate, stats


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


N = np.array([0.0, 0.0, 1.0])


@pytest.mark.parametrize("alpha", [0.01, 0.1, 0.3, 0.7, 1.0])
def test_ggx_normalisation(oracle_lib, alpha):
    # int D(h) (n.h) dw_h = 1 over the hemisphere
    f = lambda th: oracle_lib.ggx_d(alpha, np.cos(th)) * np.cos(th) * np.sin(th) * 2 * np.pi
    pts = [0.0, min(10 * alpha, 1.0), np.pi / 2]
    val = sum(integrate.quad(f, a, b, limit=400, epsabs=1e-12)[0] for a, b in zip(pts[:-1], pts[1:]))
    assert abs(val - 1.0) < 1e-6
    assert abs(oracle_lib.ggx_d(alpha, 1.0) - 1.0 / (np.pi * alpha ** 2)) < 1e-9 / alpha ** 2


def test_smith_g1_limits(oracle_lib):
    assert abs(oracle_lib.ggx_g1(0.5, 1.0) - 1.0) < 1e-15
    # Lambda for alpha -> 0 vanishes
    assert abs(oracle_lib.ggx_g1(1e-6, 0.3) - 1.0) < 1e-9
    # closed form at alpha = 1, theta = 60 deg: tan^2 = 3, Lambda = (-1 + 2)/2
    assert abs(oracle_lib.ggx_g1(1.0, 0.5) - 1.0 / 1.5) < 1e-12


def _hemi_integral(fn, n_t=200, n_p=400):
    th = (np.arange(n_t) + 0.5) * (np.pi / 2) / n_t
    ph = (np.arange(n_p) + 0.5) * 2 * np.pi / n_p
    tot = 0.0
    for t in th:
        for p in ph:
            tot += fn(np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])) * np.sin(t)
    return tot * (np.pi / 2 / n_t) * (2 * np.pi / n_p)


def test_lambert_albedo_integral(oracle_lib):
    m = [0.2, 0.5, 0.8, 0.6, 0.0]
    wo = _unit([0.3, -0.2, 0.9])
    val = _hemi_integral(lambda wi: oracle_lib.brdf_eval(N, wo, wi, m, brdf=0) * wi[2], 100, 200)
    assert np.allclose(val, [0.2, 0.5, 0.8], rtol=1e-3)


def test_reciprocity_and_zero_below(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(200):
        a = _unit(rng.normal(size=3)); a[2] = abs(a[2])
        b = _unit(rng.normal(size=3)); b[2] = abs(b[2])
        m = rng.uniform(0, 1, 5)
        assert np.allclose(oracle_lib.brdf_eval(N, a, b, m), oracle_lib.brdf_eval(N, b, a, m), rtol=1e-12)
        below = b * np.array([1, 1, -1])
        assert np.all(oracle_lib.brdf_eval(N, a, below, m) == 0)


def test_vndf_identity(oracle_lib):
    """Specular-only lobe: f cos / pdf_vndf = F * G1(wi)."""
    rng = np.random.default_rng(2)
    for _ in range(300):
        wo = _unit(rng.normal(size=3)); wo[2] = abs(wo[2]) + 0.05; wo = _unit(wo)
        r = rng.uniform(0.1, 1.0)
        m = [1.0, 1.0, 1.0, r, 1.0]              # F0 = 1 (metal, white): diffuse = 0, F = 1
        lobe, wi = oracle_lib.brdf_sample(N, wo, m, [0.0, *rng.random(2)])
        if lobe == 0:
            continue
        assert lobe == 2
        f = oracle_lib.brdf_eval(N, wo, wi, m)
        pmix = oracle_lib.brdf_pdf(N, wo, wi, m)
        p_spec = 0.9                              # clamp(1 / (1 + 0), 0.1, 0.9)
        pv = (pmix - (1 - p_spec) * wi[2] / np.pi) / p_spec
        g1 = oracle_lib.ggx_g1(r * r, wi[2])
        assert np.allclose(f * wi[2] / pv, g1, rtol=1e-9)


@pytest.mark.parametrize("m", [[0.5, 0.4, 0.3, 0.3, 0.0], [0.9, 0.7, 0.2, 0.6, 1.0], [0.2, 0.2, 0.2, 0.15, 0.5]])
def test_mixture_sampler_chi2(oracle_lib, m):
    """Histogram of sampled directions (over (cos theta, phi) cells) against
    the mixture pdf integrated over each cell."""
    wo = _unit([0.4, 0.1, 0.8])
    rng = np.random.default_rng(4)
    n = 60000
    nt, npf = 8, 8
    counts = np.zeros((nt, npf))
    invalid = 0
    for u in rng.random((n, 3)):
        lobe, wi = oracle_lib.brdf_sample(N, wo, m, u)
        if lobe == 0:
            invalid += 1
            continue
        ct = wi[2]
        ph = np.arctan2(wi[1], wi[0]) % (2 * np.pi)
        counts[min(int((1 - ct) * nt), nt - 1), min(int(ph / (2 * np.pi) * npf), npf - 1)] += 1
    expect = np.zeros((nt, npf))
    sub = 12
    for i in range(nt):
        for j in range(npf):
            tot = 0.0
            for a in range(sub):
                ct = 1 - (i + (a + 0.5) / sub) / nt
                st = np.sqrt(1 - ct * ct)
                for b in range(sub):
                    ph = (j + (b + 0.5) / sub) * 2 * np.pi / npf
                    wi = np.array([st * np.cos(ph), st * np.sin(ph), ct])
                    tot += oracle_lib.brdf_pdf(N, wo, wi, m)
            expect[i, j] = tot / sub ** 2 * (1.0 / nt) * (2 * np.pi / npf) * n
    # all mass accounted for: valid samples + invalid (reflected below) = n
    assert abs(expect.sum() + invalid - n) < 0.01 * n
    mask = expect > 20
    chi2 = ((counts[mask] - expect[mask]) ** 2 / expect[mask]).sum()
    assert stats.chi2.sf(chi2, df=int(mask.sum()) - 1) > 1e-4


def test_frame_orthonormal(oracle_lib):
    """Orthonormal basis with n as third axis, also for axis-aligned normals."""
    rng = np.random.default_rng(9)
    ns = [_unit(rng.normal(size=3)) for _ in range(100)] + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                                             np.array([0, 1.0, 0]), np.array([0, -1.0, 0])]
    for n in ns:
        t, b = oracle_lib.frame(n)
        M = np.stack([t, b, n])
        assert np.allclose(M[2], n)
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert abs(abs(np.linalg.det(M)) - 1.0) < 1e-12   # handedness is irrelevant


@pytest.mark.parametrize("mu", [0.0, 0.3, 0.7, 1.0])
def test_schlick_f0_metallic_blend_at_normal_incidence(oracle_lib, mu):
    """At wo = wi = n the half vector is n, so the Schlick factor is F0 itself,
    D(1) = 1 / (pi alpha^2) and G1 = 1 on both sides:
    f = (1 - mu) a / pi + F0 / (4 pi alpha^2) with F0 = 0.04 (1 - mu) + mu a.
    A blend with the weights swapped, or F0 without the albedo, fails for
    0 < mu < 1 or for coloured albedo."""
    for a, r in [((0.2, 0.5, 0.9), 0.5), ((1.0, 0.0, 0.35), 0.3), ((0.05, 0.6, 0.75), 0.9)]:
        a = np.array(a)
        alpha = r * r
        f = oracle_lib.brdf_eval(N, N, N, [*a, r, mu], brdf=1)
        f0 = 0.04 * (1.0 - mu) + mu * a
        expect = (1.0 - mu) * a / np.pi + f0 / (4.0 * np.pi * alpha ** 2)
        assert np.allclose(f, expect, rtol=1e-12, atol=0), (a, r, f, expect)
        # the Lambert-only BRDF keeps the diffuse part alone
        fl = oracle_lib.brdf_eval(N, N, N, [*a, r, mu], brdf=0)
        assert np.allclose(fl, (1.0 - mu) * a / np.pi, rtol=1e-12, atol=0)
