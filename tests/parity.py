"""Helpers shared by the GPU parity tests: compare the HIP path with the FP64
oracle per sample or per pixel, with the decision-hash flip mask.

Conditioning.  The FP32 kernels carry a few ulps of rounding in every unit
vector they derive (camera ray, geometric normal, frame, candidate and
continuation directions).  Some results are ill-conditioned at that level:
a texel's share of a bilinear footprint on a small triangle, a grazing
cosine, or a near-mirror GGX lobe move by up to 1e-2 when those vectors move
by a few ulps.  So every comparison also evaluates the oracle with its
conditioning hook on (orc_options.jitter: each such vector moved by up to
JITTER units of 2^-24 per component, TRIALS seeded trials).  A sample whose
decisions change in some trial sits on a decision boundary and counts like
a flip; and an element may differ from the oracle by up to SPREAD_FACTOR
times the spread of the oracle's own results over the trials, on top of the
fixed bar.  Every report prints how many elements needed that allowance."""
import copy

import numpy as np

REL, ABS = 1e-4, 1e-6      # per-pixel bar: 1e-4 relative or 1e-6 absolute
PIXEL_FRAC = 1e-3          # at most 0.1 % of pixels outside it, each one on a decision flip
GRAD_REL = 1e-3            # gradient bar: 1e-3 relative to the FP64 gradient ...
GRAD_FLOOR = 1e-3          # ... with an absolute floor of 1e-3 x RMS of the group (cancelled texels)
JITTER = 8.0               # oracle trials: unit vectors moved by up to this many 2^-24 per component
TRIALS = 4
SPREAD_FACTOR = 2.0


def within(g, o, rel=REL, abs_=ABS):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return (np.abs(g - o) <= rel * np.abs(o) + abs_).all(-1)


def sample_report(g_rgb, g_hash, o_rgb, o_hash):
    ok = within(g_rgb, o_rgb)
    flip = np.asarray(g_hash).view(np.uint32) != np.asarray(o_hash).view(np.uint32)
    return ok, flip


def pixel_report(g_pix, o_rgb, g_hash, o_hash, spp):
    """Per pixel: the GPU's pixel value against the mean of the oracle's
    samples of that pixel (items ordered pixel after pixel, `spp` samples
    each), and whether any of its samples took another decision."""
    spp = np.asarray(spp, np.int64)
    first = np.concatenate([[0], np.cumsum(spp)[:-1]])
    o_pix = np.add.reduceat(np.asarray(o_rgb, np.float64), first, axis=0) / spp[:, None]
    fs = np.asarray(g_hash).view(np.uint32) != np.asarray(o_hash).view(np.uint32)
    flip = np.add.reduceat(fs.astype(np.int64), first) > 0
    ok = within(g_pix, o_pix)
    return ok, flip, o_pix


def assert_pixel_bar(ok, unstable, name="", frac=PIXEL_FRAC, admitted=None):
    """At most `frac` of the pixels outside the bar, and every one of them on
    a decision flip (or a decision the oracle itself changes in a
    conditioning trial)."""
    n = ok.size
    bad = int(np.sum(~ok))
    unexplained = int(np.sum(~ok & ~unstable))
    extra = "" if admitted is None else f" within-conditioning={int(np.sum(admitted))}"
    print(f"[{name}] pixels={n} outside-bar={bad} unstable={int(np.sum(unstable))} "
          f"outside-without-flip={unexplained}{extra}", flush=True)
    assert unexplained == 0, f"{name}: {unexplained} pixels outside the bar without a decision flip"
    assert bad <= frac * n, f"{name}: {bad} of {n} pixels outside the bar"


def forward_pixels(g_pix, o_rgb, g_hash, o_hash, spp, trials):
    """Per pixel (items pixel after pixel, `spp` samples each): ok (within
    the bar, or within SPREAD_FACTOR x the spread of the oracle's pixel over
    the conditioning trials), unstable (a sample took another decision on the
    GPU, or changes its decision in some trial) and the conditioning-admitted
    mask (ok only through the spread)."""
    spp = np.asarray(spp, np.int64)
    first = np.concatenate([[0], np.cumsum(spp)[:-1]])
    ok_plain, flip, o_pix = pixel_report(g_pix, o_rgb, g_hash, o_hash, spp)
    near = np.zeros_like(flip)
    spread = np.zeros_like(o_pix)
    for ot, ht, _ in trials:
        near |= np.add.reduceat((np.asarray(ht) != np.asarray(o_hash)).astype(np.int64), first) > 0
        spread = np.maximum(spread, np.abs(np.add.reduceat(ot, first, axis=0) / spp[:, None] - o_pix))
    g = np.asarray(g_pix, np.float64)
    cond_ok = (np.abs(g - o_pix) <= SPREAD_FACTOR * spread).all(-1)
    ok = ok_plain | cond_ok
    return ok, flip | near, ok & ~ok_plain


def grad_report(g, o, spread=None):
    """Elements outside the gradient bar (plus SPREAD_FACTOR x the oracle's
    spread over the conditioning trials when `spread` is given), and the RMS."""
    g = np.asarray(g, np.float64).reshape(-1)
    o = np.asarray(o, np.float64).reshape(-1)
    rms = np.sqrt(np.mean(o ** 2)) + 1e-300
    tol = GRAD_REL * np.abs(o) + GRAD_FLOOR * rms
    if spread is not None:
        tol = tol + SPREAD_FACTOR * np.asarray(spread, np.float64).reshape(-1)
    bad = ~(np.abs(g - o) <= tol)
    return bad, rms


def jittered(opts, seed, jitter=JITTER):
    """A copy of the options with the oracle's conditioning hook on."""
    o = copy.copy(opts)
    o.jitter, o.jitter_seed = float(jitter), int(seed)
    return o


def oracle_trials(orc, views, opts, items, dl=None, trials=TRIALS, seed=1234, **kw):
    """The oracle with its conditioning hook on: per trial the sample values
    and hashes, and (with dl) the gradients.  Extra keywords (the reuse
    history `prev`) go to the oracle calls."""
    res = []
    for t in range(trials):
        oj = jittered(opts, seed + t)
        o, h = orc.render(views, oj, items, **kw)[:2]
        g = orc.grad(views, oj, items, dl, **kw) if dl is not None else None
        res.append((o, h, g))
    return res


def describe_bad(g, o, bad, rms, k=8):
    """The worst elements outside the gradient bar, for the log."""
    g = np.asarray(g, np.float64).reshape(-1)
    o = np.asarray(o, np.float64).reshape(-1)
    idx = np.flatnonzero(bad)
    if idx.size == 0:
        return ""
    err = np.abs(g[idx] - o[idx]) / (GRAD_REL * np.abs(o[idx]) + GRAD_FLOOR * rms)
    top = idx[np.argsort(-err)[:k]]
    return " ".join(f"[{i}] gpu={g[i]:.6e} orc={o[i]:.6e} |o|/rms={abs(o[i]) / rms:.2e} "
                    f"err/bar={abs(g[i] - o[i]) / (GRAD_REL * abs(o[i]) + GRAD_FLOOR * rms):.2f}" for i in top)


def unstable_samples(orc, views, opts, items, o_hash, trials=TRIALS, seed=1234, **kw):
    """Samples whose oracle decisions change in some conditioning trial."""
    near = np.zeros(len(items), bool)
    for t in range(trials):
        h = orc.render(views, jittered(opts, seed + t), items, **kw)[1]
        near |= np.asarray(h) != np.asarray(o_hash)
    return near


def check_gradients(got, orc, views, opts, items, dl, label, trials=TRIALS, seed=1234, **kw):
    """Every element of every parameter group within the gradient bar, with
    SPREAD_FACTOR x the spread of the oracle's gradient over the conditioning
    trials added to the tolerance.  `got` maps group names to the GPU's
    arrays; returns the oracle's gradients."""
    og = orc.grad(views, opts, items, dl, **kw)
    spread = {k: np.zeros_like(v) for k, v in og.items()}
    for t in range(trials):
        gt = orc.grad(views, jittered(opts, seed + t), items, dl, **kw)
        for k in og:
            spread[k] = np.maximum(spread[k], np.abs(gt[k] - og[k]))
    failed = []
    for k in og:
        a = np.asarray(got[k], np.float64)
        assert np.all(np.isfinite(a)), f"{label}: non-finite {k} gradient"
        bad, rms = grad_report(a, og[k], spread[k])
        plain, _ = grad_report(a, og[k])
        print(f"[{label}] grad {k}: rms={rms:.3e} outside-bar={int(bad.sum())}/{bad.size} "
              f"within-conditioning={int((plain & ~bad).sum())} {describe_bad(a, og[k], bad, rms)}", flush=True)
        if bad.any():
            failed.append(k)
    assert not failed, f"{label}: gradients outside the bar: {failed}"
    return og

