"""Helpers shared by the GPU parity tests: compare the HIP path with the FP64
oracle per sample, with the decision-hash flip mask."""
import numpy as np

REL, ABS = 1e-4, 1e-6      # per-pixel bar: 1e-4 relative or 1e-6 absolute
GRAD_REL = 1e-3            # gradient bar: 1e-3 relative to the FP64 gradient ...
GRAD_FLOOR = 1e-3          # ... with an absolute floor of 1e-3 x RMS of the group (cancelled texels)


def within(g, o, rel=REL, abs_=ABS):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return (np.abs(g - o) <= rel * np.abs(o) + abs_).all(-1)


def sample_report(g_rgb, g_hash, o_rgb, o_hash):
    ok = within(g_rgb, o_rgb)
    flip = np.asarray(g_hash).view(np.uint32) != np.asarray(o_hash).view(np.uint32)
    return ok, flip


def grad_report(g, o):
    g = np.asarray(g, np.float64).reshape(-1)
    o = np.asarray(o, np.float64).reshape(-1)
    rms = np.sqrt(np.mean(o ** 2)) + 1e-300
    bad = np.abs(g - o) > GRAD_REL * np.abs(o) + GRAD_FLOOR * rms
    return bad, rms
