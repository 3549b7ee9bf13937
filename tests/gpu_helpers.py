"""Helpers for GPU tests: move a seeded Problem to the device and compare
complex outputs with the oracle at the parity bar."""
import json
import os
import sys

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# Parity bar: every complex output entry within 1e-12 relative (complex
# modulus) of the oracle; an entry whose exact value is 0 must stay below
# 1e-12 times the sum of |term| that produced it.
RTOL = 1e-12


def to_device(prob, device="cuda:0"):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return dict(aqsmtemp=t(prob.aqsmtemp), aqsntemp=t(prob.aqsntemp),
                I_eps_array=t(prob.I_eps_array),
                wtilde_array=t(prob.wtilde_array), vcoul=t(prob.vcoul),
                wx_array=t(prob.wx_array))


def rel_errors(got, ref, abs_sum):
    got = np.asarray(got)
    ref = np.asarray(ref)
    err = np.abs(got - ref)
    denom = np.where(np.abs(ref) > 0, np.abs(ref), np.asarray(abs_sum) + 1e-300)
    return err / denom


def assert_parity(got, ref, abs_sum, what=""):
    r = rel_errors(got, ref, abs_sum)
    assert np.all(r <= RTOL), f"{what}: max rel err {r.max():.3e} > {RTOL} " \
                              f"(got {got}, ref {ref})"
    return float(r.max())


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def load_golden(key):
    path = os.path.join(GOLDEN, f"fwd_{key}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    c = lambda pairs: np.array([complex(a, b) for a, b in pairs])
    rec["ach"] = c(rec["achtemp"])
    rec["asx"] = c(rec["asxtemp"])
    return rec


def mixed_pole_problem(seed, dims, frac):
    """A problem whose tiles mix lanes with (Im om)^2 below 2^-60 (real om,
    or |Im om| ~ 1e-10) and ordinary lanes; a fifth of the real ones sit
    exactly on a frequency (x == om, a zero denominator).  Such lanes invert
    their denominators one by one in the kernels."""
    from paper_2008_11326_amd import inputs as I
    prob = I.make_problem(dims, seed)
    rng = np.random.default_rng(seed)
    wt = prob.wtilde_array
    low = rng.random(wt.shape) < frac
    tiny = low & (rng.random(wt.shape) < 0.3)
    wt.imag[low] = 0.0
    wt.imag[tiny] = rng.uniform(-1e-10, 1e-10, int(tiny.sum()))
    pole = low & ~tiny & (rng.random(wt.shape) < 0.2)
    wt.real[pole] = rng.choice(prob.wx_array.ravel(), size=int(pole.sum()))
    return prob
