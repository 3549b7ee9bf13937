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


def qp_bounds(ach, asx, ach_abs, asx_abs, freq_step, vxc, z, sigma_mid):
    """Error bounds for the quasiparticle quantities (Sigma re/im, dSigma/dE
    re/im, Z, E_qp) that follow from the per-output parity bar: each
    Sigma(E_w) = achtemp[w] - asxtemp[w] may be off by RTOL times the sum of
    its parts' moduli (their sums of |term| where a part is 0); the central
    difference divides two of those by 2 freq_step; Z = 1/(1 - Re dSigma)
    moves by Z^2 times that; E_qp by the change of Z times |Re Sigma - V_xc|
    plus Z times the error of Sigma.  A few ulp of the epilogue's own
    arithmetic are added to each."""
    ach, asx = np.asarray(ach), np.asarray(asx)
    part = lambda v, s: np.where(np.abs(v) > 0, np.abs(v), np.asarray(s))
    eps = RTOL * (part(ach, ach_abs) + part(asx, asx_abs))
    m = (len(ach) - 1) // 2
    ulp = 8 * np.finfo(float).eps
    t_sig = eps[m] + ulp * abs(sigma_mid)
    t_d = (eps[m + 1] + eps[m - 1]) / (2 * freq_step)
    t_d += ulp * (abs(ach[m + 1] - asx[m + 1]) + abs(ach[m - 1] - asx[m - 1])) / (2 * freq_step)
    t_z = 2 * z * z * t_d + ulp * abs(z)
    t_e = t_z * abs(sigma_mid.real - vxc) + abs(z) * t_sig + ulp * (abs(z * (sigma_mid.real - vxc)) + 1)
    return np.array([t_sig, t_sig, t_d, t_d, t_z, t_e])


def qp_vector(q):
    """The oracle's quasiparticle dict as the library's qp[6] layout."""
    return np.array([q["sigma"].real, q["sigma"].imag, q["dsigma"].real, q["dsigma"].imag,
                     q["z"], q["e_qp"]])
