"""Pins of the oracle's quasiparticle step (oracle/qp.py) against things
other than itself.

The kernel's outputs are the Coulomb-hole and screened-exchange sums of the
self-energy at nfreq frequencies E_w = E + (w - m) h (the Sigma module of
Sec. II-A; the workloads' wx_array = E_w - e_n).  The step forms
Sigma(E_w) = achtemp[w] - asxtemp[w], dSigma/dE at E by a central
difference, Z = 1/(1 - Re dSigma/dE) and E_qp = E + Z (Re Sigma(E) - V_xc).

* a central difference is exact for a self-energy affine in E;
* single-pole closed forms (uniform arrays): Sigma at each frequency, the
  difference quotient, Z and E_qp in exact rationals, from the oracle's own
  forward outputs;
* with a small step the difference quotient approaches the exact
  derivative of the closed form, d/dx of the plasmon-pole terms, within
  the h^2 truncation bound -- which pins the spacing factor, the sign of
  the exchange part and the choice of the middle frequency.
"""
import math
from fractions import Fraction

import pytest

import oracle
from tests.test_oracle_pins import _Q, _uniform_problem


def test_affine_self_energy_is_differenced_exactly():
    h, E, vxc = 0.375, -0.25, 0.125
    alpha, beta = complex(1.5, -0.75), complex(-0.3125, 0.0625)
    gamma = complex(0.5, 0.25)   # constant split between the two parts
    for nw in (3, 5, 7):
        m = (nw - 1) // 2
        Ew = [E + (w - m) * h for w in range(nw)]
        sig = [alpha + beta * e for e in Ew]
        ach = [s + gamma for s in sig]
        asx = [gamma] * nw
        q = oracle.quasiparticle(ach, asx, h, energy=E, vxc=vxc)
        assert q["dsigma"] == beta
        assert q["sigma"] == alpha + beta * E
        z = 1.0 / (1.0 - beta.real)
        assert q["z"] == z
        assert abs(q["e_qp"] - (E + z * ((alpha + beta * E).real - vxc))) <= 1e-16


def test_rejects_even_or_short_frequency_sets():
    for nw in (1, 2, 4):
        with pytest.raises(ValueError):
            oracle.quasiparticle([0j] * nw, [0j] * nw, 0.5)
    with pytest.raises(ValueError):
        oracle.quasiparticle([0j] * 3, [0j] * 3, 0.0)


# uniform arrays: every (p, g) repeats the same term
OM = _Q(Fraction(5, 4), Fraction(1, 16))
EPS, A, B, V = _Q(Fraction(1, 2), Fraction(-1, 4)), _Q(1, Fraction(1, 2)), \
    _Q(Fraction(-1, 4), Fraction(3, 4)), Fraction(3, 8)
NB, NV, NG, NP = 4, 2, 40, 6


def _exact_sigma(x, n):
    """(CH, SX) terms of band n at frequency argument x (exact), summed over
    every (p, g): NP NG v M e times the plasmon-pole value."""
    d = x + _Q(-OM.re, -OM.im)
    s = x + OM
    pref = _Q(NP * NG) * A * B.conj() * EPS
    if d.re ** 2 + d.im ** 2 > Fraction(1, 4):
        ch = pref * _Q(V / 2) * OM * d.inv()
        sx = pref * _Q(V) * OM * OM * (d * s).inv()
    else:
        ch = _Q(0)
        sx = pref * _Q(V) * _Q(Fraction(-1, 2)) * OM * s.inv()
    return ch, (sx if n < NV else _Q(0))


def _exact_dsigma(x, n):
    """d/dx of band n's (CH - SX) terms: the derivative of the plasmon-pole
    values in their branch (the branch does not change near x)."""
    d = x + _Q(-OM.re, -OM.im)
    s = x + OM
    pref = _Q(NP * NG) * A * B.conj() * EPS
    if d.re ** 2 + d.im ** 2 > Fraction(1, 4):
        # d/dx om/(x - om) = -om/(x - om)^2;  d/dx om^2/((x-om)(x+om)) = -2 x om^2/((x-om)(x+om))^2
        dch = pref * _Q(V / 2) * _Q(-1) * OM * (d * d).inv()
        ds = d * s
        dsx = pref * _Q(V) * _Q(-2) * x * OM * OM * (ds * ds).inv()
    else:
        # d/dx -om/(2 (x + om)) = om / (2 (x + om)^2)
        dch = _Q(0)
        dsx = pref * _Q(V) * _Q(Fraction(1, 2)) * OM * (s * s).inv()
    return dch + _Q(-1) * (dsx if n < NV else _Q(0))


def _problem(E, h, e_n, nw=3):
    m = (nw - 1) // 2
    xs = [[float(E + (w - m) * h - en) for w in range(nw)] for en in e_n]
    return _uniform_problem(NB, NV, NG, NP, xs, OM.c(), EPS.c(), A.c(), B.c(), float(V)), xs


def test_single_pole_closed_form():
    E, h, vxc = Fraction(1, 4), Fraction(1, 2), Fraction(-3, 8)
    e_n = [Fraction(-2), Fraction(-3, 4), Fraction(3, 2), Fraction(5, 2)]
    prob, xs = _problem(E, h, e_n)
    ach, asx, _, _ = oracle.sigma_fwd(prob, nthreads=1)
    q = oracle.quasiparticle(ach, asx, float(h), energy=float(E), vxc=float(vxc))
    sig = []
    for w in range(3):
        tot = _Q(0)
        for n in range(NB):
            ch, sx = _exact_sigma(_Q(Fraction(xs[n][w])), n)
            tot = tot + ch + _Q(-1) * sx
        sig.append(tot)
    dsig = (sig[2] + _Q(-1) * sig[0]) * _Q(1 / (2 * h))
    z = 1 / (1 - dsig.re)
    e_qp = E + z * (sig[1].re - vxc)
    scale = max(abs(sig[w].c()) for w in range(3))
    assert abs(q["sigma"] - sig[1].c()) <= 1e-14 * scale
    assert abs(q["dsigma"] - dsig.c()) <= 1e-14 * scale / float(h)
    assert abs(q["z"] - float(z)) <= 1e-13 * abs(float(z))
    assert abs(q["e_qp"] - float(e_qp)) <= 1e-13 * max(1.0, abs(float(e_qp)))


def test_difference_quotient_approaches_the_derivative():
    """h = 2^-10: the central difference differs from the exact derivative
    by h^2/6 times the third derivative, here below 1e-5 relative; a step
    counted once instead of twice, a flipped exchange sign or the wrong
    middle frequency is off by far more."""
    E, vxc = Fraction(1, 4), Fraction(1, 8)
    h = Fraction(1, 1024)
    e_n = [Fraction(-2), Fraction(-3, 4), Fraction(3, 2), Fraction(5, 2)]
    prob, xs = _problem(E, h, e_n)
    ach, asx, _, _ = oracle.sigma_fwd(prob, nthreads=1)
    q = oracle.quasiparticle(ach, asx, float(h), energy=float(E), vxc=float(vxc))
    exact = _Q(0)
    sig_mid = _Q(0)
    for n in range(NB):
        x = _Q(E - e_n[n])
        exact = exact + _exact_dsigma(x, n)
        ch, sx = _exact_sigma(x, n)
        sig_mid = sig_mid + ch + _Q(-1) * sx
    assert abs(q["dsigma"] - exact.c()) <= 1e-5 * abs(exact.c())
    z = 1.0 / (1.0 - exact.c().real)
    assert abs(q["z"] - z) <= 1e-5 * abs(z) * abs(exact.c()) / abs(1.0 - exact.c().real) + 1e-12
    e_qp = float(E) + z * (sig_mid.c().real - float(vxc))
    assert math.isclose(q["e_qp"], e_qp, rel_tol=1e-4)
