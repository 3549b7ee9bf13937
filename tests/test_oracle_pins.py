"""Pins of the CPU oracle against things other than itself.

* hand-derived single-term values (tests/golden/single_terms.json);
* a long-double brute force that evaluates the terms in their delw form;
* single-pole closed forms (uniform arrays, the sum collapses to a short
  sum over bands evaluated in exact rationals);
* the pole-cancellation identity between the A and B formulas;
* index and linearity invariants that a transposed operand, a dropped
  conjugate or a wrong index would break.

Loop nest and reductions: paper Sec. II-A; branch: Sec. III v2/v3.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2008_11326_amd.inputs import Dims, Problem, make_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _single(case, nv=1):
    c = lambda v: np.array([[complex(v[0], v[1])]], dtype=np.complex128)
    return Problem(Dims(1, nv, 1, 1, 1), aqsmtemp=c(case["aqsmtemp"]),
                   aqsntemp=c(case["aqsntemp"]), I_eps_array=c(case["I_eps"]),
                   wtilde_array=c(case["wtilde"]),
                   vcoul=np.array([case["vcoul"]]),
                   wx_array=np.array([[case["x"]]]))


def _frac(pair):
    return float(Fraction(pair[0], pair[1]))


def _close(got, want_re, want_im, rtol=4e-16):
    scale = max(abs(want_re), abs(want_im), 1e-300)
    assert abs(got.real - want_re) <= rtol * scale + 1e-300, (got, want_re)
    assert abs(got.imag - want_im) <= rtol * scale + 1e-300, (got, want_im)


with open(os.path.join(GOLDEN, "single_terms.json")) as f:
    SINGLE = json.load(f)["cases"]


def _modulus(pair_re, pair_im):
    """|re + i im| of a complex value given as exact [num, den] pairs."""
    re, im = Fraction(*pair_re), Fraction(*pair_im)
    return math.sqrt(re * re + im * im)


@pytest.mark.parametrize("case", SINGLE, ids=[c["name"] for c in SINGLE])
def test_single_term_hand_values(case):
    prob = _single(case)
    ach, asx, ach_abs, asx_abs = oracle.sigma_fwd(prob, nthreads=1)
    _close(ach[0], _frac(case["achtemp"][0]), _frac(case["achtemp"][1]))
    _close(asx[0], _frac(case["asxtemp"][0]), _frac(case["asxtemp"][1]))
    # one term each: the sums of |term| are the moduli of the hand values
    want_ach = _modulus(*case["achtemp"])
    want_asx = _modulus(*case["asxtemp"])
    assert abs(ach_abs[0] - want_ach) <= 4e-16 * want_ach
    assert abs(asx_abs[0] - want_asx) <= 4e-16 * want_asx
    om = complex(*case["wtilde"])
    assert oracle.branch(case["x"], om) == case["branch"]
    # an unoccupied band contributes nothing to asxtemp
    ach2, asx2, _, _ = oracle.sigma_fwd(_single(case, nv=0), nthreads=1)
    assert ach2[0] == ach[0] and asx2[0] == 0


def test_branch_neighbours_of_ties():
    # one ulp above |x-om|^2 = 1/4 enters A; the tie itself is B
    om = 1.0 + 0j
    assert oracle.branch(1.5, om) == 1
    assert oracle.branch(np.nextafter(1.5, 2.0), om) == 0
    # |om|^2 = 250000 |d|^2 tie is B, moving x away by one ulp enters A
    assert oracle.branch(499.0, 500.0 + 0j) == 1
    assert oracle.branch(np.nextafter(499.0, 0.0), 500.0 + 0j) == 0
    # om = 0 with |d| > 1/2 is A (value 0), not B or C
    assert oracle.branch(1.0, 0j) == 0
    # exact pole: B;  tiny om far from x: C
    assert oracle.branch(0.7, 0.7 + 0j) == 1
    assert oracle.branch(0.25 + 2.0 ** -24, 2.0 ** -24 + 0j) == 2


def _tiny(seed, nb=5, nv=2, ng=23, npw=7, nw=3, poles=0.0):
    return make_problem(Dims(nb, nv, ng, npw, nw), seed, poles)


@pytest.mark.parametrize("seed", range(6))
def test_matches_long_double_brute_force(seed):
    prob = _tiny(seed, poles=0.2 if seed % 2 else 0.0)
    ach, asx, ach_abs, asx_abs = oracle.sigma_fwd(prob, nthreads=1)
    ach_ld, asx_ld = oracle.sigma_ld(prob)
    for got, ref, s in ((ach, ach_ld, ach_abs), (asx, asx_ld, asx_abs)):
        err = np.abs(got - ref)
        assert np.all(err <= 1e-13 * np.abs(ref) + 1e-15 * s), (got, ref)


def test_long_double_near_poles_and_all_occupied():
    # every band occupied, 30 % of wtilde planted within 1e-6 of a wx value
    prob = _tiny(11, nb=4, nv=4, ng=17, npw=5, poles=0.3)
    ach, asx, ach_abs, asx_abs = oracle.sigma_fwd(prob, nthreads=1)
    ach_ld, asx_ld = oracle.sigma_ld(prob)
    assert np.all(np.abs(ach - ach_ld) <= 1e-13 * np.abs(ach_ld) + 1e-15 * ach_abs)
    assert np.all(np.abs(asx - asx_ld) <= 1e-13 * np.abs(asx_ld) + 1e-15 * asx_abs)


def _uniform_problem(nb, nv, ng, npw, xs, om, e, a, b, v):
    nw = len(xs[0])
    return Problem(
        Dims(nb, nv, ng, npw, nw),
        aqsmtemp=np.full((nb, ng), b, np.complex128),
        aqsntemp=np.full((nb, ng), a, np.complex128),
        I_eps_array=np.full((npw, ng), e, np.complex128),
        wtilde_array=np.full((npw, ng), om, np.complex128),
        vcoul=np.full(ng, v),
        wx_array=np.ascontiguousarray(np.array(xs, dtype=np.float64).T))


class _Q:
    """Exact complex rationals for closed forms."""

    def __init__(self, re, im=0):
        self.re, self.im = Fraction(re), Fraction(im)

    def __add__(self, o):
        return _Q(self.re + o.re, self.im + o.im)

    def __mul__(self, o):
        return _Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def inv(self):
        d = self.re * self.re + self.im * self.im
        return _Q(self.re / d, -self.im / d)

    def conj(self):
        return _Q(self.re, -self.im)

    def c(self):
        return complex(float(self.re), float(self.im))


def test_single_pole_closed_form():
    """Uniform arrays: every (p, g) is the same term, so
    achtemp[w] = NP NG v/2 a conj(b) e sum_n [A] om/(x_nw - om) and
    asxtemp[w] = NP NG v a conj(b) e sum_{n<NV} ssx_n/e  (B bands: -om/(2(x+om)))."""
    om = _Q(Fraction(5, 4), Fraction(1, 16))
    e, a, b, v = _Q(Fraction(1, 2), Fraction(-1, 4)), _Q(1, Fraction(1, 2)), \
        _Q(Fraction(-1, 4), Fraction(3, 4)), Fraction(3, 8)
    # bands: 0 -> A at every w, 1 -> B at every w, 2..5 -> A
    xs = [[-1.0, -0.75, -0.5], [1.25, 1.375, 1.5], [2.5, 3.0, 4.0],
          [-2.0, -1.5, 0.0], [0.5, 0.25, -0.25], [3.5, 2.0, 2.25]]
    nb, nv, ng, npw = len(xs), 2, 300, 40
    prob = _uniform_problem(nb, nv, ng, npw, xs, om.c(), e.c(), a.c(), b.c(),
                            float(v))
    ach, asx, ach_abs, asx_abs = oracle.sigma_fwd(prob, nthreads=3)
    pref = _Q(npw * ng) * a * b.conj() * e
    unit = a * b.conj() * e
    want_abs = [[0.0] * 3, [0.0] * 3]
    for w in range(3):
        for n in range(nb):
            x = _Q(Fraction(xs[n][w]))
            d = x + _Q(-om.re, -om.im)
            s = x + om
            if d.re ** 2 + d.im ** 2 > Fraction(1, 4):
                tch = unit * _Q(v / 2) * om * d.inv()
                tsx = unit * _Q(v) * om * om * (d * s).inv()
            else:
                tch = _Q(0)
                tsx = unit * _Q(v) * _Q(Fraction(-1, 2)) * om * s.inv()
            want_abs[0][w] += npw * ng * _abs_q(tch)
            if n < nv:
                want_abs[1][w] += npw * ng * _abs_q(tsx)
    for w in range(3):
        s_ch, s_sx = _Q(0), _Q(0)
        for n in range(nb):
            x = _Q(Fraction(xs[n][w]))
            d = x + _Q(-om.re, -om.im)
            s = x + om
            isA = (d.re ** 2 + d.im ** 2 > Fraction(1, 4))
            assert isA == (n != 1)
            if isA:
                s_ch = s_ch + om * d.inv()
                if n < nv:
                    s_sx = s_sx + om * om * (d * s).inv()
            elif n < nv:
                s_sx = s_sx + _Q(Fraction(-1, 2)) * om * s.inv()
        want_ch = (pref * _Q(v / 2) * s_ch).c()
        want_sx = (pref * _Q(v) * s_sx).c()
        assert abs(ach[w] - want_ch) <= 1e-14 * abs(want_ch)
        assert abs(asx[w] - want_sx) <= 1e-14 * abs(want_sx)
        # every (p, g) repeats the same term, so the sums of |term| are
        # NP NG sum_n |term_n|, each modulus from its exact square
        assert abs(ach_abs[w] - want_abs[0][w]) <= 1e-14 * want_abs[0][w]
        assert abs(asx_abs[w] - want_abs[1][w]) <= 1e-14 * want_abs[1][w]


def _abs_q(z):
    return math.sqrt(z.re * z.re + z.im * z.im)


def test_abs_sums_of_cancelling_bands():
    """Two bands with opposite aqsntemp rows and equal frequencies cancel
    term by term: the outputs vanish while the sums of |term| are
    2 NP NG sum_w-wise |term|, which a dropped 1/2, a squared modulus or a
    signed sum would change."""
    om = _Q(Fraction(3, 2), Fraction(1, 8))
    e, a, b, v = _Q(Fraction(3, 4), Fraction(1, 2)), _Q(Fraction(5, 4), Fraction(-1, 2)), \
        _Q(Fraction(1, 2), Fraction(1, 4)), Fraction(5, 8)
    xs = [[-1.0, 3.5], [-1.0, 3.5]]          # both bands: A at both frequencies
    nb, nv, ng, npw = 2, 2, 7, 3
    prob = _uniform_problem(nb, nv, ng, npw, xs, om.c(), e.c(), a.c(), b.c(),
                            float(v))
    prob.aqsntemp[1] = -prob.aqsntemp[0]
    ach, asx, ach_abs, asx_abs = oracle.sigma_fwd(prob, nthreads=1)
    unit = a * b.conj() * e
    for w in range(2):
        x = _Q(Fraction(xs[0][w]))
        d = x + _Q(-om.re, -om.im)
        s = x + om
        t_ch = _abs_q(unit * _Q(v / 2) * om * d.inv())
        t_sx = _abs_q(unit * _Q(v) * om * om * (d * s).inv())
        assert abs(ach_abs[w] - 2 * npw * ng * t_ch) <= 1e-15 * 2 * npw * ng * t_ch
        assert abs(asx_abs[w] - 2 * npw * ng * t_sx) <= 1e-15 * 2 * npw * ng * t_sx
        assert abs(ach[w]) <= 1e-15 * ach_abs[w]
        assert abs(asx[w]) <= 1e-15 * asx_abs[w]


def test_pole_cancellation_identity():
    """With every band occupied, sch/2 - ssx = e om / (2 (x + om)) for both A
    and B terms, so achtemp - asxtemp equals a branch-free sum over non-C
    terms (here no C terms occur)."""
    prob = _tiny(7, nb=6, nv=6, ng=40, npw=9, poles=0.25)
    ach, asx, ach_abs, _ = oracle.sigma_fwd(prob, nthreads=1)
    x = prob.wx_array[:, :, None, None]                    # [w, n, 1, 1]
    om = prob.wtilde_array[None, None]                     # [1, 1, p, g]
    e = prob.I_eps_array[None, None]
    M = prob.aqsntemp[:, None, :] * np.conj(prob.aqsmtemp[:, :9, None])  # [n,p,g]
    t = prob.vcoul * M[None] * e * om / (2 * (x + om))
    want = t.reshape(t.shape[0], -1).sum(axis=1)
    assert np.all(np.abs((ach - asx) - want) <= 1e-13 * ach_abs)


def test_sesquilinear_and_linear():
    prob = _tiny(3)
    ach, asx, s1, s2 = oracle.sigma_fwd(prob, nthreads=1)
    c = 0.75 - 1.25j
    for name, factor in (("aqsntemp", c), ("aqsmtemp", np.conj(c)),
                         ("I_eps_array", c), ("vcoul", 2.5)):
        q = make_problem(prob.dims, 3)
        setattr(q, name, getattr(q, name) * (factor if name != "aqsmtemp" else c))
        a2, x2, _, _ = oracle.sigma_fwd(q, nthreads=1)
        assert np.all(np.abs(a2 - factor * ach) <= 1e-14 * abs(factor) * s1)
        assert np.all(np.abs(x2 - factor * asx) <= 1e-14 * abs(factor) * s2)


def test_permutations_of_g_and_p():
    prob = _tiny(5, ng=31, npw=6)
    ach, asx, s1, s2 = oracle.sigma_fwd(prob, nthreads=1)
    rng = np.random.default_rng(99)
    pg = rng.permutation(prob.dims.ncouls)
    q = make_problem(prob.dims, 5)
    # rows G: permute every array indexed by g (aqsmtemp is indexed by G')
    q.aqsntemp = q.aqsntemp[:, pg].copy()
    q.I_eps_array = q.I_eps_array[:, pg].copy()
    q.wtilde_array = q.wtilde_array[:, pg].copy()
    q.vcoul = q.vcoul[pg].copy()
    a2, x2, _, _ = oracle.sigma_fwd(q, nthreads=1)
    assert np.all(np.abs(a2 - ach) <= 1e-14 * s1)
    assert np.all(np.abs(x2 - asx) <= 1e-14 * s2)
    # columns G': rows of wtilde/I_eps together with columns p < ngpown of aqsmtemp
    pp = rng.permutation(prob.dims.ngpown)
    q = make_problem(prob.dims, 5)
    q.I_eps_array = q.I_eps_array[pp].copy()
    q.wtilde_array = q.wtilde_array[pp].copy()
    head = q.aqsmtemp[:, :prob.dims.ngpown][:, pp]
    q.aqsmtemp = q.aqsmtemp.copy()
    q.aqsmtemp[:, :prob.dims.ngpown] = head
    a3, x3, _, _ = oracle.sigma_fwd(q, nthreads=1)
    assert np.all(np.abs(a3 - ach) <= 1e-14 * s1)
    assert np.all(np.abs(x3 - asx) <= 1e-14 * s2)
    # permuting g in aqsmtemp alone must change the result (it is indexed by G')
    q = make_problem(prob.dims, 5)
    q.aqsmtemp = q.aqsmtemp[:, pg].copy()
    a4, _, _, _ = oracle.sigma_fwd(q, nthreads=1)
    assert np.max(np.abs(a4 - ach)) > 1e-6 * np.max(s1)


def test_slices_add_up_and_threads_agree():
    prob = _tiny(8, nb=6, ng=50, npw=11)
    full = oracle.sigma_fwd(prob, nthreads=1)
    parts = [oracle.sigma_fwd_slice(prob, p=(a, b), nthreads=1)
             for a, b in ((0, 4), (4, 5), (5, 11))]
    gparts = [oracle.sigma_fwd_slice(prob, g=(a, b), nthreads=1)
              for a, b in ((0, 17), (17, 50))]
    nparts = [oracle.sigma_fwd_slice(prob, n=(a, b), nthreads=1)
              for a, b in ((0, 1), (1, 3), (3, 6))]
    for split in (parts, gparts, nparts):
        for k in (0, 1):
            tot = sum(s[k] for s in split)
            assert np.all(np.abs(tot - full[k]) <= 1e-14 * full[2 + k])
    for T in (2, 3, 7):
        r = oracle.sigma_fwd(prob, nthreads=T)
        assert np.all(np.abs(r[0] - full[0]) <= 1e-15 * full[2])


def test_real_inputs_give_real_outputs():
    prob = _tiny(9)
    for name in ("aqsmtemp", "aqsntemp", "I_eps_array", "wtilde_array"):
        arr = getattr(prob, name)
        setattr(prob, name, arr.real.astype(np.complex128))
    ach, asx, _, _ = oracle.sigma_fwd(prob, nthreads=1)
    assert np.all(ach.imag == 0) and np.all(asx.imag == 0)


def test_empty_and_degenerate_sizes():
    for dims in (Dims(0, 0, 8, 4, 3), Dims(4, 0, 8, 4, 3), Dims(4, 4, 8, 4, 1),
                 Dims(3, 1, 5, 0, 2), Dims(2, 1, 0, 0, 2)):
        prob = make_problem(dims, 1)
        ach, asx, _, _ = oracle.sigma_fwd(prob, nthreads=2)
        if dims.number_bands == 0 or dims.ngpown == 0:
            assert np.all(ach == 0)
        if dims.nvband == 0 or dims.ngpown == 0:
            assert np.all(asx == 0)
    with pytest.raises(ValueError):
        oracle.sigma_fwd(make_problem(Dims(2, 3, 4, 4, 1), 0))
