"""Pins of the oracle's analytic gradients against central finite
differences (h = 1e-6) of its forward.

Loss L = sum_w Re(conj(ga[w]) achtemp[w] + conj(gs[w]) asxtemp[w]); the
gradient of a complex input z is dL/dRe z + i dL/dIm z.  The slice-restricted
loss keeps only the terms that touch the perturbed entry, so the difference
quotient does not cancel against the whole sum; stencils that move any
touched term across a branch boundary are skipped and counted.
"""
import numpy as np
import pytest

import oracle
from paper_2008_11326_amd.inputs import Dims, make_fd_entries, make_problem, \
    make_upstream_grad

H = 1e-6
ARRAYS = ("wtilde_array", "I_eps_array", "aqsntemp", "aqsmtemp")


def _problem():
    prob = make_problem(Dims(6, 2, 24, 5, 3), 21, pole_fraction=0.2)
    rng = np.random.default_rng(12)
    ga, gs = make_upstream_grad(3, rng)
    return prob, ga, gs, rng


def _entry_value(prob, array, i, j):
    return getattr(prob, array)[i, j]


@pytest.mark.parametrize("array", ARRAYS)
def test_grad_matches_slice_fd(array):
    prob, ga, gs, rng = _problem()
    entries = make_fd_entries(prob.dims, rng, count=40)[array]
    grads = oracle.grad_entries(prob, ga, gs, array, entries, nthreads=2)
    checked = skipped = 0
    for (i, j), gr in zip(entries, grads):
        z0 = _entry_value(prob, array, i, j)
        fd = []
        straddle = False
        _, b0 = oracle.slice_loss(prob, ga, gs, array, i, j, z0)
        for step in (H, 1j * H):
            lp, bp = oracle.slice_loss(prob, ga, gs, array, i, j, z0 + step)
            lm, bm = oracle.slice_loss(prob, ga, gs, array, i, j, z0 - step)
            straddle |= not (np.array_equal(bp, b0) and np.array_equal(bm, b0))
            fd.append((lp - lm) / (2 * H))
        if straddle:
            skipped += 1
            continue
        checked += 1
        fdz = complex(fd[0], fd[1])
        assert abs(fdz - gr) <= 1e-7 * max(abs(gr), 1e-3), (array, i, j, gr, fdz)
    assert checked >= 30 and skipped <= 10


def _full_loss(prob, ga, gs):
    ach, asx, _, _ = oracle.sigma_fwd(prob, nthreads=1)
    return float(np.sum((np.conj(ga) * ach + np.conj(gs) * asx).real))


@pytest.mark.parametrize("array", ARRAYS)
def test_grad_matches_full_loss_fd(array):
    """Same check through the full forward (not the slice routine)."""
    prob, ga, gs, rng = _problem()
    entries = make_fd_entries(prob.dims, rng, count=6)[array]
    grads = oracle.grad_entries(prob, ga, gs, array, entries)
    for (i, j), gr in zip(entries, grads):
        arr = getattr(prob, array)
        z0 = arr[i, j]
        _, b0 = oracle.slice_loss(prob, ga, gs, array, i, j, z0)
        fd = []
        ok = True
        for step in (H, 1j * H):
            vals = []
            for sgn in (1, -1):
                arr[i, j] = z0 + sgn * step
                _, b = oracle.slice_loss(prob, ga, gs, array, i, j, z0 + sgn * step)
                ok &= np.array_equal(b, b0)
                vals.append(_full_loss(prob, ga, gs))
            arr[i, j] = z0
            fd.append((vals[0] - vals[1]) / (2 * H))
        if not ok:
            continue
        assert abs(complex(*fd) - gr) <= 1e-6 * max(abs(gr), 1e-2)


def test_aqsmtemp_columns_beyond_ngpown_have_zero_grad():
    prob, ga, gs, _ = _problem()
    npw, ng = prob.dims.ngpown, prob.dims.ncouls
    idx = np.array([[0, npw], [3, ng - 1]])
    assert np.all(oracle.grad_entries(prob, ga, gs, "aqsmtemp", idx) == 0)
