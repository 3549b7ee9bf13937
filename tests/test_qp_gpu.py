"""GPU parity of the quasiparticle epilogue (gpp_sigma_qp): Sigma(E),
dSigma/dE, Z and E_qp computed in the forward's last reduction kernel,
against the oracle's quasiparticle step (oracle/qp.py) applied to the
oracle's forward outputs.  The bar on each quantity is the per-output
1e-12 parity bar propagated through the step (gpu_helpers.qp_bounds).  The
full-size workload is checked in test_fwd_gpu.py::test_full_size_against_golden."""
import numpy as np
import pytest

import oracle
from paper_2008_11326_amd import inputs as I
from tests.gpu_helpers import assert_parity, qp_bounds, qp_vector, say, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpp():
    import paper_2008_11326_amd as gpp
    from paper_2008_11326_amd import _lib
    _lib.load()
    return gpp


def run_qp(gpp, prob, vxc):
    import torch
    d = to_device(prob)
    ach, asx, qp = gpp.sigma_qp(**d, nvband=prob.dims.nvband, freq_step=prob.freq_step,
                                energy=prob.e_lk, vxc=vxc)
    fa, fs = gpp.sigma_fwd(**d, nvband=prob.dims.nvband)
    torch.cuda.synchronize()
    return ach.cpu().numpy(), asx.cpu().numpy(), qp.cpu().numpy(), fa.cpu().numpy(), fs.cpu().numpy()


@pytest.mark.parametrize("shape,poles,vxc", [
    ((32, 2, 512, 64, 3), 0.0, -0.3),      # the small workload's sizes
    ((20, 2, 300, 7, 3), 0.1, 0.0),
    ((17, 3, 200, 9, 5), 0.05, 0.7),
    ((9, 9, 130, 5, 7), 0.0, 1.25),
])
def test_qp_against_oracle(gpp, shape, poles, vxc):
    prob = I.make_problem(I.Dims(*shape), sum(shape) + 5, poles)
    say(f"[qp] {shape} poles={poles}")
    ach, asx, qp, fa, fs = run_qp(gpp, prob, vxc)
    # the forward part is the plain forward, bit for bit
    assert np.array_equal(ach, fa) and np.array_equal(asx, fs)
    ra, rs, sa, ss = oracle.sigma_fwd(prob)
    assert_parity(ach, ra, sa, "achtemp")
    assert_parity(asx, rs, ss, "asxtemp")
    q = oracle.quasiparticle(ra, rs, prob.freq_step, energy=prob.e_lk, vxc=vxc)
    want = qp_vector(q)
    tol = qp_bounds(ra, rs, sa, ss, prob.freq_step, vxc, q["z"], q["sigma"])
    err = np.abs(qp - want)
    assert np.all(err <= tol), (qp, want, err, tol)
    # the epilogue's own arithmetic on the kernel's sums
    own = qp_vector(oracle.quasiparticle(ach, asx, prob.freq_step, energy=prob.e_lk, vxc=vxc))
    assert np.allclose(qp, own, rtol=1e-14, atol=1e-14 * np.max(np.abs(own)))


def test_qp_of_an_empty_sum(gpp):
    prob = I.make_problem(I.Dims(0, 0, 64, 4, 3), 1)
    ach, asx, qp, _, _ = run_qp(gpp, prob, 0.4)
    assert np.all(ach == 0) and np.all(asx == 0)
    assert np.array_equal(qp, np.array([0.0, 0.0, 0.0, 0.0, 1.0, prob.e_lk - 0.4]))


def test_qp_rejects_even_frequency_counts(gpp):
    from paper_2008_11326_amd import GppError
    prob = I.make_problem(I.Dims(4, 1, 64, 4, 4), 1)
    with pytest.raises(GppError, match="odd"):
        run_qp(gpp, prob, 0.0)
