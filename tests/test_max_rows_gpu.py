"""The forward and the adjoint at the largest sizes along one axis: the
boundary's largest row count (GPP_MAX_NCOULS = 2^26 G rows; the kernels
address a row with 32-bit byte offsets, which reach 2^30 bytes there), with
two bands (one occupied), one G' column, three frequencies and 0.1 %
planted near-poles; and 2^20 bands (2048 band chunks of the forward's
tiles, 2^18 band tiles of the adjoint, band offsets of 2^30 bytes) with 64
rows and two G' columns.  The sizes along the other axes keep the oracle's
work to seconds; every output, and sampled gradient entries that include
the last rows and bands, are checked against it."""
import numpy as np
import pytest

import oracle
from paper_2008_11326_amd import _lib
from paper_2008_11326_amd import inputs as I
from tests.gpu_helpers import assert_parity, say, to_device
from tests.test_bwd_gpu import check_entries, gpu_grads

pytestmark = pytest.mark.gpu

NG = 1 << 26


@pytest.fixture(scope="module")
def gpp():
    import paper_2008_11326_amd as gpp
    _lib.load()
    return gpp


@pytest.fixture(scope="module")
def prob():
    import ctypes as C
    lib = _lib.load()
    d = I.Dims(2, 1, NG, 1, 3)
    assert lib.gpp_sigma_fwd_workspace(C.byref(_lib.dims_struct(*d.as_tuple()))) > 0
    assert lib.gpp_sigma_fwd_workspace(C.byref(_lib.dims_struct(2, 1, NG + 1, 1, 3))) == 0
    say(f"[max rows] generating {d}")
    return I.make_problem(d, 26, 0.001)


def test_forward_at_the_largest_row_count(gpp, prob):
    import torch
    say(f"[max rows] forward {prob.dims}")
    dev = to_device(prob)
    ach, asx = gpp.sigma_fwd(**dev, nvband=prob.dims.nvband)
    torch.cuda.synchronize()
    del dev
    torch.cuda.empty_cache()
    ref = oracle.sigma_fwd(prob)
    assert_parity(ach.cpu().numpy(), ref[0], ref[2], "max rows achtemp")
    assert_parity(asx.cpu().numpy(), ref[1], ref[3], "max rows asxtemp")


def test_adjoint_at_the_largest_row_count(gpp, prob):
    import torch
    say(f"[max rows] adjoint {prob.dims}")
    ga, gs = I.make_upstream_grad(prob.dims.nfreq, np.random.default_rng(26))
    g = gpu_grads(gpp, prob, ga, gs)
    torch.cuda.empty_cache()
    rows = np.random.default_rng(27).integers(0, NG, 60)
    last = [NG - 1, NG - 2, NG - 64, NG // 2]
    g_idx = np.concatenate([rows, last])
    an_idx = np.array([(n, j) for n in (0, 1) for j in g_idx], dtype=np.int64)
    pg_idx = np.array([(0, j) for j in g_idx], dtype=np.int64)
    check_entries("aqsntemp", g["aqsntemp"], prob, ga, gs, an_idx)
    check_entries("I_eps_array", g["I_eps_array"], prob, ga, gs, pg_idx)
    check_entries("wtilde_array", g["wtilde_array"], prob, ga, gs, pg_idx)
    check_entries("aqsmtemp", g["aqsmtemp"], prob, ga, gs,
                  np.array([(0, 0), (1, 0)], dtype=np.int64))
    assert np.all(g["aqsmtemp"][:, 1:] == 0)


NB_MANY = 1 << 20


@pytest.fixture(scope="module")
def many_bands():
    d = I.Dims(NB_MANY, 3, 64, 2, 3)
    say(f"[max bands] generating {d}")
    return I.make_problem(d, 20, 0.01)


def test_forward_with_a_million_bands(gpp, many_bands):
    import torch
    prob = many_bands
    say(f"[max bands] forward {prob.dims}")
    dev = to_device(prob)
    ach, asx = gpp.sigma_fwd(**dev, nvband=prob.dims.nvband)
    torch.cuda.synchronize()
    del dev
    torch.cuda.empty_cache()
    ref = oracle.sigma_fwd(prob)
    assert_parity(ach.cpu().numpy(), ref[0], ref[2], "max bands achtemp")
    assert_parity(asx.cpu().numpy(), ref[1], ref[3], "max bands asxtemp")


def test_adjoint_with_a_million_bands(gpp, many_bands):
    import torch
    prob = many_bands
    say(f"[max bands] adjoint {prob.dims}")
    ga, gs = I.make_upstream_grad(prob.dims.nfreq, np.random.default_rng(20))
    g = gpu_grads(gpp, prob, ga, gs)
    torch.cuda.empty_cache()
    rng = np.random.default_rng(21)
    bands = np.concatenate([rng.integers(0, NB_MANY, 40), [0, 1, 2, NB_MANY - 1, NB_MANY - 2]])
    rows = rng.integers(0, 64, bands.size)
    rows[-2:] = 63
    nm_idx = np.stack([bands, rows], axis=1).astype(np.int64)
    check_entries("aqsntemp", g["aqsntemp"], prob, ga, gs, nm_idx)
    am_idx = np.stack([bands, rng.integers(0, 2, bands.size)], axis=1).astype(np.int64)
    check_entries("aqsmtemp", g["aqsmtemp"], prob, ga, gs, am_idx)
    pg_idx = np.array([(p, r) for p in (0, 1) for r in (0, 17, 63)], dtype=np.int64)
    check_entries("I_eps_array", g["I_eps_array"], prob, ga, gs, pg_idx)
    check_entries("wtilde_array", g["wtilde_array"], prob, ga, gs, pg_idx)
    assert np.all(g["aqsmtemp"][:, 2:] == 0)
