"""The calibration kernels behind the measured ceilings and the counter
scaling (include/gpp_microbench.h): the streaming copy must move every byte
it claims (FETCH_SIZE / WRITE_SIZE are scaled by what they read for it),
the read kernel must read the window it is given, the FMA kernel must
run the chains it counts, and the LDS pattern kernel must touch the entries
it states.  Each is checked against values computed on the
host."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2008_11326_amd import _lib
    return _lib.load()


def test_copy_moves_every_byte(lib):
    import torch
    nbytes = 256 << 20
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda:0", generator=g)
    dst = torch.zeros(nbytes + 4096, dtype=torch.uint8, device="cuda:0")
    say(f"[mb] copy of {nbytes >> 20} MiB")
    assert lib.gpp_mb_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                           256 * 8, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].count_nonzero()) == 0  # nothing beyond the copy
    # a byte count that leaves a partial last round of the grid
    odd = (nbytes // 3) // 16 * 16
    dst.zero_()
    assert lib.gpp_mb_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), odd,
                           1000, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(dst[:odd], src[:odd]) and int(dst[odd:].count_nonzero()) == 0


def _read_reference(vals, win, shared, blocks, reps):
    """Per-lane sums of mb_read's walk, computed on the host: workgroup b,
    lane t reads elements t, t + 256, ... of its window (from a start
    rotated by 4096 b elements when the window is shared), reps times, and
    adds re + im.  Values are small integers, so every sum is exact."""
    out = np.zeros(blocks * 256)
    per = vals.real + vals.imag
    for b in range(blocks):
        base = 0 if shared else b * win
        start = (b * 4096) % win if shared else 0
        for t in range(256):
            idx = (start + np.arange(t, win, 256)) % win
            out[b * 256 + t] = reps * per[base + idx].sum()
    return out


@pytest.mark.parametrize("shared", [0, 1])
def test_read_reads_its_window(lib, shared):
    import torch
    win, blocks, reps = 3000, 5, 3   # 3000 elements: whole 1024-element steps and a tail
    nelem = win if shared else win * blocks
    rng = np.random.default_rng(3 + shared)
    vals = (rng.integers(-50, 50, nelem) + 1j * rng.integers(-50, 50, nelem)).astype(np.complex128)
    buf = torch.from_numpy(vals).to("cuda:0")
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda:0")
    assert lib.gpp_mb_read(C.c_void_p(buf.data_ptr()), win * 16, shared, blocks, reps,
                           C.c_void_p(out.data_ptr()), None) == 0
    torch.cuda.synchronize()
    want = _read_reference(vals, win, shared, blocks, reps)
    assert np.array_equal(out.cpu().numpy(), want)


def test_fma_chains_closed_form(lib):
    """Each lane runs 16 chains a <- a c + d from a0 = 1.5 + 1e-3 t + k; after
    n rounds a = c^n a0 + d (1 - c^n)/(1 - c), and the lane writes the sum
    of its chains.  The flop count is 2 x 16 x n per lane."""
    import torch
    blocks, iters = 7, 64
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda:0")
    flops = C.c_double(0.0)
    assert lib.gpp_mb_fp64_fma(C.c_void_p(out.data_ptr()), blocks, iters, None,
                               C.byref(flops)) == 0
    torch.cuda.synchronize()
    assert flops.value == 2.0 * 16 * iters * 256 * blocks
    c, d = 0.9999999, 1e-9
    cn = c ** iters
    t = np.arange(256, dtype=np.float64)
    a0 = 1.5 + 1e-3 * t[:, None] + np.arange(16, dtype=np.float64)[None, :]
    want = (cn * a0 + d * (1.0 - cn) / (1.0 - c)).sum(axis=1)
    got = out.cpu().numpy().reshape(blocks, 256)
    for b in range(blocks):
        assert np.allclose(got[b], want, rtol=1e-13, atol=0.0)


def _lds_reference(pattern, blocks, reps):
    """mb_lds's per-lane result, computed on the host (include/gpp_microbench.h)."""
    lane = np.arange(64)
    tj, tk = lane // 8, lane % 8
    c = np.arange(8)
    if pattern == 0:
        one = 64 * (8 * (reps - 1) + lane % 8) + 63 - lane
    else:
        if pattern == 1:
            e = 8 * tk[:, None] + (c[None, :] + tk[:, None] + tj[:, None]) % 8
        elif pattern == 2:
            e = tk[:, None] + 8 * ((c[None, :] + tj[:, None]) % 8)
        else:
            e = 8 * tk[:, None] + c[None, :]
        one = reps * ((64 * tj[:, None] + e) + 1).sum(axis=1)
    return np.tile(one.astype(np.float64), blocks)


@pytest.mark.parametrize("pattern", [0, 1, 2, 3])
def test_lds_patterns_read_and_write_what_they_claim(lib, pattern):
    """The LDS pattern kernel behind the bank-conflict measurements touches
    exactly the entries its header states (sums of small integers, exact)."""
    import torch
    blocks, reps = 3, 9
    out = torch.empty(blocks * 64, dtype=torch.float64, device="cuda:0")
    say(f"[mb] lds pattern {pattern}")
    assert lib.gpp_mb_lds(pattern, blocks, reps, C.c_void_p(out.data_ptr()), None) == 0
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), _lds_reference(pattern, blocks, reps))
