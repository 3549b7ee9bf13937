"""gpp_sigma_fwd_noalloc (the forward with its workspace in a fixed device
array inside the library, for callers that cannot allocate) against
gpp_sigma_fwd with a caller workspace, both called through the C ABI: two
calls in a row, the second on smaller inputs, so the second reuses the
array the first filled.  Results must match bit for bit (same kernels,
same partial layout) and the oracle at the 1e-12 parity bar; sizes beyond
the array are refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2008_11326_amd import inputs as I
from tests.gpu_helpers import assert_parity, say, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2008_11326_amd import _lib
    return _lib.load()


def _abi_args(prob, dev):
    from paper_2008_11326_amd import _lib
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t.numel() else C.c_void_p(0)
    dims = _lib.dims_struct(*prob.dims.as_tuple())
    ins = _lib.GppInputs(*[ptr(dev[k]) for k in ("aqsmtemp", "aqsntemp", "I_eps_array",
                                                  "wtilde_array", "vcoul", "wx_array")])
    return dims, ins, ptr


def _both(lib, prob):
    import torch
    dev = to_device(prob)
    dims, ins, ptr = _abi_args(prob, dev)
    nw = prob.dims.nfreq
    out = [torch.full((nw,), complex(7, 7), dtype=torch.complex128, device="cuda:0")
           for _ in range(4)]
    ws = torch.empty(max(lib.gpp_sigma_fwd_workspace(C.byref(dims)), 1), dtype=torch.uint8,
                     device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    assert lib.gpp_sigma_fwd(C.byref(dims), C.byref(ins), ptr(out[0]), ptr(out[1]), ptr(ws),
                             ws.numel(), C.c_void_p(st)) == 0
    rc = lib.gpp_sigma_fwd_noalloc(C.byref(dims), C.byref(ins), ptr(out[2]), ptr(out[3]),
                                   C.c_void_p(st))
    assert rc == 0, lib.gpp_last_error().decode()
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def test_noalloc_matches_the_workspace_form_twice(lib):
    big = I.make_problem(I.Dims(96, 3, 3000, 150, 3), 61, 0.02)
    small = I.make_problem(I.Dims(20, 2, 333, 17, 3), 62, 0.05)
    for what, prob in (("first call", big), ("second, smaller call", small)):
        say(f"[noalloc] {what}: {prob.dims}")
        ach, asx, na, nx = _both(lib, prob)
        assert np.array_equal(na, ach) and np.array_equal(nx, asx), (what, na, ach)
        ref = oracle.sigma_fwd(prob)
        assert_parity(na, ref[0], ref[2], what + " achtemp")
        assert_parity(nx, ref[1], ref[3], what + " asxtemp")


def test_noalloc_other_frequency_counts_and_empty(lib):
    for k, dims in enumerate((I.Dims(10, 2, 200, 9, 5), I.Dims(12, 1, 130, 6, 1),
                              I.Dims(0, 0, 64, 4, 3))):
        prob = I.make_problem(dims, 70 + k)
        say(f"[noalloc] {dims}")
        ach, asx, na, nx = _both(lib, prob)
        assert np.array_equal(na, ach) and np.array_equal(nx, asx)


def test_noalloc_refuses_sizes_beyond_the_array(lib):
    from paper_2008_11326_amd import _lib
    d = _lib.dims_struct(1024, 4, 65536, 8192, 3)
    need = lib.gpp_sigma_fwd_workspace(C.byref(d))
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    fake = 0x7F0000000000
    ins = _lib.GppInputs(*[C.c_void_p(fake + k * 0x100000) for k in range(6)])
    rc = lib.gpp_sigma_fwd_noalloc(C.byref(d), C.byref(ins), C.c_void_p(fake + 0x600000),
                                   C.c_void_p(fake + 0x600100), None)
    assert rc == 4 and "scratch" in lib.gpp_last_error().decode()
    # the large workload fits
    d2 = _lib.dims_struct(1024, 4, 65536, 3276, 3)
    assert lib.gpp_sigma_fwd_workspace(C.byref(d2)) <= _lib.NOALLOC_SCRATCH_BYTES


def test_noalloc_python_binding(lib):
    import torch
    import paper_2008_11326_amd as gpp
    prob = I.make_problem(I.Dims(16, 2, 256, 12, 3), 80)
    dev = to_device(prob)
    out = (torch.empty(3, dtype=torch.complex128, device="cuda:0"),
           torch.empty(3, dtype=torch.complex128, device="cuda:0"))
    ach, asx = gpp.sigma_fwd_noalloc(**dev, nvband=2, out=out)
    fa, fs = gpp.sigma_fwd(**dev, nvband=2)
    torch.cuda.synchronize()
    assert torch.equal(ach, fa) and torch.equal(asx, fs)


def test_noalloc_under_graph_capture(lib):
    """The use the entry point is for: after one eager call, the same call
    captured into a graph on a side stream (nothing allocated inside the
    capture) and replayed three times, with unrelated eager work and a
    refill of the outputs between replays; every replay equals the eager
    result bit for bit, and that matches the oracle."""
    import torch
    prob = I.make_problem(I.Dims(40, 2, 700, 30, 3), 63, 0.03)
    dev = to_device(prob)
    dims, ins, ptr = _abi_args(prob, dev)
    nw = prob.dims.nfreq
    mk = lambda: torch.full((nw,), complex(7, 7), dtype=torch.complex128, device="cuda:0")
    eager, outs = [mk(), mk()], [mk(), mk()]
    st = torch.cuda.current_stream().cuda_stream
    assert lib.gpp_sigma_fwd_noalloc(C.byref(dims), C.byref(ins), ptr(eager[0]),
                                     ptr(eager[1]), C.c_void_p(st)) == 0
    torch.cuda.synchronize()
    ref = [e.cpu().numpy() for e in eager]
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    say("[noalloc] capture")
    with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
        rc = lib.gpp_sigma_fwd_noalloc(C.byref(dims), C.byref(ins), ptr(outs[0]),
                                       ptr(outs[1]), C.c_void_p(side.cuda_stream))
    assert rc == 0, lib.gpp_last_error().decode()
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
        junk.sum().item()
        for o in outs:
            o.fill_(complex(7, 7))
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip(outs, ref):
            assert np.array_equal(got.cpu().numpy(), want), f"replay {rep}"
    ra, rs, sa, ss = oracle.sigma_fwd(prob)
    assert_parity(ref[0], ra, sa, "captured noalloc achtemp")
    assert_parity(ref[1], rs, ss, "captured noalloc asxtemp")

