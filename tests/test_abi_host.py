"""Host-only checks of the C ABI: the library loads, exports every function
include/gpp.h declares, and rejects invalid arguments before any device
call (these tests never reach a kernel launch)."""
import ctypes as C
import os
import re

import pytest

from paper_2008_11326_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            text = open(os.path.join(INCLUDE, h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(gpp_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "gpp_sigma_fwd" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTED) == names


def test_status_strings(lib):
    for code, name in _lib.STATUS.items():
        assert lib.gpp_status_string(code).decode().startswith(name)
    assert lib.gpp_version() >= 100


def _dims(nb=8, nv=2, ng=100, npw=10, nw=3):
    return _lib.GppDims(nb, nv, ng, npw, nw)


# Fake, aligned device addresses: every case below fails validation first.
FAKE = 0x7F0000000000


def _inputs(**override):
    vals = dict(aqsmtemp=FAKE, aqsntemp=FAKE + 0x100000,
                I_eps_array=FAKE + 0x200000, wtilde_array=FAKE + 0x300000,
                vcoul=FAKE + 0x400000, wx_array=FAKE + 0x500000)
    vals.update(override)
    return _lib.GppInputs(*[C.c_void_p(vals[k]) for k, _ in _lib.GppInputs._fields_])


def _call(lib, dims, ins, ach=FAKE + 0x600000, asx=FAKE + 0x600100, ws=None,
          ws_bytes=None):
    need = lib.gpp_sigma_fwd_workspace(C.byref(dims))
    ws = FAKE + 0x700000 if ws is None else ws
    ws_bytes = need if ws_bytes is None else ws_bytes
    return lib.gpp_sigma_fwd(C.byref(dims), C.byref(ins), C.c_void_p(ach),
                             C.c_void_p(asx), C.c_void_p(ws), ws_bytes, None)


@pytest.mark.parametrize("dims,msg", [
    (_dims(nv=9), "nvband"),
    (_dims(npw=101), "ngpown"),
    (_dims(nw=0), "nfreq"),
    (_dims(nw=9), "nfreq"),
    (_dims(nb=-1), "negative"),
    (_dims(ng=1 << 31, npw=1), "ncouls"),
    (_dims(ng=(1 << 26) + 1, npw=1), "ncouls"),
    (_dims(nb=1 << 31), "number_bands"),
    (_dims(nb=(1 << 30) + 1, nv=0, ng=64, npw=1), "number_bands"),
    # passes the per-dimension bounds, but 2048 band chunks of 8192 two-column
    # tiles x 16384 g-tiles would need 2^36 workgroups
    (_dims(nb=1 << 20, nv=0, ng=1 << 20, npw=1 << 14), "too large for one launch"),
])
def test_invalid_dims(lib, dims, msg):
    assert _call(lib, dims, _inputs()) == 1
    assert msg in lib.gpp_last_error().decode()
    assert lib.gpp_sigma_fwd_workspace(C.byref(dims)) == 0


def test_largest_band_count_is_accepted(lib):
    # GPP_MAX_NBANDS = 2^30 bands: 2^21 chunks of 512 bands for one tile
    d = _dims(nb=1 << 30, nv=0, ng=64, npw=1)
    assert lib.gpp_sigma_fwd_workspace(C.byref(d)) > 0
    assert lib.gpp_sigma_bwd_workspace(C.byref(d)) > 0


def test_last_error_is_per_thread(lib):
    """gpp_last_error is thread-local: two threads that fail differently at
    the same time each read their own message, and the calling thread's
    message is untouched."""
    import threading
    assert _call(lib, _dims(nw=9), _inputs()) == 1
    mine = lib.gpp_last_error().decode()
    assert "nfreq" in mine
    gate = threading.Barrier(2)
    seen = {}

    def worker(key, dims):
        st = _call(lib, dims, _inputs())
        gate.wait()  # both threads have failed before either reads
        seen[key] = (st, lib.gpp_last_error().decode())

    ts = [threading.Thread(target=worker, args=("nv", _dims(nv=9))),
          threading.Thread(target=worker, args=("np", _dims(npw=101)))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert seen["nv"][0] == 1 and "nvband" in seen["nv"][1] and "ngpown" not in seen["nv"][1]
    assert seen["np"][0] == 1 and "ngpown" in seen["np"][1] and "nvband" not in seen["np"][1]
    assert lib.gpp_last_error().decode() == mine


def test_adjoint_grid_beyond_one_launch_is_refused(lib):
    # the bands kernel's grid: 8 row blocks x 2^28 four-band tiles = 2^31
    # workgroups; the forward's 2^27 fit
    d = _dims(nb=1 << 30, nv=0, ng=2048, npw=16)
    assert lib.gpp_sigma_fwd_workspace(C.byref(d)) > 0
    assert lib.gpp_sigma_bwd_workspace(C.byref(d)) == 0
    z = C.c_void_p(0)
    f = C.c_void_p(FAKE + 0x600000)
    assert lib.gpp_sigma_bwd(C.byref(d), C.byref(_inputs()), f, f, z, z, z, z,
                             C.c_void_p(FAKE + 0x700000), 1 << 40, None) == 1
    assert "too large for one launch" in lib.gpp_last_error().decode()


@pytest.mark.parametrize("field", [f for f, _ in _lib.GppInputs._fields_])
def test_null_and_misaligned_inputs(lib, field):
    assert _call(lib, _dims(), _inputs(**{field: 0})) == 1
    assert field in lib.gpp_last_error().decode()
    align = 16 if field not in ("vcoul", "wx_array") else 8
    assert _call(lib, _dims(), _inputs(**{field: FAKE + 0x800000 + align // 2})) == 1
    assert "aligned" in lib.gpp_last_error().decode()


def test_null_pointer_allowed_for_empty_array(lib):
    # nvband = 0 and ngpown = 0 are valid; with ngpown = 0 the G'-indexed
    # arrays may be NULL -- but the workspace check below still fails, so
    # nothing launches
    d = _dims(npw=0)
    ins = _inputs(I_eps_array=0, wtilde_array=0)
    assert _call(lib, d, ins, ws=0) == 4


def test_outputs_and_workspace(lib):
    assert _call(lib, _dims(), _inputs(), ach=0) == 1
    assert _call(lib, _dims(), _inputs(), asx=FAKE + 8) == 1
    assert _call(lib, _dims(), _inputs(), ws=0) == 4
    d = _dims()
    need = lib.gpp_sigma_fwd_workspace(C.byref(d))
    assert need > 0
    assert _call(lib, d, _inputs(), ws_bytes=need - 1) == 4
    assert "workspace" in lib.gpp_last_error().decode()


def test_workspace_size_is_host_only_and_monotone(lib):
    small = lib.gpp_sigma_fwd_workspace(C.byref(_dims(ng=64, npw=4)))
    big = lib.gpp_sigma_fwd_workspace(C.byref(_dims(ng=32768, npw=1638)))
    assert 0 < small <= big
    assert lib.gpp_sigma_fwd_workspace(None) == 0


def _fwd_workgroups(lib, nb, ng, npw, nw):
    """Workgroups of the forward's tile kernel, from its workspace size: one
    partial row of 4 * nw doubles per workgroup, plus as many first-stage
    rows while there are at most 512 workgroups."""
    ws = lib.gpp_sigma_fwd_workspace(C.byref(_dims(nb, 1, ng, npw, nw)))
    row = 32 * nw
    assert ws % (2 * row) == 0
    assert ws // (2 * row) <= 512
    return ws // (2 * row)


def test_forward_band_chunks(lib):
    """Above 512 bands the forward splits the band loop into chunks of at
    most 512 bands (whole band groups but the last), each tile chunk a
    workgroup row of its own: the tile count, and so the partial rows,
    scale with the chunk count.  64 rows x 40 columns at nfreq 3 are 20
    two-column tiles, i.e. 5 workgroups per chunk."""
    for nb, chunks in ((512, 1), (513, 2), (1024, 2), (1025, 3), (1536, 3), (1537, 4)):
        assert _fwd_workgroups(lib, nb, 64, 40, 3) == 5 * chunks, nb
    # nfreq 2 takes three columns per tile: 14 tiles per chunk, 3 chunks of
    # at most 512 bands, four tiles per workgroup
    assert _fwd_workgroups(lib, 1030, 64, 40, 2) == (14 * 3 + 3) // 4


def test_python_binding_rejects_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()


def _bwd(lib, dims, ins, ga=FAKE + 0x900000, gs=FAKE + 0x900100, outs=(0, 0, 0, 0),
         ws=FAKE + 0xA00000, ws_bytes=None):
    need = lib.gpp_sigma_bwd_workspace(C.byref(dims))
    ws_bytes = need if ws_bytes is None else ws_bytes
    return lib.gpp_sigma_bwd(C.byref(dims), C.byref(ins), C.c_void_p(ga), C.c_void_p(gs),
                             *[C.c_void_p(o) for o in outs], C.c_void_p(ws), ws_bytes,
                             None)


def test_bwd_validation(lib):
    d = _dims()
    assert _bwd(lib, _dims(nv=9), _inputs()) == 1
    assert _bwd(lib, d, _inputs(aqsntemp=0)) == 1
    assert _bwd(lib, d, _inputs(), ga=0) == 1
    assert "grad_achtemp" in lib.gpp_last_error().decode()
    assert _bwd(lib, d, _inputs(), gs=FAKE + 8) == 1
    assert _bwd(lib, d, _inputs(), outs=(FAKE + 8, 0, 0, 0)) == 1
    assert "grad_aqsmtemp" in lib.gpp_last_error().decode()
    assert _bwd(lib, d, _inputs(), ws=0) == 4
    need = lib.gpp_sigma_bwd_workspace(C.byref(d))
    assert need > 0
    assert _bwd(lib, d, _inputs(), ws_bytes=need - 1) == 4
    assert _bwd(lib, d, _inputs(), ws=FAKE + 0xA00010) == 1
    assert "256-byte" in lib.gpp_last_error().decode()


def test_bwd_workspace_grows_with_rows_bands_columns(lib):
    a = lib.gpp_sigma_bwd_workspace(C.byref(_dims(nb=8, ng=256, npw=10)))
    b = lib.gpp_sigma_bwd_workspace(C.byref(_dims(nb=8, ng=512, npw=10)))
    c = lib.gpp_sigma_bwd_workspace(C.byref(_dims(nb=16, ng=512, npw=10)))
    assert 0 < a < b < c
    assert lib.gpp_sigma_bwd_workspace(None) == 0


def _bwd_segments(lib, nb, nv, ng, npw, nw):
    """Segments of the aqsntemp-gradient pass's G' range, read back from the
    workspace size: the unsplit layout plus S * nb * ng complex partials."""
    up = lambda e: (e * 16 + 255) // 256 * 256
    unsplit = up(nw) + up(nw * nb) + up(((ng + 255) // 256) * nb * npw)
    extra = lib.gpp_sigma_bwd_workspace(C.byref(_dims(nb, nv, ng, npw, nw))) - unsplit
    return 1 if extra == 0 else extra // (16 * nb * ng)


def test_bwd_bands_pass_segments(lib):
    # ~16 rounds of 4096 resident waves, segments of >= 64 G' columns
    assert _bwd_segments(lib, 256, 2, 16384, 819, 3) == 4      # adjoint workload
    assert _bwd_segments(lib, 512, 2, 32768, 1638, 3) == 1     # Si-shaped: grid already long
    assert _bwd_segments(lib, 1024, 4, 65536, 3276, 3) == 1
    assert _bwd_segments(lib, 8, 2, 200, 130, 3) == 2          # capped by 130 // 64
    assert _bwd_segments(lib, 13, 2, 300, 200, 3) == 3
    assert _bwd_segments(lib, 32, 2, 512, 63, 3) == 1          # fewer than 2 x 64 columns
    assert lib.gpp_sigma_bwd_workspace(C.byref(_dims(256, 2, 16384, 819, 3))) == 483143936


def test_plan_validation_before_any_device_call(lib):
    handle = C.c_void_p(123)
    bad = (_lib.GppDims * 2)(_lib.GppDims(8, 2, 100, 10, 3), _lib.GppDims(8, 9, 100, 10, 3))
    assert lib.gpp_plan_create(2, bad, C.byref(handle)) == 1
    assert "state 1" in lib.gpp_last_error().decode() and handle.value is None
    mixed = (_lib.GppDims * 2)(_lib.GppDims(8, 2, 100, 10, 3), _lib.GppDims(8, 2, 100, 10, 2))
    assert lib.gpp_plan_create(2, mixed, C.byref(handle)) == 1
    assert "nfreq" in lib.gpp_last_error().decode()
    assert lib.gpp_plan_create(0, bad, C.byref(handle)) == 1
    assert lib.gpp_plan_create(1, None, C.byref(handle)) == 1
    assert lib.gpp_plan_create(1, bad, None) == 1
    assert lib.gpp_sigma_batched(None, None, None, None, None, 0, None) == 1
    assert lib.gpp_plan_workspace(None) == 0
    info = _lib.GppPlanInfo()
    assert lib.gpp_plan_get_info(None, C.byref(info)) == 1
    lib.gpp_plan_destroy(None)  # no-op


def _ladder_call(lib, step, dims, ins=None, ws_bytes=None, ws=FAKE + 0x700000):
    ins = _inputs() if ins is None else ins
    need = lib.gpp_ladder_workspace(step, C.byref(dims))
    ws_bytes = need if ws_bytes is None else ws_bytes
    return lib.gpp_ladder_fwd(step, C.byref(dims), C.byref(ins), C.c_void_p(FAKE + 0x600000),
                              C.c_void_p(FAKE + 0x600100), C.c_void_p(ws), ws_bytes, None)


def test_ladder_names_and_validation(lib):
    n = lib.gpp_ladder_steps()
    assert n == 12
    names = [lib.gpp_ladder_name(s).decode() for s in range(n)]
    assert [s[:2] for s in names[:9]] == [f"v{k}" for k in range(9)]
    assert [s[:2] for s in names[9:11]] == ["m1", "m2"]
    assert "production" in names[n - 1]
    assert lib.gpp_ladder_name(-1) is None and lib.gpp_ladder_name(n) is None
    d = _dims()
    for bad in (-1, n):
        assert lib.gpp_ladder_workspace(bad, C.byref(d)) == 0
        assert _ladder_call(lib, bad, d, ws_bytes=256) == 1
        assert "step" in lib.gpp_last_error().decode()
    # steps 0-10 take nfreq <= 4; the production step takes up to 8
    d5 = _dims(nw=5)
    for step in range(n - 1):
        assert lib.gpp_ladder_workspace(step, C.byref(d5)) == 0
        assert _ladder_call(lib, step, d5, ws_bytes=1 << 20) == 1
        assert "nfreq" in lib.gpp_last_error().decode()
    assert lib.gpp_ladder_workspace(n - 1, C.byref(d5)) == lib.gpp_sigma_fwd_workspace(C.byref(d5))
    for step in range(n - 1):
        assert lib.gpp_ladder_workspace(step, C.byref(d)) > 0
        assert _ladder_call(lib, step, d, ins=_inputs(aqsntemp=0)) == 1
        assert _ladder_call(lib, step, d, ws=0) == 4
        assert _ladder_call(lib, step, d, ws_bytes=lib.gpp_ladder_workspace(step, C.byref(d)) - 1) == 4
        assert "workspace" in lib.gpp_last_error().decode()
    # the transposed aqsmtemp copy of steps 7-8 lives in the workspace
    big = _dims(nb=512, ng=32768, npw=1638)
    assert lib.gpp_ladder_workspace(7, C.byref(big)) >= \
        lib.gpp_ladder_workspace(6, C.byref(big)) + 512 * 1638 * 16


def _hip_device_count():
    """Devices the HIP runtime sees (hipGetDeviceCount), or None if the
    runtime cannot be asked."""
    try:
        hip = C.CDLL("libamdhip64.so")
    except OSError:
        return None
    n = C.c_int(-1)
    rc = hip.hipGetDeviceCount(C.byref(n))
    return n.value if rc == 0 else 0


@pytest.mark.skipif(_hip_device_count() != 0,
                    reason="checks the no-device path; this host has (or may have) a GPU")
def test_no_device_is_unsupported(lib):
    """With valid arguments and no device, every compute entry point returns
    GPP_ERR_UNSUPPORTED and enqueues nothing (the addresses are fake)."""
    d = _dims()
    assert _call(lib, d, _inputs()) == 5
    assert "no HIP device" in lib.gpp_last_error().decode()
    assert _bwd(lib, d, _inputs(), outs=(FAKE + 0xB00000, 0, 0, 0)) == 5
    assert "gpp_sigma_bwd" in lib.gpp_last_error().decode()
    for step in (0, 10):
        assert _ladder_call(lib, step, d) == 5
    handle = C.c_void_p()
    ok = (_lib.GppDims * 1)(_lib.GppDims(8, 2, 100, 10, 3))
    assert lib.gpp_plan_create(1, ok, C.byref(handle)) == 5 and handle.value is None
    flops = C.c_double(0.0)
    assert lib.gpp_mb_fp64_fma(C.c_void_p(FAKE), 1, 1, None, C.byref(flops)) == 5
    assert lib.gpp_mb_copy(C.c_void_p(FAKE), C.c_void_p(FAKE + 0x100000), 4096, 1, None) == 5
    assert lib.gpp_mb_read(C.c_void_p(FAKE), 4096, 0, 1, 1, C.c_void_p(FAKE + 0x100000),
                           None) == 5
    assert lib.gpp_mb_lds(2, 1, 1, C.c_void_p(FAKE), None) == 5
    for bad in ((4, 1, 1), (-1, 1, 1), (0, 0, 1), (0, 1, 0)):
        assert lib.gpp_mb_lds(*bad, C.c_void_p(FAKE), None) == 1
    assert lib.gpp_mb_lds(0, 1, 1, None, None) == 1


def _qp(lib, dims, ins=None, step=0.5, energy=0.1, vxc=0.0, qp=FAKE + 0xC00000,
        ws=FAKE + 0x700000, ws_bytes=None):
    ins = _inputs() if ins is None else ins
    need = lib.gpp_sigma_fwd_workspace(C.byref(dims))
    ws_bytes = need if ws_bytes is None else ws_bytes
    return lib.gpp_sigma_qp(C.byref(dims), C.byref(ins), step, energy, vxc,
                            C.c_void_p(FAKE + 0x600000), C.c_void_p(FAKE + 0x600100),
                            C.c_void_p(qp), C.c_void_p(ws), ws_bytes, None)


def test_qp_validation(lib):
    for nw in (1, 2, 4, 8):
        assert _qp(lib, _dims(nw=nw)) == 1
        assert "odd" in lib.gpp_last_error().decode()
    inf, nan = float("inf"), float("nan")
    for step in (0.0, -0.5, inf, nan):
        assert _qp(lib, _dims(), step=step) == 1
        assert "freq_step" in lib.gpp_last_error().decode()
    for e, v in ((nan, 0.0), (0.0, inf), (-inf, 0.0)):
        assert _qp(lib, _dims(), energy=e, vxc=v) == 1
    assert _qp(lib, _dims(), qp=0) == 1 and "qp" in lib.gpp_last_error().decode()
    assert _qp(lib, _dims(), qp=FAKE + 4) == 1
    assert _qp(lib, _dims(), ins=_inputs(aqsntemp=0)) == 1
    assert _qp(lib, _dims(), ws=0) == 4
    assert _qp(lib, _dims(nw=5), ws_bytes=lib.gpp_sigma_fwd_workspace(C.byref(_dims(nw=5))) - 1) == 4
    if _hip_device_count() == 0:
        assert _qp(lib, _dims(nw=5)) == 5
