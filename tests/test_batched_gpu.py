"""GPU parity of the persistent batched forward (gpp_sigma_batched) against
the oracle and the plain forward, its graph replays, and its autotuner
cache.  Every state's achtemp/asxtemp must match at 1e-12 relative."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2008_11326_amd import inputs as I
from tests.gpu_helpers import assert_parity, load_golden, mixed_pole_problem, say, to_device

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

UNEVEN = [I.Dims(9, 2, 300, 15, 3), I.Dims(33, 2, 777, 38, 3), I.Dims(4, 0, 64, 3, 3),
          I.Dims(6, 6, 129, 7, 3), I.Dims(5, 1, 70, 0, 3), I.Dims(1, 1, 1, 1, 3),
          I.Dims(64, 2, 2048, 102, 3), I.Dims(17, 3, 500, 25, 3)]


@pytest.fixture(scope="module")
def gpp():
    import paper_2008_11326_amd as gpp
    from paper_2008_11326_amd import _lib
    _lib.load()
    return gpp


@pytest.fixture(scope="module")
def uneven():
    probs = [I.make_problem(d, [17, k], 0.05 if k % 2 else 0.0) for k, d in enumerate(UNEVEN)]
    refs = [oracle.sigma_fwd(p) for p in probs]
    return probs, refs, [to_device(p) for p in probs]


def test_uneven_states_vs_oracle_and_plain(gpp, uneven, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("GPP_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs, refs, dev = uneven
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    ach, asx = gpp.sigma_batched(plan, dev)
    torch.cuda.synchronize()
    info = plan.info()
    say(f"[batched] plan {info}")
    assert info["tuned"] == 1 and info["candidates"] >= 2
    for k, (p, ref, d) in enumerate(zip(probs, refs, dev)):
        assert_parity(ach[k].cpu().numpy(), ref[0], ref[2], f"state {k} achtemp")
        assert_parity(asx[k].cpu().numpy(), ref[1], ref[3], f"state {k} asxtemp")
        pa, px = gpp.sigma_fwd(**d, nvband=p.dims.nvband)
        g = pa.cpu().numpy(), px.cpu().numpy()
        for got, plain in ((ach[k].cpu().numpy(), g[0]), (asx[k].cpu().numpy(), g[1])):
            scale = np.abs(plain) + 1e-300
            assert np.all(np.abs(got - plain) <= 1e-12 * scale + 1e-300)
    plan.close()


@pytest.mark.parametrize("sched", [0, 1, 2, 3, 4])
def test_every_schedule_vs_oracle(gpp, uneven, sched, monkeypatch):
    """Each schedule alone (GPP_BATCHED_SCHEDULE): round-robin, XCD chunks,
    global queue, per-XCD queues and the flat grid, on the uneven states
    (including an empty one and a 1x1x1 one) against the oracle."""
    import torch
    monkeypatch.setenv("GPP_BATCHED_SCHEDULE", str(sched))
    probs, refs, dev = uneven
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    ach, asx = gpp.sigma_batched(plan, dev)
    torch.cuda.synchronize()
    info = plan.info()
    say(f"[batched] schedule {sched}: {info}")
    assert info["schedule"] == sched and info["from_cache"] == 0
    for k, ref in enumerate(refs):
        assert_parity(ach[k].cpu().numpy(), ref[0], ref[2], f"state {k} achtemp")
        assert_parity(asx[k].cpu().numpy(), ref[1], ref[3], f"state {k} asxtemp")
    plan.close()


def _plan_bands(nw):
    """Bands per group the plan offers its persistent kernels for nw
    frequencies (gpp_plan_create)."""
    return (3, 2) if nw <= 3 else ((2, 1) if nw == 4 else (1,))


# every batched tile variant: frequency count x persistent schedule x bands
# per group, and the flat grid (the plain forward's tile) per frequency count
VARIANTS = [(nw, sched, bu) for nw in range(1, 9) for sched in (0, 1, 2, 3)
            for bu in _plan_bands(nw)] + [(nw, 4, None) for nw in (1, 2, 4, 5, 6, 7, 8)]


@pytest.fixture(scope="module")
def uneven_by_nfreq():
    """The uneven states with another frequency count (one set kept at a
    time), their oracle outputs and device copies."""
    held = {}

    def get(nw):
        if nw not in held:
            held.clear()
            dims = [I.Dims(d.number_bands, d.nvband, d.ncouls, d.ngpown, nw) for d in UNEVEN]
            probs = [I.make_problem(d, [19, k], 0.05 if k % 2 else 0.0)
                     for k, d in enumerate(dims)]
            held[nw] = (probs, [oracle.sigma_fwd(p) for p in probs],
                        [to_device(p) for p in probs])
        return held[nw]
    return get


@pytest.mark.parametrize("nw,sched,bu", VARIANTS,
                         ids=[f"nw{a}-s{b}-bu{c}" for a, b, c in VARIANTS])
def test_every_tile_variant_vs_oracle(gpp, uneven_by_nfreq, nw, sched, bu, monkeypatch):
    """One schedule and one tile variant at a time (GPP_BATCHED_SCHEDULE,
    GPP_BATCHED_BANDS) for 1 to 8 frequencies, on the uneven states, against
    the oracle."""
    import torch
    monkeypatch.setenv("GPP_BATCHED_SCHEDULE", str(sched))
    if bu is not None:
        monkeypatch.setenv("GPP_BATCHED_BANDS", str(bu))
    probs, refs, dev = uneven_by_nfreq(nw)
    say(f"[batched] nfreq {nw} schedule {sched} bands {bu}")
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    ach, asx = gpp.sigma_batched(plan, dev)
    torch.cuda.synchronize()
    info = plan.info()
    assert info["schedule"] == sched and info["from_cache"] == 0
    if bu is not None:
        assert info["bands_per_group"] == bu
    for k, ref in enumerate(refs):
        assert_parity(ach[k].cpu().numpy(), ref[0], ref[2], f"state {k} achtemp")
        assert_parity(asx[k].cpu().numpy(), ref[1], ref[3], f"state {k} asxtemp")
    plan.close()


@pytest.fixture(scope="module")
def many():
    """3000 tiny uneven states (1-6 bands, 1-100 rows, 0-5 G' columns, some
    empty), their oracle outputs and device copies."""
    rng = np.random.default_rng(31)
    dims = []
    for _ in range(3000):
        nb = int(rng.integers(1, 7))
        ng = int(rng.integers(1, 101))
        dims.append(I.Dims(nb, int(rng.integers(0, nb + 1)), ng,
                           int(rng.integers(0, min(ng, 5) + 1)), 3))
    probs = [I.make_problem(d, [31, k], 0.05 if k % 3 == 0 else 0.0) for k, d in enumerate(dims)]
    refs = [oracle.sigma_fwd(p, nthreads=1) for p in probs]
    return probs, refs, [to_device(p) for p in probs]


@pytest.mark.parametrize("sched", [0, 1, 2, 3, 4])
def test_many_small_states(gpp, many, sched, monkeypatch):
    """One plan over 3000 tiny states (the state lookup of the flat grid,
    the static schedules' per-state row slots, the per-XCD queues' regions
    and the per-state reductions over many states), each schedule alone,
    against the oracle.  Every schedule's partial rows number at most the
    plan's tiles, so the workspace stays far below states x waves rows."""
    import torch
    monkeypatch.setenv("GPP_BATCHED_SCHEDULE", str(sched))
    probs, refs, dev = many
    say(f"[batched] {len(probs)} small states, schedule {sched}")
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    ach, asx = gpp.sigma_batched(plan, dev)
    torch.cuda.synchronize()
    info = plan.info()
    assert info["schedule"] == sched
    row = 4 * 3 * 8
    assert plan.workspace_bytes <= 256 + (info["total_tiles"] * row + 255) // 256 * 256
    a, x = ach.cpu().numpy(), asx.cpu().numpy()
    for k, ref in enumerate(refs):
        assert_parity(a[k], ref[0], ref[2], f"state {k} achtemp")
        assert_parity(x[k], ref[1], ref[3], f"state {k} asxtemp")
    plan.close()


MAX_STATES_BASE = [I.Dims(1, 1, 1, 1, 3), I.Dims(3, 2, 64, 2, 3), I.Dims(2, 0, 65, 3, 3),
                   I.Dims(5, 5, 100, 4, 3), I.Dims(4, 1, 30, 0, 3), I.Dims(6, 2, 129, 5, 3),
                   I.Dims(1, 0, 17, 1, 3), I.Dims(2, 2, 200, 2, 3)]


@pytest.mark.parametrize("sched", [0, 1, 2, 3, 4])
def test_the_largest_state_count(gpp, sched, monkeypatch):
    """GPP_MAX_STATES = 65536 states in one plan, through the C ABI: state s
    has the sizes and inputs of MAX_STATES_BASE[s % 8] (one of them empty),
    so the oracle values of eight problems check every state; each schedule
    alone, and its workspace within one partial row per tile."""
    import ctypes as C
    import torch
    from paper_2008_11326_amd import _lib
    lib = _lib.load()
    monkeypatch.setenv("GPP_BATCHED_SCHEDULE", str(sched))
    nbase, nmax = len(MAX_STATES_BASE), 65536
    probs = [I.make_problem(d, [43, k], 0.05 if k % 2 else 0.0)
             for k, d in enumerate(MAX_STATES_BASE)]
    refs = [oracle.sigma_fwd(p, nthreads=1) for p in probs]
    dev = [to_device(p) for p in probs]
    keys = ("aqsmtemp", "aqsntemp", "I_eps_array", "wtilde_array", "vcoul", "wx_array")
    one = [_lib.GppInputs(*[C.c_void_p(t[k].data_ptr()) for k in keys]) for t in dev]
    ins = (_lib.GppInputs * nmax)(*[one[s % nbase] for s in range(nmax)])
    say(f"[batched] {nmax} states, schedule {sched}")
    plan = gpp.Plan([probs[s % nbase].dims.as_tuple() for s in range(nmax)])
    info = plan.info()
    row = 4 * 3 * 8
    assert plan.workspace_bytes <= 256 + (info["total_tiles"] * row + 255) // 256 * 256
    ach = torch.empty((nmax, 3), dtype=torch.complex128, device="cuda:0")
    asx = torch.empty_like(ach)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda:0")
    _lib.check(lib.gpp_sigma_batched(plan._h, ins, ach.data_ptr(), asx.data_ptr(),
                                     ws.data_ptr(), ws.numel(), None), "gpp_sigma_batched")
    torch.cuda.synchronize()
    assert plan.info()["schedule"] == sched
    a, x = ach.cpu().numpy(), asx.cpu().numpy()
    for k, ref in enumerate(refs):
        assert_parity(a[k::nbase], ref[0], ref[2], f"base problem {k} achtemp")
        assert_parity(x[k::nbase], ref[1], ref[3], f"base problem {k} asxtemp")
    plan.close()


def test_tiny_imaginary_lanes(gpp, tmp_path, monkeypatch):
    """States whose tiles mix lanes with (Im om)^2 below 2^-60 (one-by-one
    reciprocals, exact poles) with ordinary lanes, against the oracle."""
    import torch
    monkeypatch.setenv("GPP_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs = [mixed_pole_problem(50 + k, d, f) for k, (d, f) in enumerate(
        [(I.Dims(20, 2, 300, 7, 3), 0.5), (I.Dims(11, 2, 129, 5, 3), 1.0),
         (I.Dims(30, 2, 500, 12, 3), 0.05)])]
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    ach, asx = gpp.sigma_batched(plan, [to_device(p) for p in probs])
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        ref = oracle.sigma_fwd(p)
        assert_parity(ach[k].cpu().numpy(), ref[0], ref[2], f"state {k} achtemp")
        assert_parity(asx[k].cpu().numpy(), ref[1], ref[3], f"state {k} asxtemp")
    plan.close()


def test_graph_replays_are_bitwise_identical(gpp, uneven, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("GPP_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs, _, dev = uneven
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    nw = probs[0].dims.nfreq
    out = (torch.empty((len(probs), nw), dtype=torch.complex128, device="cuda:0"),
           torch.empty((len(probs), nw), dtype=torch.complex128, device="cuda:0"))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda:0")
    gpp.sigma_batched(plan, dev, out=out, workspace=ws)  # tunes, captures
    torch.cuda.synchronize()
    first = [o.cpu().numpy().copy() for o in out]
    for rep in range(4):
        # unrelated eager work and synchronisation between replays
        junk = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
        junk.sum().item()
        out[0].zero_()
        out[1].zero_()
        gpp.sigma_batched(plan, dev, out=out, workspace=ws)
        torch.cuda.synchronize()
        for a, b in zip(first, out):
            assert np.array_equal(a, b.cpu().numpy()), f"replay {rep} differs"
    plan.close()


def test_new_input_pointers_and_outputs(gpp, uneven, tmp_path, monkeypatch):
    """Alternate two input sets (descriptor re-upload, same graph) and move
    the outputs (re-capture); every call matches its own oracle values."""
    import torch
    monkeypatch.setenv("GPP_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs, refs, dev_a = uneven
    probs_b = [I.make_problem(p.dims, [23, k]) for k, p in enumerate(probs)]
    refs_b = [oracle.sigma_fwd(p) for p in probs_b]
    dev_b = [to_device(p) for p in probs_b]
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    for it, (dv, rf) in enumerate([(dev_a, refs), (dev_b, refs_b), (dev_a, refs),
                                   (dev_b, refs_b)]):
        ach, asx = gpp.sigma_batched(plan, dv)  # fresh outputs each call
        torch.cuda.synchronize()
        for k, ref in enumerate(rf):
            assert_parity(ach[k].cpu().numpy(), ref[0], ref[2], f"call {it} state {k}")
            assert_parity(asx[k].cpu().numpy(), ref[1], ref[3], f"call {it} state {k}")
    plan.close()


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_capturing_stream_is_refused(gpp, uneven, tmp_path, monkeypatch):
    """A stream that is being captured is refused before anything is
    enqueued (the plan replays a graph of its own); the plan then works as
    usual on an ordinary stream."""
    import torch
    monkeypatch.setenv("GPP_TUNE_CACHE", str(tmp_path / "tune.json"))
    probs, refs, dev = uneven
    plan = gpp.Plan([p.dims.as_tuple() for p in probs])
    nw = probs[0].dims.nfreq
    out = (torch.empty((len(probs), nw), dtype=torch.complex128, device="cuda:0"),
           torch.empty((len(probs), nw), dtype=torch.complex128, device="cuda:0"))
    ws = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device="cuda:0")
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        with pytest.raises(gpp.GppError) as err:
            gpp.sigma_batched(plan, dev, out=out, workspace=ws, stream=side.cuda_stream)
    assert "capturing" in str(err.value)
    assert plan.info()["tuned"] == 0  # nothing ran, not even the tuner
    torch.cuda.synchronize()
    ach, asx = gpp.sigma_batched(plan, dev, out=out, workspace=ws)
    torch.cuda.synchronize()
    for k, ref in enumerate(refs):
        assert_parity(ach[k].cpu().numpy(), ref[0], ref[2], f"state {k} achtemp")
        assert_parity(asx[k].cpu().numpy(), ref[1], ref[3], f"state {k} asxtemp")
    plan.close()


TUNE_SCRIPT = r"""
import json, sys, os
sys.path.insert(0, {root!r})
import numpy as np, torch
import paper_2008_11326_amd as gpp
from paper_2008_11326_amd import inputs as I
dims = [I.Dims(8, 2, 256, 12, 3), I.Dims(20, 2, 640, 30, 3)]
states = []
for k, d in enumerate(dims):
    p = I.make_problem(d, [5, k])
    states.append([torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in p.arrays()])
plan = gpp.Plan([d.as_tuple() for d in dims])
ach, asx = gpp.sigma_batched(plan, states)
torch.cuda.synchronize()
print(json.dumps(plan.info()))
"""


def _tune_proc(cache, env_extra=None):
    env = dict(os.environ, GPP_TUNE_CACHE=str(cache))
    env.update(env_extra or {})
    r = subprocess.run([sys.executable, "-c", TUNE_SCRIPT.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_tuning_cache_roundtrip_and_corruption(tmp_path):
    cache = tmp_path / "tune.json"
    first = _tune_proc(cache)
    assert first["tuned"] == 1 and first["from_cache"] == 0 and first["tuned_ms"] > 0
    saved = json.loads(cache.read_text())
    assert len(saved) == 1
    second = _tune_proc(cache)
    assert second["from_cache"] == 1
    assert (second["bands_per_group"], second["schedule_order"]) == \
        (first["bands_per_group"], first["schedule_order"])
    cache.write_text("{ this is not json ]")
    third = _tune_proc(cache)
    assert third["from_cache"] == 0 and third["tuned"] == 1
    assert json.loads(cache.read_text())  # rewritten as valid JSON
    off = _tune_proc(tmp_path / "other.json", {"GPP_AUTOTUNE": "off"})
    assert off["tuned"] == 1 and off["tuned_ms"] == 0
    assert not (tmp_path / "other.json").exists()


def test_batched_workload_all_states_against_golden(gpp, tmp_path, monkeypatch):
    """All 64 states of the batched workload at full size (about 53 GB of
    inputs, drawn and uploaded state by state) in one plan -- the launch
    configuration bench.py times -- against oracle outputs written by
    tests/golden/make_golden.py."""
    import torch
    path = os.path.join(ROOT, "tests", "golden", "fwd_batched.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/fwd_batched.json not generated")
    gold = json.load(open(path))["states"]
    dims = I.batched_dims()
    if sorted(int(s) for s in gold) != list(range(len(dims))):
        pytest.skip("tests/golden/fwd_batched.json does not hold every state")
    need = sum(16 * (2 * d.number_bands * d.ncouls + 2 * d.ngpown * d.ncouls)
               + 8 * (d.ncouls + d.nfreq * d.number_bands) for d in dims)
    free, _ = torch.cuda.mem_get_info()
    if free < need + (8 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} free")
    monkeypatch.setenv("GPP_TUNE_CACHE", str(tmp_path / "tune.json"))
    say(f"[batched] uploading all {len(dims)} states ({need / 2**30:.1f} GiB)")
    dev = []
    for s, prob in I.make_batched():
        dev.append(to_device(prob))
        if s % 8 == 7:
            say(f"[batched] {s + 1} states uploaded")
    plan = gpp.Plan([d.as_tuple() for d in dims])
    ach, asx = gpp.sigma_batched(plan, dev)
    torch.cuda.synchronize()
    c = lambda pairs: np.array([complex(a, b) for a, b in pairs])
    worst = 0.0
    for k in range(len(dims)):
        g = gold[str(k)]
        worst = max(worst,
                    assert_parity(ach[k].cpu().numpy(), c(g["achtemp"]), g["ach_abs_sum"], f"state {k}"),
                    assert_parity(asx[k].cpu().numpy(), c(g["asxtemp"]), g["asx_abs_sum"], f"state {k}"))
    say(f"[batched] all states max rel err {worst:.2e}, plan {plan.info()}")
    plan.close()
    del dev
    torch.cuda.empty_cache()
