#!/usr/bin/env python3
"""Benchmark of the GPP forward reduction (achtemp/asxtemp, Sec. II-A) on
one MI355X.

A step is one gpp_sigma_fwd call (tile kernel + fixed-order reduction
kernels) over the larger synthetic system: number_bands=1024, nvband=4,
ncouls=65536, ngpown=3276, nfreq=3, 1 % of wtilde planted within 1e-6 of a
frequency, seed 2; inputs resident in HBM.  Prints one JSON line on stdout.

    python bench.py [--steps K] [--warmup W] [--workload large|si|small|adjoint]
    python bench.py --leg adjoint|batched|batched_small|batched_tiny|si   # one leg alone

`value` is the fp64 FLOP rate the hardware counts (the paper's measure,
Eq. 2): the fp64 VALU instructions of the tile kernel, counted once with
rocprofv3 for the same sources and workload (profiles/gpp_fwd_tiles_*.json,
keyed by a digest of the forward sources' code, comments left out), divided
by the time measured here.  Beside it: the algorithmic rate (21 fp64 operations per Coulomb-hole
and per screened-exchange term, fixed by the method), the FMA-share
ceiling of Sec. III (the closing FMA-ratio paragraph), the share of the
fp64 FMA rate a microbenchmark reaches on this GPU, and the Si-shaped
workload's rate.  The roofline block compares the algorithmic rate of the
tile kernel with the MI355X fp64 vector-ALU peak.  The CPU baseline times
the plain oracle on a bounded slice of the same workload.  The extra legs
time the adjoint against the forward, and the batched plan against
separate forwards on 64 uneven states, 256 small ones and 3000 tiny ones.
"""
import argparse
import ctypes as C
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GPP FP64 TFLOP/s and % FP64 peak; batched/adjoint vs plain at 1e-12 rel"
FLOP_PER_TERM = 21
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 fp64 FLOP/clk/CU
FWD_SOURCES = ("gpp_fwd.hip", "gpp_fwd_tile.h", "gpp_device.h", "gpp_fwd_shape.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _code_only(text):
    """Source text without comments and with runs of whitespace collapsed, so
    that editing a comment does not change the digest (the sources hold no
    string literal with a comment marker in it)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def fwd_source_digest():
    h = hashlib.sha256()
    for f in FWD_SOURCES:
        with open(os.path.join(ROOT, "paper_2008_11326_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def kernel_counters(workload_name):
    """The committed counter record of the tile kernel on this workload
    (rocprofv3 --pmc passes over the same sources), or None when the
    forward sources changed since the counters were taken."""
    import glob
    digest = fwd_source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "gpp_fwd_tiles_*.json"))):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("workload") == workload_name and rec.get("source_digest") == digest:
            rec["path"] = os.path.relpath(path, ROOT)
            return rec
    return None


def counted_fp64(rec):
    """fp64 operations the hardware counts per launch (64 lanes per wave
    instruction, an FMA counts 2) and the FMA share of the fp64 add, multiply
    and FMA instructions, from a counter record."""
    v = rec["valu_f64"]
    flops = 64.0 * (v["add"] + v["mul"] + v["trans"] + 2.0 * v["fma"])
    fma_share = v["fma"] / (v["add"] + v["mul"] + v["fma"])
    return flops, fma_share


def cpu_baseline(prob, target_seconds):
    """Time the CPU oracle on the first k G' columns (all bands and rows)."""
    import oracle  # test infrastructure: only this leg of the benchmark uses it
    d = prob.dims
    threads = len(os.sched_getaffinity(0))
    per_col = (d.number_bands + d.nvband) * d.ncouls * d.nfreq
    k0 = min(threads, d.ngpown)
    t0 = time.perf_counter()
    oracle.sigma_fwd_slice(prob, p=(0, k0), nthreads=threads)
    t_cal = time.perf_counter() - t0
    rate = k0 * per_col / max(t_cal, 1e-6)
    k = int(max(k0, min(d.ngpown, target_seconds * rate / per_col)))
    k = max(threads, (k // threads) * threads) if k > threads else k
    k = min(k, d.ngpown)
    t0 = time.perf_counter()
    oracle.sigma_fwd_slice(prob, p=(0, k), nthreads=threads)
    dt = time.perf_counter() - t0
    terms = k * per_col
    # one thread on one column, for the per-core rate
    t0 = time.perf_counter()
    oracle.sigma_fwd_slice(prob, p=(0, 1), nthreads=1)
    dt1 = time.perf_counter() - t0
    return {
        "value": FLOP_PER_TERM * terms / dt / 1e12, "unit": "TFLOP/s",
        "cores": min(threads, k), "kind": "oracle",
        "sample": f"G' columns p in [0,{k}) of {d.ngpown}, all {d.number_bands} bands "
                  f"and {d.ncouls} rows, nfreq={d.nfreq}: {terms:.3e} terms in {dt:.1f} s",
        "terms_per_s": terms / dt,
        "single_thread_terms_per_s": per_col / dt1,
        "cpu_model": _cpu_model(),
    }


def _cpu_model():
    """lscpu's model name, with vendor, family/model/stepping and hypervisor
    (a virtual machine may report only a generic name)."""
    fields = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if not fields.get("Model name"):
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        fields["Model name"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    name = fields.get("Model name")
    if not name:
        return None
    extra = [fields.get("Vendor ID")]
    if fields.get("CPU family"):
        extra.append(f"family {fields['CPU family']} model {fields.get('Model')} "
                     f"stepping {fields.get('Stepping')}")
    if fields.get("Hypervisor vendor"):
        extra.append(f"{fields['Hypervisor vendor']} guest")
    extra = [e for e in extra if e]
    return name + (f" ({', '.join(extra)})" if extra else "")


def timed_ms(fn, stream, reps):
    """Average milliseconds of fn() over reps runs, HIP events on `stream`."""
    import torch
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def fwd_leg(gpp, I, key, steps, warmup, stream):
    """Time `steps` gpp_sigma_fwd calls on workload `key` after `warmup`
    untimed ones: events on the launch stream around the whole run and
    around every call.  Returns (numbers, Problem, outputs)."""
    import numpy as np
    import torch
    wl = I.WORKLOADS[key]
    d = wl.dims
    log(f"[bench] generating {wl.name}")
    t0 = time.perf_counter()
    prob = I.make_problem(d, wl.seed, wl.pole_fraction)
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    t_in = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in prob.arrays()]
    ach = torch.empty(d.nfreq, dtype=torch.complex128, device=dev)
    asx = torch.empty(d.nfreq, dtype=torch.complex128, device=dev)
    ws = torch.empty(gpp.fwd_workspace_bytes(*d.as_tuple()), dtype=torch.uint8, device=dev)

    def step():
        gpp.sigma_fwd(*t_in, nvband=d.nvband, out=(ach, asx), workspace=ws,
                      stream=stream.cuda_stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_all0.record(stream)
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    t_all1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_all0.elapsed_time(t_all1)
    per_launch = [a.elapsed_time(b) for a, b in ev]
    log(f"[bench] {wl.name}: {steps} steps {total_ms:.3f} ms on device, "
        f"{wall * 1e3:.3f} ms wall; per call min {min(per_launch):.3f} "
        f"max {max(per_launch):.3f} ms")
    res = (ach.cpu().numpy(), asx.cpu().numpy())
    del t_in, ws, ach, asx
    torch.cuda.empty_cache()
    return {"workload": wl, "ms_per_step": total_ms / steps,
            "launch_ms": sum(per_launch) / len(per_launch),
            "launch_ms_min": min(per_launch), "launch_ms_max": max(per_launch)}, prob, res


def rates(wl, launch_ms, ms_per_step):
    """Algorithmic and (where the committed counters match) counted rates."""
    d = wl.dims
    terms = d.ch_terms + d.sx_terms
    alg = FLOP_PER_TERM * terms
    out = {"terms": terms, "algorithmic_tflops": alg / (ms_per_step * 1e-3) / 1e12,
           "algorithmic_tflops_launch": alg / (launch_ms * 1e-3) / 1e12,
           "terms_per_s": terms / (ms_per_step * 1e-3)}
    rec = kernel_counters(wl.name)
    if rec is not None and "valu_f64" in rec:
        flops, f = counted_fp64(rec)
        ceiling = (2.0 * f + (1.0 - f)) / 2.0 * FP64_VECTOR_PEAK_TFLOPS
        out.update({
            "counted_tflops": flops / (ms_per_step * 1e-3) / 1e12,
            "counted_flops_per_launch": flops, "fma_share": f,
            "fma_ceiling_tflops": ceiling, "counters": rec["path"],
            "traffic": rec.get("traffic_bytes"),
        })
    elif rec is not None:
        out["traffic"] = rec.get("traffic_bytes")
    return out


def max_rel_err(key, res):
    from tests.gpu_helpers import load_golden, rel_errors
    gold = load_golden(key)
    if gold is None:
        return None
    return float(max(rel_errors(res[0], gold["ach"], gold["ach_abs_sum"]).max(),
                     rel_errors(res[1], gold["asx"], gold["asx_abs_sum"]).max()))


def fma_peak_leg(stream, reps=5):
    """fp64 FMA rate of the microbenchmark kernel (16 independent chains per
    lane, 8 waves per SIMD) on this GPU, best of `reps`."""
    import torch
    from paper_2008_11326_amd import _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    blocks = cus * 8
    out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    flops = C.c_double(0.0)

    def run():
        _lib.check(lib.gpp_mb_fp64_fma(C.c_void_p(out.data_ptr()), blocks, 4096,
                                       C.c_void_p(stream.cuda_stream), C.byref(flops)),
                   "gpp_mb_fp64_fma")
    best = min(timed_ms(run, stream, 1) for _ in range(reps))
    return flops.value / (best * 1e-3) / 1e12


def adjoint_leg(gpp, I, stream, reps=5):
    """Forward and hand-written adjoint on the adjoint workload."""
    import numpy as np
    import torch
    wl = I.WORKLOADS["adjoint"]
    d = wl.dims
    prob = I.make_problem(d, wl.seed)
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in prob.arrays()]
    ga, gs = I.make_upstream_grad(d.nfreq, np.random.default_rng([wl.seed, 1]))
    ga = torch.from_numpy(ga).to(dev)
    gs = torch.from_numpy(gs).to(dev)
    ws = torch.empty(gpp.bwd_workspace_bytes(*d.as_tuple()), dtype=torch.uint8, device=dev)
    fwd = timed_ms(lambda: gpp.sigma_fwd(*t, nvband=d.nvband, stream=stream.cuda_stream),
                   stream, reps)
    bwd = timed_ms(lambda: gpp.sigma_bwd(*t, d.nvband, ga, gs, workspace=ws,
                                         stream=stream.cuda_stream), stream, reps)
    terms = d.ch_terms + d.sx_terms
    return {"workload": wl.name, "fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4),
            "bwd_over_fwd_time": round(bwd / fwd, 3),
            "bwd_terms_per_s": terms / (bwd * 1e-3),
            "bwd_throughput_vs_plain": round(fwd / bwd, 4),
            "grads": "aqsmtemp, aqsntemp, I_eps_array, wtilde_array"}


def batched_leg(gpp, I, stream, reps=3):
    """64 uneven states in one persistent graph-replayed launch vs 64
    sequential plain forwards on the same device-resident inputs."""
    import torch
    dims = I.batched_dims()
    states = [I.make_problem_device(dd, 1000 + k) for k, dd in enumerate(dims)]
    plan = gpp.Plan([dd.as_tuple() for dd in dims])
    nw = dims[0].nfreq
    dev = torch.device("cuda:0")
    out = (torch.empty((len(dims), nw), dtype=torch.complex128, device=dev),
           torch.empty((len(dims), nw), dtype=torch.complex128, device=dev))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    gpp.sigma_batched(plan, states, out=out, workspace=ws, stream=stream.cuda_stream)
    torch.cuda.synchronize()  # first call tunes (or reads the cache) and captures
    bat = timed_ms(lambda: gpp.sigma_batched(plan, states, out=out, workspace=ws,
                                             stream=stream.cuda_stream), stream, reps)
    plain_out = []

    def plain():
        plain_out.clear()
        for st, dd in zip(states, dims):
            plain_out.append(gpp.sigma_fwd(**st, nvband=dd.nvband, stream=stream.cuda_stream))
    seq = timed_ms(plain, stream, 1)
    worst = 0.0
    for k, (a, x) in enumerate(plain_out):
        for got, ref in ((out[0][k], a), (out[1][k], x)):
            worst = max(worst, float(torch.max(torch.abs(got - ref) / torch.abs(ref))))
    terms = sum(dd.ch_terms + dd.sx_terms for dd in dims)
    info = plan.info()
    plan.close()
    return {"states": len(dims), "terms": terms, "batched_ms": round(bat, 3),
            "sequential_plain_ms": round(seq, 3),
            "batched_tflops": round(FLOP_PER_TERM * terms / (bat * 1e-3) / 1e12, 3),
            "speedup_vs_sequential_plain": round(seq / bat, 4),
            "max_rel_diff_vs_plain": worst,
            "plan": {k: info[k] for k in ("bands_per_group", "schedule_order", "schedule",
                                           "waves", "candidates", "from_cache")},
            "data": "synthetic: the 64 state sizes of the seed-3 batched workload, values "
                    "drawn on the device from the same distributions with torch's "
                    "generator, seed 1000+s for state s (not the seed-3 host values)"}


def batched_small_leg(gpp, I, stream, reps=5, tiny=False):
    """Many small states (256 states of 32..128 bands and 1024..4096 rows;
    with tiny, 3000 states of 1..6 bands, 1..100 rows and 1..5 G' columns):
    one graph-replayed gpp_sigma_batched call against as many gpp_sigma_fwd
    calls in a row, both straight through the C ABI with argument structs
    built once, so that neither side pays the Python binding's per-call
    checks.  Each small state alone leaves most of the GPU idle."""
    import torch
    from paper_2008_11326_amd import _lib
    lib = _lib.load()
    dims = I.tiny_batched_dims() if tiny else I.small_batched_dims()
    seed0 = 3000 if tiny else 2000
    states = [I.make_problem_device(dd, seed0 + k) for k, dd in enumerate(dims)]
    nw = dims[0].nfreq
    dev = torch.device("cuda:0")
    keys = ("aqsmtemp", "aqsntemp", "I_eps_array", "wtilde_array", "vcoul", "wx_array")
    ins = (_lib.GppInputs * len(dims))()
    for k, st in enumerate(states):
        ins[k] = _lib.GppInputs(*[C.c_void_p(st[key].data_ptr()) for key in keys])
    cdims = [_lib.dims_struct(*dd.as_tuple()) for dd in dims]
    plan = gpp.Plan([dd.as_tuple() for dd in dims])
    out = (torch.empty((len(dims), nw), dtype=torch.complex128, device=dev),
           torch.empty((len(dims), nw), dtype=torch.complex128, device=dev))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    seq_out = (torch.empty_like(out[0]), torch.empty_like(out[1]))
    seq_ws = torch.empty(max(int(lib.gpp_sigma_fwd_workspace(C.byref(cd))) for cd in cdims),
                         dtype=torch.uint8, device=dev)
    sp = C.c_void_p(stream.cuda_stream)
    row = 16 * nw

    def batched():
        _lib.check(lib.gpp_sigma_batched(plan._h, ins, out[0].data_ptr(), out[1].data_ptr(),
                                         ws.data_ptr(), ws.numel(), sp), "gpp_sigma_batched")

    def sequential():
        a0, x0 = seq_out[0].data_ptr(), seq_out[1].data_ptr()
        w0, wn = seq_ws.data_ptr(), seq_ws.numel()
        for k, cd in enumerate(cdims):
            st = lib.gpp_sigma_fwd(C.byref(cd), C.byref(ins[k]), a0 + k * row, x0 + k * row,
                                   w0, wn, sp)
            if st:
                _lib.check(st, "gpp_sigma_fwd")
    batched()
    torch.cuda.synchronize()  # first call tunes (or reads the cache) and captures
    bat = min(timed_ms(batched, stream, 1) for _ in range(reps))
    seq = min(timed_ms(sequential, stream, 1) for _ in range(reps))
    worst = 0.0
    for got, ref in ((out[0], seq_out[0]), (out[1], seq_out[1])):
        worst = max(worst, float(torch.max(torch.abs(got - ref) / torch.abs(ref))))
    terms = sum(dd.ch_terms + dd.sx_terms for dd in dims)
    info = plan.info()
    plan.close()
    return {"states": len(dims), "terms": terms, "batched_ms": round(bat, 4),
            "sequential_plain_ms": round(seq, 4),
            "batched_tflops": round(FLOP_PER_TERM * terms / (bat * 1e-3) / 1e12, 3),
            "sequential_tflops": round(FLOP_PER_TERM * terms / (seq * 1e-3) / 1e12, 3),
            "speedup_vs_sequential_plain": round(seq / bat, 3),
            "max_rel_diff_vs_plain": worst,
            "plan": {k: info[k] for k in ("bands_per_group", "schedule_order", "schedule",
                                           "waves", "candidates", "from_cache")},
            "timing": "best of 5, HIP events on the launch stream; both sides call the C ABI",
            "data": ("synthetic: 3000 state sizes from default_rng(31) (1..6 bands, 1..100 rows, "
                     "1..5 G' columns, nvband min(2, bands), nfreq 3), values drawn on the "
                     "device, seed 3000+s for state s") if tiny else
                    ("synthetic: 256 state sizes from default_rng(5) (32..128 bands, "
                     "1024..4096 rows, ngpown = ncouls // 20, nvband 2, nfreq 3), values "
                     "drawn on the device, seed 2000+s for state s")}


def si_leg(gpp, I, stream, steps=5, warmup=2):
    """The Si-shaped per-task workload (512 bands, 32768 rows, 1638 columns)."""
    r, _, res = fwd_leg(gpp, I, "si", steps, warmup, stream)
    wl = r["workload"]
    q = rates(wl, r["launch_ms"], r["ms_per_step"])
    out = {"workload": wl.name, "ms_per_step": round(r["ms_per_step"], 4),
           "algorithmic_tflops": round(q["algorithmic_tflops"], 4),
           "terms_per_s": q["terms_per_s"], "max_rel_err_vs_oracle": max_rel_err("si", res)}
    if "counted_tflops" in q:
        out["counted_tflops"] = round(q["counted_tflops"], 4)
        out["fma_share"] = round(q["fma_share"], 4)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the Si-shaped, adjoint, batched and FMA-peak legs")
    ap.add_argument("--leg", choices=("all", "adjoint", "batched", "batched_small",
                                      "batched_tiny", "si"),
                    default="all",
                    help="adjoint, batched or si: run only that leg and print its JSON "
                         "(for per-kernel profiling); all: the benchmark line")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = (f"bench.py measures one GPU only (asked for --gpus {args.gpus}, "
               f"WORLD_SIZE={world}); multi-GPU G'-column sharding is not built")
        print(msg, file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    import paper_2008_11326_amd as gpp
    from paper_2008_11326_amd import _lib
    from paper_2008_11326_amd import inputs as I

    _lib.load()  # fail loudly if the HIP library is missing
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    if args.leg != "all":
        leg = {"adjoint": adjoint_leg, "batched": batched_leg,
               "batched_small": batched_small_leg, "si": si_leg,
               "batched_tiny": lambda *a: batched_small_leg(*a, tiny=True)}[args.leg]
        log(f"[bench] {args.leg} leg only")
        print(json.dumps({"leg": args.leg, **leg(gpp, I, stream)}), flush=True)
        return

    r, prob, res = fwd_leg(gpp, I, args.workload, args.steps, args.warmup, stream)
    wl = r["workload"]
    d = wl.dims
    q = rates(wl, r["launch_ms"], r["ms_per_step"])
    counted = "counted_tflops" in q
    value = q["counted_tflops"] if counted else q["algorithmic_tflops"]
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "number_bands": d.number_bands,
                   "nvband": d.nvband, "ncouls": d.ncouls, "ngpown": d.ngpown,
                   "nfreq": d.nfreq, "seed": wl.seed,
                   "pole_fraction": wl.pole_fraction},
        "value_kind": ("hardware-counted fp64 FLOPs per launch (" + q["counters"] +
                       ") / measured time" if counted else
                       "algorithmic (21 per term): no counter record matches these sources"),
        "pct_fp64_peak": round(100.0 * value / FP64_VECTOR_PEAK_TFLOPS, 2),
        "algorithmic_tflops": round(q["algorithmic_tflops"], 4),
        "pct_fp64_peak_algorithmic": round(100.0 * q["algorithmic_tflops"] /
                                           FP64_VECTOR_PEAK_TFLOPS, 2),
        "terms_per_s": q["terms_per_s"],
        "roofline": {"bound": "alu", "achieved": round(q["algorithmic_tflops_launch"], 4),
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(q["algorithmic_tflops_launch"] /
                                   FP64_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": q.get("traffic"),
                     "kernel": f"gpp::fwd_tiles<{d.nfreq},2> + two reduce_rows<{d.nfreq}> "
                               f"(one gpp_sigma_fwd), algorithmic FLOPs",
                     "launch_ms": round(r["launch_ms"], 4)},
        "max_rel_err_vs_oracle": max_rel_err(args.workload, res),
        # the paper's best figure (Table I, v8): another machine, workload and
        # FLOP count (counted on the V100), so context only, not a target
        "paper_context": {"tflops": 3.71, "pct_of_fp64_peak": 55,
                          "machine": "NVIDIA V100, 6.7 TFLOP/s fp64 peak",
                          "workload": "BerkeleyGW Si-214, 2 frequencies (Table I, v8)"},
    }
    if counted:
        out["fp64_counted"] = {
            "flops_per_launch": q["counted_flops_per_launch"],
            "fma_share": round(q["fma_share"], 4),
            "fma_ceiling_tflops": round(q["fma_ceiling_tflops"], 3),
            "pct_of_fma_ceiling": round(100.0 * value / q["fma_ceiling_tflops"], 2),
            "source": q["counters"]}
    if q.get("traffic"):
        out["hbm_gbps"] = round(q["traffic"] / (r["launch_ms"] * 1e-3) / 1e9, 1)
    if not args.no_extras:
        log("[bench] fp64 FMA microbenchmark")
        peak = fma_peak_leg(stream)
        out["fma_microbench"] = {"tflops": round(peak, 3),
                                 "pct_of_measured_fma_peak": round(100.0 * value / peak, 2)}
        log("[bench] Si-shaped leg")
        out["si"] = si_leg(gpp, I, stream)
        log("[bench] adjoint leg")
        out["adjoint"] = adjoint_leg(gpp, I, stream)
        log("[bench] batched leg")
        out["batched"] = batched_leg(gpp, I, stream)
        log("[bench] batched leg, many small states")
        out["batched_small"] = batched_small_leg(gpp, I, stream)
        log("[bench] batched leg, many tiny states")
        out["batched_tiny"] = batched_small_leg(gpp, I, stream, tiny=True)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded slice")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
