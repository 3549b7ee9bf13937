#!/usr/bin/env python3
"""Benchmark of the GPP forward reduction (achtemp/asxtemp, Sec. II-A) on
one MI355X.

A step is one gpp_sigma_fwd call (tile kernel + fixed-order reduction
kernel) over the synthetic workload with the per-task shape of the paper's
Si-system run: number_bands=512, nvband=2, ncouls=32768, ngpown=1638,
nfreq=3, inputs resident in HBM.  Prints one JSON line on stdout.

    python bench.py [--steps K] [--warmup W] [--workload si|small|adjoint|large]
    python bench.py --leg adjoint|batched     # one leg alone, for profiling

Throughput is algorithmic: 21 fp64 operations per Coulomb-hole term plus
21 per screened-exchange term (the arithmetic the method needs, fixed
independently of the implementation), divided by the measured time.  The
roofline block compares it with the MI355X fp64 vector-ALU peak.  The CPU
baseline times the plain oracle on a bounded slice of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GPP FP64 TFLOP/s and % FP64 peak; batched/adjoint vs plain at 1e-12 rel"
FLOP_PER_TERM = 21
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 fp64 FLOP/clk/CU


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def fwd_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("gpp_fwd.hip", "gpp_fwd_tile.h", "gpp_device.h"):
        with open(os.path.join(ROOT, "paper_2008_11326_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name):
    """HBM-side bytes per launch from the committed counter run
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
    copy of known size), or None when the kernel sources changed since."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "gpp_fwd_tiles_*.json")):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("workload") == workload_name and \
                rec.get("source_digest") == fwd_source_digest():
            return rec["traffic_bytes"]
    return None


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
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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
            "data": "synthetic, drawn on the device (same distributions)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="si")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint and batched legs")
    ap.add_argument("--leg", choices=("all", "adjoint", "batched"), default="all",
                    help="adjoint or batched: run only that leg and print its JSON "
                         "(for per-kernel profiling); all: the benchmark line")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = (f"bench.py measures one GPU only (asked for --gpus {args.gpus}, "
               f"WORLD_SIZE={world}); multi-GPU G'-column sharding is not built")
        print(msg, file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2008_11326_amd as gpp
    from paper_2008_11326_amd import _lib
    from paper_2008_11326_amd import inputs as I

    _lib.load()  # fail loudly if the HIP library is missing
    if args.leg != "all":
        stream = torch.cuda.current_stream(torch.device("cuda:0"))
        leg = adjoint_leg if args.leg == "adjoint" else batched_leg
        log(f"[bench] {args.leg} leg only")
        print(json.dumps({"leg": args.leg, **leg(gpp, I, stream)}), flush=True)
        return
    wl = I.WORKLOADS[args.workload]
    d = wl.dims
    log(f"[bench] generating {wl.name}")
    t0 = time.perf_counter()
    prob = I.make_problem(d, wl.seed, wl.pole_fraction)
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s")

    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    t_in = [to(a) for a in prob.arrays()]
    ach = torch.empty(d.nfreq, dtype=torch.complex128, device=dev)
    asx = torch.empty(d.nfreq, dtype=torch.complex128, device=dev)
    ws = torch.empty(gpp.fwd_workspace_bytes(*d.as_tuple()), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        gpp.sigma_fwd(*t_in, nvband=d.nvband, out=(ach, asx), workspace=ws,
                      stream=stream.cuda_stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # events on the stream the kernels are launched on
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
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
    per_launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = total_ms / args.steps
    launch_ms = sum(per_launch_ms) / len(per_launch_ms)
    log(f"[bench] {args.steps} steps: {total_ms:.3f} ms on device, {wall * 1e3:.3f} ms wall; "
        f"per launch min {min(per_launch_ms):.3f} max {max(per_launch_ms):.3f} ms")

    terms = d.ch_terms + d.sx_terms
    flops = FLOP_PER_TERM * terms
    value = flops / (ms_per_step * 1e-3) / 1e12
    achieved = flops / (launch_ms * 1e-3) / 1e12

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "number_bands": d.number_bands,
                   "nvband": d.nvband, "ncouls": d.ncouls, "ngpown": d.ngpown,
                   "nfreq": d.nfreq, "seed": wl.seed,
                   "pole_fraction": wl.pole_fraction},
        "pct_fp64_peak": round(100.0 * value / FP64_VECTOR_PEAK_TFLOPS, 2),
        "terms_per_s": terms / (ms_per_step * 1e-3),
        "roofline": {"bound": "alu", "achieved": round(achieved, 4),
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(wl.name),
                     "kernel": "gpp::fwd_tiles<3,2> + two reduce_rows<3> (one gpp_sigma_fwd)",
                     "launch_ms": round(launch_ms, 4)},
    }
    res = (ach.cpu().numpy(), asx.cpu().numpy())
    from tests.gpu_helpers import load_golden, rel_errors
    gold = load_golden(args.workload)
    if gold is not None:
        e = max(rel_errors(res[0], gold["ach"], gold["ach_abs_sum"]).max(),
                rel_errors(res[1], gold["asx"], gold["asx_abs_sum"]).max())
        out["max_rel_err_vs_oracle"] = float(e)
    if not args.no_extras:
        del t_in, ws
        torch.cuda.empty_cache()
        log("[bench] adjoint leg")
        out["adjoint"] = adjoint_leg(gpp, I, stream)
        log("[bench] batched leg")
        out["batched"] = batched_leg(gpp, I, stream)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded slice")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
