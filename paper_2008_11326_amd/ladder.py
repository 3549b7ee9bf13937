"""The paper's optimisation steps (Sec. III v0-v8, Table I) replayed on
MI355X: binding of include/gpp_ladder.h and a measurement driver.

    python -m paper_2008_11326_amd.ladder [--workload adjoint] [--reps 3]
        [--steps 0,1,...]

prints one JSON line per step: time per call (HIP events on the launch
stream, median of --reps after one warm-up call), algorithmic TFLOP/s (21
fp64 operations per term, as in bench.py), the fraction of the 78.6 TFLOP/s
fp64 vector peak, the speed-up over the previous step and the largest
relative error against the oracle's stored outputs for the workload
(tests/golden).  Inputs are the workload's seeded synthetic draws, resident
on the device before timing.
"""
import argparse
import ctypes as C
import json
import os
import sys

from . import _lib
from . import _check_tensor, _prepare, _ptr, _torch

FLOP_PER_TERM = 21
FP64_VECTOR_PEAK_TFLOPS = 78.6


def ladder_steps() -> int:
    return int(_lib.load().gpp_ladder_steps())


def ladder_name(step: int) -> str:
    name = _lib.load().gpp_ladder_name(int(step))
    if name is None:
        raise ValueError(f"no ladder step {step}")
    return name.decode()


def ladder_workspace_bytes(step, number_bands, nvband, ncouls, ngpown, nfreq) -> int:
    dims = _lib.dims_struct(number_bands, nvband, ncouls, ngpown, nfreq)
    return int(_lib.load().gpp_ladder_workspace(int(step), C.byref(dims)))


def ladder_fwd(step, aqsmtemp, aqsntemp, I_eps_array, wtilde_array, vcoul, wx_array,
               nvband: int, *, out=None, workspace=None, stream=None):
    """achtemp, asxtemp computed by ladder step `step` (gpp_ladder_fwd);
    arguments as sigma_fwd."""
    torch = _torch()
    lib = _lib.load()
    dims, ins, dev = _prepare(aqsmtemp, aqsntemp, I_eps_array, wtilde_array,
                              vcoul, wx_array, nvband)
    nw = dims.nfreq
    if out is None:
        ach = torch.empty(nw, dtype=torch.complex128, device=dev)
        asx = torch.empty(nw, dtype=torch.complex128, device=dev)
    else:
        ach, asx = out
        _check_tensor("achtemp", ach, torch.complex128, (nw,), dev)
        _check_tensor("asxtemp", asx, torch.complex128, (nw,), dev)
    if workspace is None:
        need = int(lib.gpp_ladder_workspace(int(step), C.byref(dims)))
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        st = lib.gpp_ladder_fwd(int(step), C.byref(dims), C.byref(ins), _ptr(ach), _ptr(asx),
                                _ptr(workspace), workspace.numel(), C.c_void_p(stream))
    _lib.check(st, "gpp_ladder_fwd")
    return ach, asx


def _stored_outputs(key):
    """The oracle's outputs for a workload as stored under tests/golden (a
    JSON data file written by the oracle), or None."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "tests", "golden", f"fwd_{key}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _rel_err(got, ref_pairs, abs_sum):
    """Largest per-entry complex-modulus error relative to the reference
    entry (to abs_sum for a zero entry)."""
    worst = 0.0
    for z, (re, im) in zip(got, ref_pairs):
        ref = complex(re, im)
        worst = max(worst, abs(complex(z) - ref) / (abs(ref) if ref != 0 else abs_sum + 1e-300))
    return worst


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="adjoint")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--steps", default=None, help="comma-separated subset")
    args = ap.parse_args(argv)

    import numpy as np
    torch = _torch()
    from . import inputs as I

    wl = I.WORKLOADS[args.workload]
    d = wl.dims
    prob = I.make_problem(d, wl.seed, wl.pole_fraction)
    dev = torch.device("cuda:0")
    t_in = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in prob.arrays()]
    gold = _stored_outputs(args.workload)
    stream = torch.cuda.current_stream(dev)
    flops = FLOP_PER_TERM * (d.ch_terms + d.sx_terms)
    steps = (range(ladder_steps()) if args.steps is None
             else [int(s) for s in args.steps.split(",")])
    prev = None
    for step in steps:
        ws = torch.empty(max(1, ladder_workspace_bytes(step, *d.as_tuple())),
                         dtype=torch.uint8, device=dev)
        ach = torch.empty(d.nfreq, dtype=torch.complex128, device=dev)
        asx = torch.empty_like(ach)

        def call():
            ladder_fwd(step, *t_in, nvband=d.nvband, out=(ach, asx), workspace=ws,
                       stream=stream.cuda_stream)
        print(f"[ladder] step {step}: {ladder_name(step)}", file=sys.stderr, flush=True)
        call()
        torch.cuda.synchronize()
        times = []
        for _ in range(args.reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            call()
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ms = sorted(times)[len(times) // 2]
        rec = {"step": step, "name": ladder_name(step), "workload": wl.name,
               "ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
               "pct_fp64_peak": round(100 * flops / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                                      2),
               "speedup_vs_previous": None if prev is None else round(prev / ms, 3)}
        if gold is not None:
            rec["max_rel_err_vs_oracle"] = max(
                _rel_err(ach.cpu().numpy(), gold["achtemp"], gold["ach_abs_sum"]),
                _rel_err(asx.cpu().numpy(), gold["asxtemp"], gold["asx_abs_sum"]))
        print(json.dumps(rec), flush=True)
        prev = ms
        del ws


if __name__ == "__main__":
    main()
