"""Write full-size expected outputs with the CPU oracle.

Calls only the oracle (and the shared seeded input generator); no value in
the files it writes comes from the HIP path.  Usage:

    python tests/golden/make_golden.py si adjoint [--threads 8]
    python tests/golden/make_golden.py batched --states 0-63

Each workload writes tests/golden/fwd_<key>.json with achtemp/asxtemp
(complex [nfreq] as [re, im] pairs), the sums of |term| (for the condition
number) and the oracle source digest, so a changed oracle is visible.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2008_11326_amd import inputs as I  # noqa: E402


def oracle_digest() -> str:
    h = hashlib.sha256()
    for name in ("gpp_oracle.c",):
        with open(os.path.join(ROOT, "oracle", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _pairs(z):
    return [[float(v.real), float(v.imag)] for v in z]


def run_one(prob, threads):
    t0 = time.time()
    ach, asx, ach_abs, asx_abs = oracle.sigma_fwd(prob, nthreads=threads)
    return {
        "achtemp": _pairs(ach), "asxtemp": _pairs(asx),
        "ach_abs_sum": [float(v) for v in ach_abs],
        "asx_abs_sum": [float(v) for v in asx_abs],
        "oracle_seconds": round(time.time() - t0, 2), "threads": threads,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("keys", nargs="+")
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--states", default="0-63")
    a = ap.parse_args()
    for key in a.keys:
        if key == "batched":
            lo, hi = (int(v) for v in a.states.split("-"))
            path = os.path.join(HERE, "fwd_batched.json")
            doc = {"seed": I.BATCHED_SEED, "oracle": oracle_digest(),
                   "states": {}}
            if os.path.exists(path):
                with open(path) as f:
                    doc = json.load(f)
            for s, prob in I.make_batched(states=range(lo, hi + 1)):
                rec = run_one(prob, a.threads)
                rec["dims"] = list(prob.dims.as_tuple())
                doc["states"][str(s)] = rec
                with open(path, "w") as f:
                    json.dump(doc, f, indent=1)
                print(f"batched state {s} {prob.dims} {rec['oracle_seconds']}s",
                      flush=True)
            continue
        wl = I.WORKLOADS[key]
        prob = I.make_problem(wl.dims, wl.seed, wl.pole_fraction)
        rec = run_one(prob, a.threads)
        rec.update({"workload": wl.name, "dims": list(wl.dims.as_tuple()),
                    "seed": wl.seed, "pole_fraction": wl.pole_fraction,
                    "oracle": oracle_digest()})
        with open(os.path.join(HERE, f"fwd_{key}.json"), "w") as f:
            json.dump(rec, f, indent=1)
        print(f"{key}: {rec['oracle_seconds']}s", flush=True)


if __name__ == "__main__":
    main()
