"""Build libgpp.so (HIP, gfx950 only) in-tree.

    python -m paper_2008_11326_amd.build        # or build() from Python
    python -m paper_2008_11326_amd.build --define GPP_FWD_COLS=1 --out $VDIR/libgpp_c1.so

The second form builds a variant with compile-time tuning knobs (the
GPP_* macros the sources document) into a library of its own, for
measurement; the package loads it when GPP_LIBRARY names it.

Each .hip source compiles to an object with hipcc for gfx950, then they
link into paper_2008_11326_amd/libgpp.so.  Packed-fp32 instructions are
disabled for all device code.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgpp.so")
SOURCES = ["gpp_api.hip", "gpp_fwd.hip", "gpp_bwd.hip", "gpp_batched.hip", "gpp_plan.hip",
           "gpp_ladder.hip", "gpp_noalloc.hip",
           "gpp_microbench.hip"]
HEADERS = ["gpp_device.h", "gpp_fwd_tile.h", "gpp_fwd_shape.h", "gpp_internal.h"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}",
]


def _compile(src: str, verbose: bool, objdir: str = OBJDIR, defines=()) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; drop that note
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err and verbose:
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False, defines=(), out: str = LIB) -> str:
    """Compile every HIP source for gfx950 and link libgpp.so (always
    rebuilds).  With defines (NAME=VALUE strings) the objects go to a
    directory of their own next to `out`, which must then be given too."""
    if defines and os.path.abspath(out) == LIB:
        raise ValueError("a variant build needs its own output path")
    objdir = OBJDIR if not defines else os.path.splitext(os.path.abspath(out))[0] + "_obj"
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, objdir, defines), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    files = [os.path.join(CSRC, f) for f in SOURCES + HEADERS]
    files += [os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE)]
    return any(os.path.getmtime(f) > t for f in files)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="build libgpp.so for gfx950")
    ap.add_argument("--define", action="append", default=[], metavar="NAME=VALUE")
    ap.add_argument("--out", default=LIB)
    a = ap.parse_args()
    build(verbose=True, defines=a.define, out=a.out)
