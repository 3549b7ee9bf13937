"""Empirical ceilings on this GPU: fp64 FMA rate, streaming-copy
bandwidth and the read bandwidth of vL1D, L2, MALL and HBM
(include/gpp_microbench.h).  Prints one JSON line.

    python -m paper_2008_11326_amd.microbench [--copy-mib 2048]
    python -m paper_2008_11326_amd.microbench --lds-only

The copy moves exactly 2 * bytes (read + write); under rocprofv3 --pmc its
FETCH_SIZE / WRITE_SIZE give the factor between counted and real bytes.
With --lds-only it launches the four LDS access patterns once each, in
pattern order (one dispatch of gpp::mb_lds per pattern), for the
bank-conflict counters.
"""
import argparse
import ctypes as C
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--fma-iters", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-read-levels", dest="read_levels", action="store_false",
                    help="skip the per-level read-bandwidth kernels")
    ap.add_argument("--lds-only", action="store_true",
                    help="only the LDS access patterns, one launch each")
    args = ap.parse_args()

    import torch

    from . import _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(args.reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(st)
            fn()
            b.record(st)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        return best

    res = {"device": props.name, "compute_units": cus}
    if args.lds_only:
        blocks, reps = 64, 4096
        out = torch.empty(blocks * 64, dtype=torch.float64, device=dev)
        for pattern in range(4):
            _lib.check(lib.gpp_mb_lds(pattern, blocks, reps, C.c_void_p(out.data_ptr()),
                                      C.c_void_p(st.cuda_stream)), "gpp_mb_lds")
        torch.cuda.synchronize()
        res["lds_patterns"] = {"blocks": blocks, "reps": reps,
                               "lds_instructions_per_pattern": blocks * reps * 8}
        print(json.dumps(res), flush=True)
        return
    fma = {}
    for waves_per_simd in (2, 4, 8):
        blocks = cus * waves_per_simd  # 4 waves per workgroup
        out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
        flops = C.c_double(0.0)

        def run():
            _lib.check(lib.gpp_mb_fp64_fma(C.c_void_p(out.data_ptr()), blocks,
                                           args.fma_iters, C.c_void_p(st.cuda_stream),
                                           C.byref(flops)), "gpp_mb_fp64_fma")
        ms = timed(run)
        fma[str(waves_per_simd)] = round(flops.value / (ms * 1e-3) / 1e12, 3)
    res["fp64_fma_tflops_by_waves_per_simd"] = fma
    res["fp64_fma_tflops"] = max(fma.values())

    nbytes = args.copy_mib << 20
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    src.fill_(1)

    def copy():
        _lib.check(lib.gpp_mb_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                   nbytes, cus * 8, C.c_void_p(st.cuda_stream)),
                   "gpp_mb_copy")
    ms = timed(copy)
    res["copy_bytes_each_way"] = nbytes
    res["copy_ms"] = round(ms, 4)
    res["copy_gbps_read_plus_write"] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del src, dst

    if args.read_levels:
        # (shared, window bytes, workgroups per CU, reps) per level
        levels = {
            "vl1d": (0, 4 << 10, 4, 4096),    # 4 x 4 KiB per CU: inside the 32 KiB L1
            "l2": (1, 2 << 20, 8, 8),         # one 2 MiB window: inside each XCD's L2
            "mall": (1, 64 << 20, 8, 1),      # 64 MiB: beyond the L2s, inside the MALL
            "hbm": (0, 2 << 20, 8, 2),        # 2 MiB per workgroup, 4 GiB in all
        }
        read = {}
        for name, (shared, win, per_cu, reps) in levels.items():
            blocks = cus * per_cu
            nbuf = win if shared else win * blocks
            buf = torch.ones(nbuf // 8, dtype=torch.float64, device=dev)
            out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)

            def rd():
                _lib.check(lib.gpp_mb_read(C.c_void_p(buf.data_ptr()), win, shared, blocks,
                                           reps, C.c_void_p(out.data_ptr()),
                                           C.c_void_p(st.cuda_stream)), "gpp_mb_read")
            ms = timed(rd)
            read[name] = round(blocks * win * reps / (ms * 1e-3) / 1e12, 2)
            del buf, out
        res["read_tbps"] = read
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
