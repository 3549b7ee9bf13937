"""Host checks of bench.py's measurement logic: the counted-FLOP formula
(64 lanes per wave instruction, an FMA counting 2), the FMA share and its
ceiling (the closing FMA-ratio paragraph of Sec. III: with a share f of
FMAs, a machine that issues one instruction per slot reaches (2f + 1 - f)/2
of the FMA peak), and that committed counter records are used only while
the forward sources hash to the digest they were taken with."""
import json
import os

import pytest

import bench


def test_counted_flops_and_fma_share():
    rec = {"valu_f64": {"add": 10.0, "mul": 20.0, "fma": 30.0, "trans": 4.0}}
    flops, f = bench.counted_fp64(rec)
    assert flops == 64 * (10 + 20 + 4 + 2 * 30)
    assert f == 30.0 / 60.0
    # the paper's own figures: a 58 % FMA share gives a 79 % ceiling
    f = 0.58
    assert abs((2 * f + (1 - f)) / 2 - 0.79) < 1e-12


def test_counter_records_follow_the_source_digest(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    csrc = tmp_path / "paper_2008_11326_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.FWD_SOURCES:
        (csrc / name).write_text(f"// {name}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    digest = bench.fwd_source_digest()
    rec = {"workload": "w", "source_digest": digest, "traffic_bytes": 5,
           "valu_f64": {"add": 1, "mul": 1, "fma": 1, "trans": 0}}
    (prof / "gpp_fwd_tiles_w.json").write_text(json.dumps(rec))
    got = bench.kernel_counters("w")
    assert got is not None and got["path"] == os.path.join("profiles", "gpp_fwd_tiles_w.json")
    assert bench.kernel_counters("other") is None
    # a comment edit keeps the record, a code edit drops it
    (csrc / bench.FWD_SOURCES[0]).write_text(f"// {bench.FWD_SOURCES[0]}, reworded\n/* and */\n")
    assert bench.kernel_counters("w") is not None
    (csrc / bench.FWD_SOURCES[0]).write_text("int x;\n")
    assert bench.kernel_counters("w") is None


def test_multi_gpu_request_exits_with_a_message(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
