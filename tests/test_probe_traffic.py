"""Host logic of the counter-to-traffic tool: per-dispatch reading, the scale
from the copy kernel, and dropping launches that ran no correlation pass."""
from __future__ import annotations

import json
import subprocess
import sys

from paper_0809_1833_amd.probe import traffic

HEAD = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"


def _csv(path, rows):
    path.write_text(HEAD + "".join(f"{d},{k},X,{v}\n" for d, k, v in rows))


def test_pass_positions_drops_small_launches():
    assert traffic.pass_positions([100.0, 101.0, 0.6, 99.0], 0.5) == [0, 1, 3]
    assert traffic.pass_positions([5.0, 5.0], 0.5) == [0, 1]


def test_tool_scales_and_filters(tmp_path):
    f, w = tmp_path / "f", tmp_path / "w"
    f.mkdir(), w.mkdir()
    # copy kernel: 1 MiB known; FETCH reads half the bytes, WRITE all of them
    _csv(f / "copy_counter_collection.csv", [(1, "k_copy", 512.0)])
    _csv(w / "copy_counter_collection.csv", [(1, "k_copy", 1024.0)])
    # dispatch ids out of order in the file; the 3rd launch ran no pass
    _csv(f / "bench_counter_collection.csv",
         [(12, "mp::k_step(x)", 1.0), (10, "mp::k_step(x)", 100.0), (11, "mp::k_step(x)", 100.0),
          (13, "other", 7.0)])
    _csv(w / "bench_counter_collection.csv",
         [(12, "mp::k_step(x)", 9.0), (10, "mp::k_step(x)", 2.0), (11, "mp::k_step(x)", 4.0)])
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    out = tmp_path / "t.json"
    subprocess.run([sys.executable, "-m", "paper_0809_1833_amd.probe.traffic", "--kernel", "k_step",
                    "--source", str(src), "--n", "4", "--m", "8", "--fetch", str(f), "--write",
                    str(w), "--copy-bytes", str(1 << 20), "--algorithmic-bytes", "207872",
                    "--pass-only", "0.5", "--out", str(out)], check=True, capture_output=True)
    d = json.loads(out.read_text())
    assert d["dispatches"] == {"fetch": 2, "write": 2, "dropped_without_pass": 1}
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    assert d["fetch_bytes_per_launch"] == 100 * 1024 * 2
    assert d["write_bytes_per_launch"] == 3 * 1024
    assert d["traffic_over_algorithmic"] == 1.0
    assert d["kernel_sha"] == traffic.source_sha([str(src)])


def test_pmc_summary_means_per_dispatch(tmp_path):
    from paper_0809_1833_amd.probe import pmc_summary
    p = tmp_path / "b_counter_collection.csv"
    p.write_text("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
                 "1,void mp::k_a<4>(int),X,10\n1,void mp::k_a<4>(int),Y,2\n"
                 "2,void mp::k_a<4>(int),X,30\n2,void mp::k_a<4>(int),Y,4\n"
                 "3,mp::k_b(int),X,5\n")
    d = pmc_summary.summarize(str(p), ["k_a"])
    assert list(d) == ["void mp::k_a<4>"]
    assert d["void mp::k_a<4>"] == {"dispatches": 2, "mean_per_dispatch": {"X": 20.0, "Y": 3.0}}
