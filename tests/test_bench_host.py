"""Host-side pieces of the benchmark and the profile summaries (no GPU).

* bench.py refuses more than one GPU with a JSON message and status 2;
* profsum's per-template cards on a synthetic rocprofv3 trace and counter
  set: average duration, VALU counts per dispatch, and HBM bytes scaled by
  the plain elementwise kernel (FETCH_SIZE reads 2x low in this synthetic
  set, as on the device);
* the committed counter summaries carry cards for the benchmark's dominant
  kernels, and bench.py finds them when the sources hash to their value.
"""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_profsum_cards(tmp_path):
    from paper_2308_15020_amd import profsum
    kname = "void ffsat::k_pull<4, 4, true>(ffsat::PullArgs, float const*)"
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg>(int)"
    trace = tmp_path / "trace.csv"
    # two dispatches of 10 and 30 us
    _write(trace, ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Dispatch_Id", "Start_Timestamp", "End_Timestamp"],
           [[kname, 800000, 1, 1, 1000, 11000], [kname, 800000, 1, 2, 20000, 50000]])
    hdr = ["Kernel_Name", "Grid_Size", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    sq = tmp_path / "sq.csv"
    _write(sq, hdr, [[kname, 800000, 1, "SQ_INSTS_VALU", 100], [kname, 800000, 2, "SQ_INSTS_VALU", 300],
                     [kname, 800000, 1, "SQ_ACTIVE_INST_VALU", 110], [kname, 800000, 2, "SQ_ACTIVE_INST_VALU", 310]])
    fe = tmp_path / "fetch.csv"
    # the plain kernel of 256 MiB reads as 128 MiB (2x low): scale 2
    _write(fe, hdr, [[copy, 16777216, 9, "FETCH_SIZE", 131072], [kname, 800000, 1, "FETCH_SIZE", 1000],
                     [kname, 800000, 2, "FETCH_SIZE", 3000]])
    wr = tmp_path / "write.csv"
    _write(wr, hdr, [[copy, 16777216, 9, "WRITE_SIZE", 262144], [kname, 800000, 1, "WRITE_SIZE", 500],
                     [kname, 800000, 2, "WRITE_SIZE", 500]])
    out = profsum.cards(str(trace), str(sq), str(fe), str(wr), 256, ["k_pull<4, 4, true>"])
    card = json.loads(out.split("card: ", 1)[1])
    assert card["kernel_name"] == "k_pull<4, 4, true>"
    assert card["rocprof_avg_us"] == 20.0 and card["rocprof_dispatches"] == 2
    assert card["valu_insts_per_launch"] == 200.0 and card["valu_active_per_launch"] == 210.0
    assert card["read_bytes_per_launch"] == 2000 * 1024 * 2
    assert card["write_bytes_per_launch"] == 500 * 1024
    assert card["traffic_bytes_per_launch"] == 2000 * 1024 * 2 + 500 * 1024
    assert card["source_sha256"] == profsum.kernel_source_hash()


def test_profsum_family_card(tmp_path):
    """The per-bin FP64 root-of-unity kernels (one template per segment
    shape) also get one card as a family: average over all their dispatches."""
    from paper_2308_15020_amd import profsum
    a = "void ffsat::k_eval<float, double, 16, 16, true>(ffsat::EvalArgs<float>)"
    b = "void ffsat::k_eval<float, double, 32, 16, true>(ffsat::EvalArgs<float>)"
    trace = tmp_path / "trace.csv"
    _write(trace, ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Dispatch_Id", "Start_Timestamp", "End_Timestamp"],
           [[a, 1000, 1, 1, 0, 10000], [b, 2000, 1, 2, 20000, 50000], [a, 1000, 1, 3, 60000, 70000]])
    hdr = ["Kernel_Name", "Grid_Size", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    sq = tmp_path / "sq.csv"
    _write(sq, hdr, [[a, 1000, 1, "SQ_INSTS_VALU", 100], [b, 2000, 2, "SQ_INSTS_VALU", 400],
                     [a, 1000, 3, "SQ_INSTS_VALU", 100]])
    fam = "k_eval<float, double, *, *, true>"
    assert profsum.family_of("k_eval<float, double, 32, 16, true>") == fam
    assert profsum.family_of("k_eval<float, float, 16, 4, false>") is None
    out = profsum.cards(str(trace), str(sq), str(sq), str(sq), 256, [fam])
    card = json.loads(out.split("card: ", 1)[1])
    assert card["rocprof_dispatches"] == 3 and card["rocprof_avg_us"] == 16.67   # (10 + 30 + 10) / 3 us
    assert card["valu_insts_per_launch"] == 200.0
    assert "family" in profsum.trace(str(trace))


@pytest.mark.parametrize("workload,kernel", [("large", "k_eval_group64"),
                                             ("large3sat", "k_pull<4, 4, true>"),
                                             ("mixed2000", "k_eval_group")])
def test_committed_cards_cover_dominant_kernels(workload, kernel):
    path = os.path.join(ROOT, "profiles", f"eval_step_{workload}_counters.txt")
    cards = [json.loads(l[len("card: "):]) for l in open(path) if l.startswith("card: ")]
    c = [c for c in cards if c["kernel_name"] == kernel]
    assert len(c) == 1
    for key in ("rocprof_avg_us", "valu_insts_per_launch", "traffic_bytes_per_launch", "source_sha256"):
        assert key in c[0]
    sys.path.insert(0, ROOT)
    import bench
    from paper_2308_15020_amd.profsum import kernel_source_hash
    got = bench.kernel_card(workload, kernel)
    if c[0]["source_sha256"] == kernel_source_hash():
        assert got == c[0]
    else:
        assert got is None   # stale counters are never reported
