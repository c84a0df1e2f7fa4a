"""Host logic of bench.py (no GPU): the trace summary of a rocprofv3 kernel
trace, the readers of the committed counter summaries, and the algorithmic
byte counts behind the roofline entry."""
import csv
import os

import pytest

import bench
from paper_2209_09671_amd import inputs as I

NS = "void tcf::(anonymous namespace)::"


def write_trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, a, b in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": a, "End_Timestamp": b})


def test_trace_summary_takes_the_last_steps(tmp_path):
    # three steps of: transport x3 (10 us each) and one solve kernel (5 us);
    # the window of the last two steps starts at step 2's first transport
    rows, t = [], 0
    for step in range(3):
        for _ in range(3):
            rows.append((NS + "k_transport2<float, 3, 1>(int)", t, t + 10_000))
            t += 12_000
        rows.append((NS + "k0_smooth2<float, true, 8>(int)", t, t + 5_000 * (step + 1)))
        t += 20_000
    p = tmp_path / "trace.csv"
    write_trace(p, rows)
    out = bench.trace_summary(str(p), 2)
    assert "the last 2 steps, 8 dispatches" in out
    lines = {l.split("|")[1].strip(): l for l in out.splitlines() if l.startswith("| k")}
    # transport: 3 calls per step at 10 us; the sweep: 10 and 15 us in steps 2 and 3
    assert "| 3.00 | 10.00 | 0.030 |" in lines["k_transport2<float, 3, 1>"]
    assert "| 1.00 | 12.50 | 0.013 |" in lines["k0_smooth2<float, true, 8>"]


def test_trace_summary_adjoint_window(tmp_path):
    rows = [(NS + "k_transport2<double, 3, 1>(int)", 0, 1000),
            (NS + "ka_pred_dir<3, 0, 1>(int)", 2000, 4000),
            (NS + "k0_smooth<double, 3, false>(int)", 5000, 6000),
            (NS + "ka_transport_cell<3>(int)", 7000, 9000),
            (NS + "k_copy64(int)", 10000, 11000)]
    p = tmp_path / "trace.csv"
    write_trace(p, rows)
    out = bench.trace_summary(str(p), 1, adjoint=True)
    # from the first to the last adjoint kernel: three dispatches, 7 us of span
    assert "the backward sweep of 1 adjoint steps, 3 dispatches, span 0.007 ms" in out
    assert "k_copy64" not in out and "k_transport2" not in out


def test_counter_readers_follow_the_source_hash(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "counters_smooth2_w.md").write_text(
        f"x\nkernel_source_sha256_16: {h}\nhbm_bytes_per_launch: 3.0e+08\n")
    (tmp_path / "profiles" / "sq_valu_w.md").write_text(
        "| kernel | d | us | v | busy | s | l |\n|---|---|---|---|---|---|---|\n"
        "| k0_smooth2<float, true, 8> | 50 | 96.5 | 4.3e+07 | 74% | 2.2e+07 | 6.7e+06 |\n"
        f"\nkernel_source_sha256_16: {h}\n")
    assert bench.measured_traffic("smooth2", "w") == 3.0e8
    assert bench.measured_valu_busy("k0_smooth2<float,true,8>", "w") == pytest.approx(0.74)
    assert bench.measured_valu_busy("k_transport2<float,3,1>", "w") is None
    # a summary taken on other kernel sources is not used
    (tmp_path / "profiles" / "counters_smooth2_w.md").write_text(
        "kernel_source_sha256_16: 0000000000000000\nhbm_bytes_per_launch: 3.0e+08\n")
    assert bench.measured_traffic("smooth2", "w") is None
    assert bench.measured_traffic("transport", "w") is None


def test_committed_summaries_parse():
    """The committed summaries carry a hash and a per-launch figure in the
    form the readers expect (whether or not they match these sources)."""
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")
    for fam in ("smooth2", "smooth", "transport"):
        txt = open(os.path.join(root, f"counters_{fam}_meltpool256.md")).read()
        assert "kernel_source_sha256_16:" in txt and "hbm_bytes_per_launch:" in txt
    assert "kernel_source_sha256_16:" in open(os.path.join(root, "sq_valu_meltpool256.md")).read()


def test_algorithmic_bytes_of_the_roofline_families():
    c = I.config(4)
    N = 256 ** 3
    assert bench.algorithmic_bytes("smooth2", c) == N * 4 * (4 + 1 / 8)
    assert bench.algorithmic_bytes("smooth", c) == N * 4 * 4
    # the predictor family is one timed launch of its three component kernels
    assert bench.algorithmic_bytes("predictor", c) == N * 4 * 3 * 7
    # a step moves more than its dominant kernel family
    assert bench.step_bytes_per_cell(6.7, 1.7, 1) > 4 * (4 + 1 / 8)


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
