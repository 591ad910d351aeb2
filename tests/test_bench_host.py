"""Host logic of bench.py that needs no GPU: the one-GPU guard, the rocprofv3
summary writer (kernel statistics, the numeric phase span, HBM bytes scaled
by the calibration kernels) and the traffic lookup that drops counters
taken on another kernel source."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KIB_PER_GIB = 1 << 20


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=header)
        w.writeheader()
        w.writerows(rows)


def _counters(d, counter, per_kernel):
    rows = [{"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v}
            for k, vals in per_kernel.items() for v in vals]
    _write_csv(os.path.join(d, "host", "1_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
               rows)


@pytest.fixture
def profile_dirs(tmp_path):
    trace = tmp_path / "trace"
    _write_csv(str(trace / "host" / "1_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
               [{"Name": "void dibella::k_ov_numeric<256>(Args)", "Calls": 4, "TotalDurationNs": 400000,
                 "AverageNs": 100000, "Percentage": 80.0},
                {"Name": "void dibella::k_tr_mark<128, 0>(Args)", "Calls": 4, "TotalDurationNs": 100000,
                 "AverageNs": 25000, "Percentage": 10.0},
                {"Name": "void dibella::k_tr_mark<128, 1>(Args)", "Calls": 2, "TotalDurationNs": 20000,
                 "AverageNs": 10000, "Percentage": 2.0},
                {"Name": "dibella::k_ov_write_rowptr(Args)", "Calls": 2, "TotalDurationNs": 6000,
                 "AverageNs": 3000, "Percentage": 0.5},
                {"Name": "dibella::k_tr_init_state(Args)", "Calls": 2, "TotalDurationNs": 4000,
                 "AverageNs": 2000, "Percentage": 0.4},
                {"Name": "void at::native::vectorized_elementwise_kernel<4>(Args)", "Calls": 9,
                 "TotalDurationNs": 900000, "AverageNs": 100000, "Percentage": 70.0}])
    # two overlap calls: the first one's numeric launches overlap on three
    # streams (span 10 us .. 80 us), the second has a single launch of 20 us
    ev = [("k_ov_write_rowptr", 0, 5000), ("k_ov_numeric<256>", 10000, 50000),
          ("k_ov_numeric<1024>", 20000, 80000), ("k_ov_numeric<4096>", 30000, 60000),
          ("k_tr_mark<0>", 90000, 95000), ("k_ov_write_rowptr", 100000, 105000),
          ("k_ov_numeric<256>", 110000, 130000)]
    _write_csv(str(trace / "host" / "1_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [{"Kernel_Name": f"void {n}(Args)", "Start_Timestamp": a, "End_Timestamp": b} for n, a, b in ev])
    # calibration: the copy kernel's 1 GiB read counts as 0.5 GiB in
    # FETCH_SIZE (two dispatches, mean taken), its 1 GiB write as 1.25 GiB
    _counters(str(tmp_path / "cfetch"), "FETCH_SIZE",
              {"void (anonymous namespace)::k_calib_copy(float4 const*, float4*, long)":
                   [0.4 * KIB_PER_GIB, 0.6 * KIB_PER_GIB],
               "(anonymous namespace)::k_calib_read(float4 const*, long, float*)": [0.5 * KIB_PER_GIB],
               "void (anonymous namespace)::k_calib_stride<64>(float const*, long, float*)": [0.5 * KIB_PER_GIB]})
    _counters(str(tmp_path / "cwrite"), "WRITE_SIZE",
              {"void (anonymous namespace)::k_calib_copy(float4 const*, float4*, long)": [1.25 * KIB_PER_GIB],
               "(anonymous namespace)::k_calib_write(float4*, long, float)": [1.0 * KIB_PER_GIB]})
    _counters(str(tmp_path / "fetch"), "FETCH_SIZE",
              {"void k_ov_write_rowptr(Args)": [1.0, 1.0],
               "void k_ov_numeric<256>(Args)": [1000.0, 3000.0],
               "void k_ov_numeric<1024>(Args)": [2000.0],
               "void k_ov_seg_slices(Args)": [500.0], "void k_ov_scatter(Args)": [250.0]})
    _counters(str(tmp_path / "write"), "WRITE_SIZE",
              {"void k_ov_write_rowptr(Args)": [1.0, 1.0],
               "void k_ov_numeric<256>(Args)": [100.0, 300.0],
               "void k_ov_numeric<1024>(Args)": [200.0],
               "void k_ov_seg_slices(Args)": [50.0], "void k_ov_scatter(Args)": [25.0]})
    return tmp_path


def test_summaries_from_synthetic_rocprof_output(profile_dirs):
    p = profile_dirs
    out = str(p / "out")
    bench.summarize_profiles(str(p / "trace"), str(p / "fetch"), str(p / "write"), str(p / "cfetch"),
                             str(p / "cwrite"), "t", "python3 bench.py --steps 2", out_dir=out)
    text = open(os.path.join(out, "kernels_t_trace.txt")).read()
    assert "# command: python3 bench.py --steps 2" in text
    # library kernels first, each sorted by total time, then the others
    assert text.index("k_ov_numeric") < text.index("k_tr_mark<128, 0>") < text.index("k_tr_mark<128, 1>")
    assert text.index("## library kernels") < text.index("k_tr_init_state") < text.index("## other kernels")
    assert text.index("## other kernels") < text.index("vectorized_elementwise_kernel")
    # per call: two overlap calls, two reduction calls; a unit sums all of
    # its kernels' launches
    block = text[text.index("## timed units"):].split("\n\n")[0].splitlines()[2:]
    units = {ln.split()[0]: ln.split()[2:4] for ln in block}
    assert "(2 overlap calls, 2 reduction calls)" in text
    assert units["tr_mark"] == ["3.0", "0.060"]        # 6 launches, 120 us over 2 calls
    assert units["numeric"] == ["2.0", "0.200"]        # 4 launches, 400 us over 2 calls
    assert "keys" not in units
    # spans 70 us and 20 us, 3 and 1 launches per call
    assert "2 calls, 2.0 launches per call, span avg_us 45.00" in text

    num = json.load(open(os.path.join(out, "numeric_t_pmc.json")))
    f_read, f_write = 0.5, 1.25                          # the copy kernel, mean of its dispatches
    assert num["read_calibration_factor"] == pytest.approx(f_read)
    assert num["write_calibration_factor"] == pytest.approx(f_write)
    assert num["calibration_kernel"] == "k_calib_copy"
    refs = num["reference_kernels"]
    assert refs["k_calib_read"]["fetch_factor"] == pytest.approx(0.5)
    assert refs["k_calib_write"]["write_factor"] == pytest.approx(1.0)
    # one 4-byte touch per 64 bytes over 1 GiB: 2^24 touches of 4 bytes
    assert refs["k_calib_stride<64>"]["fetch_factor"] == pytest.approx(0.5 * (1 << 30) / ((1 << 24) * 4))
    assert refs["k_calib_stride<128>"]["fetch_factor"] is None or refs["k_calib_stride<128>"]["FETCH_SIZE_bytes"] == 0
    # mean over the dispatches of the one kernel name, KiB -> bytes, / factor
    assert num["hbm_read_bytes_per_launch"] == pytest.approx(2000.0 * 1024 / f_read)
    assert num["hbm_write_bytes_per_launch"] == pytest.approx(200.0 * 1024 / f_write)
    assert num["overlap_calls"] == 2
    assert num["hbm_bytes_per_phase"] == pytest.approx((6000.0 * 1024 / f_read + 600.0 * 1024 / f_write) / 2)
    assert num["source_hash"] == bench.source_hash("overlap.hip")
    # a unit of two kernels sums one dispatch of each
    seg = json.load(open(os.path.join(out, "segments_t_pmc.json")))
    assert seg["kernel"] == "k_ov_seg_slices+k_ov_scatter"
    assert seg["hbm_bytes_per_launch"] == pytest.approx(750.0 * 1024 / f_read + 75.0 * 1024 / f_write)
    # kernels without counters get no summary
    assert not os.path.exists(os.path.join(out, "tr_mark_t_pmc.json"))
    assert not os.path.exists(os.path.join(out, "keys_t_pmc.json"))

    h = bench.source_hash("overlap.hip")
    assert bench.load_traffic("numeric_phase", "t", h, profiles=out) == pytest.approx(num["hbm_bytes_per_phase"])
    assert bench.load_traffic("numeric", "t", h, profiles=out) == pytest.approx(num["hbm_bytes_per_launch"])
    # counters taken on another source are not reported
    assert bench.load_traffic("numeric_phase", "t", "0" * 16, profiles=out) is None
    assert bench.load_traffic("tr_mark", "t", h, profiles=out) is None


def test_summaries_skip_counters_without_calibration(tmp_path, profile_dirs):
    p = profile_dirs
    out = str(p / "out2")
    empty = str(tmp_path / "none")
    os.makedirs(empty)
    bench.summarize_profiles(str(p / "trace"), str(p / "fetch"), str(p / "write"), empty, empty, "t", "",
                             out_dir=out)
    assert os.path.exists(os.path.join(out, "kernels_t_trace.txt"))
    assert not any(n.endswith("_pmc.json") for n in os.listdir(out))


def test_committed_summaries_are_well_formed():
    d = bench.PROFILES
    pmcs = [n for n in os.listdir(d) if n.endswith("_pmc.json")]
    assert pmcs
    for n in pmcs:
        s = json.load(open(os.path.join(d, n)))
        assert s["command"] and s["kernel"] and len(s["source_hash"]) == 16
        assert s["hbm_bytes_per_launch"] == pytest.approx(s["hbm_read_bytes_per_launch"]
                                                          + s["hbm_write_bytes_per_launch"])
        assert 0.25 < s["read_calibration_factor"] < 2 and 0.25 < s["write_calibration_factor"] < 2
        assert s["calibration_kernel"] == "k_calib_copy"


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
