"""CPU checks of bench.py's host logic: the one-GPU rule, the Philox ALU peak, the roofline
arithmetic and the copy calibration of the HBM traffic counters."""

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    import bench as B

    return B


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_philox_peak_from_unit_counts(bench):
    # 10 rounds x (2 v_mad_u64_u32 + 4 v_xor_b32), one lane slot each
    assert bench.PHILOX_SLOTS == 10 * (2 + 4)
    assert bench.PHILOX_PEAK_G == pytest.approx(256 * 4 * 16 * 2.4 / 60)


def test_roofline_picks_the_dominant_kernel(bench):
    ks = [
        {"name": "ic_sample_block", "launches": 4, "total_ms": 2.0, "alg_bytes": 8e6, "alg_ops": 4e8},
        {"name": "argmax", "launches": 100, "total_ms": 1.0, "alg_bytes": 4e8, "alg_ops": 0.0},
    ]
    r = bench.roofline(ks, "IC", "WC", "no-such-workload")
    # 1e8 Philox calls per 0.5 ms launch
    assert r["kernel"] == "ic_sample_block" and r["bound"] == "alu"
    assert r["achieved"] == pytest.approx(1e8 / 0.5e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.PHILOX_PEAK_G)
    assert r["traffic"] is None  # counters are tied to a workload and a source digest
    r = bench.roofline(ks[1:], "LT", "EDGE", "no-such-workload")
    # 4e6 bytes per 10 us launch
    assert r["bound"] == "hbm" and r["achieved"] == pytest.approx(4e6 / 10e-6 / 1e9)


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_traffic_calibrated_by_the_copy(bench, tmp_path, capsys):
    gib_kib = (1 << 30) / 1024.0
    # the counters read half of the copy's fetched bytes and all of its written bytes; a larger
    # copy-named kernel earlier in the run (the graph's generation) must not calibrate them
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [
        ("void at::native::copy_kernel_impl(...)", 4 * gib_kib), (copy, 1.0),
        ("void hbm::k_big_lds<1024, 2048, 13>(hbm::T2LArgs)", 100.0),
        ("void hbm::k_big_lds<1024, 2048, 13>(hbm::T2LArgs)", 300.0),
        ("void hbm::k_big_lds<1024, 8192, 14>(hbm::T2LArgs)", 7.0),
        ("void hbm::k_big_lds_g<256, 1024, 12>(hbm::GroupArgs<hbm::T2LArgs>)", 5.0),
        ("void hbm::k_argmax(hbm::SelArgs, int)", 10.0),
        (copy, gib_kib / 2 + 3), (copy, gib_kib / 2), (copy, gib_kib / 2 - 3)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [
        ("void at::native::copy_kernel_impl(...)", 4 * gib_kib),
        ("void hbm::k_big_lds<1024, 2048, 13>(hbm::T2LArgs)", 4.0),
        (copy, gib_kib), (copy, gib_kib), (copy, gib_kib)])
    _counter_csv(tmp_path / "l2.csv", "TCC_HIT_sum", [("void hbm::k_argmax(hbm::SelArgs, int)", 30.0),
                                                      ("void hbm::k_argmax(hbm::SelArgs, int)", 50.0)])
    with open(tmp_path / "l2.csv", "a", newline="") as f:
        csv.writer(f).writerow([3, "void hbm::k_argmax(hbm::SelArgs, int)", "TCC_MISS_sum", 20.0])
    out = tmp_path / "counters.json"
    bench.counters_summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "l2.csv"), "c2",
                             str(out))
    capsys.readouterr()
    t = json.load(open(out))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    k = t["traffic"]
    # mean of the two regular LDS-tier dispatches, fetched x2, plus written; the extra-large
    # pass and the 1024-member tier are told apart by their template arguments
    assert k["ic_sample_block"] == pytest.approx(200.0 * 1024 * 2 + 4.0 * 1024)
    assert k["ic_sample_block_xl"] == pytest.approx(7.0 * 1024 * 2)
    assert k["ic_sample_block_s"] == pytest.approx(5.0 * 1024 * 2)  # the 1024-member tier, grouped form
    assert k["argmax"] == pytest.approx(10.0 * 1024 * 2)
    assert t["l2_hit"] == {"argmax": pytest.approx(80.0 / 100.0)}
    assert t["workload_key"] == "c2" and t["csrc_digest"] == bench.csrc_digest()


def test_roofline_reports_hbm_fraction_beside_alu(bench):
    ks = [{"name": "ic_sample_block", "launches": 2, "total_ms": 1.0, "alg_bytes": 8e6, "alg_ops": 4e8}]
    r = bench.roofline(ks, "IC", "WC", "no-such-workload")
    # 4e6 bytes per 0.5 ms launch = 8 GB/s = 0.001 of 8 TB/s
    assert r["hbm_achieved_gbs"] == pytest.approx(8.0) and r["hbm_frac"] == pytest.approx(0.001)
    rates = bench.kernel_rates(ks)
    assert rates[0]["hbm_frac"] == pytest.approx(0.001) and rates[0]["gphilox_s"] == pytest.approx(400.0)


def test_host_info_caps_threads(bench):
    h = bench.host_info()
    assert 1 <= h["threads"] <= bench.HOST_THREADS_CAP and h["nproc"] >= 1
