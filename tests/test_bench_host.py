"""Host logic of bench.py (no GPU): the copy-calibrated HBM traffic record,
its staleness check against the kernel source, the roofline arithmetic and
the one-GPU guard."""
import csv
import json
import os
import shutil
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    """A scratch tree with a copy of the kernel source and an empty profiles/,
    so the committed traffic record is never touched."""
    src = os.path.join(HERE, "paper_1708_06127_amd", "csrc", "vc_kernels.hip")
    dst = tmp_path / "paper_1708_06127_amd" / "csrc"
    dst.mkdir(parents=True)
    shutil.copy(src, dst / "vc_kernels.hip")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def write_pmc(path, counter, rows):
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for i, (name, kib) in enumerate(rows):
            wr.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_record_traffic_scales_by_the_copy_probe(fake_root):
    copy_kib = bench.COPY_PROBE_BYTES / 1024
    small = "void vc::(anonymous namespace)::k_lp_tile<false>(int const*)"
    big = "void vc::(anonymous namespace)::k_lp_tile_big<false>(int const*)"
    other = "void vc::(anonymous namespace)::k_emit_tile(int const*)"
    # FETCH_SIZE reads half of the copy's bytes (scale 2), WRITE_SIZE all (scale 1)
    write_pmc(fake_root / "f.csv", "FETCH_SIZE",
              [("__amd_rocclr_copyBuffer", copy_kib / 2), (small, 100.0), (small, 300.0), (big, 50.0),
               (other, 9999.0)])
    write_pmc(fake_root / "w.csv", "WRITE_SIZE",
              [("__amd_rocclr_copyBuffer", copy_kib), (small, 10.0), (big, 4.0), (big, 6.0)])
    bench.record_traffic(str(fake_root / "f.csv"), str(fake_root / "w.csv"), "k_lp_tile", "wl", "cmd")
    rec = json.load(open(fake_root / "profiles" / "traffic_k_lp_tile_wl.json"))
    # per unit: the mean per dispatch of each kernel of the unit, summed
    fetch = (200.0 + 50.0) * 1024 * 2.0
    write = (10.0 + 5.0) * 1024 * 1.0
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == round(fetch)
    assert rec["write_bytes_per_launch"] == round(write)
    assert rec["bytes_per_launch"] == round(fetch + write)
    assert rec["dispatches"] == [[2, 1], [1, 2]]
    assert rec["source_sha"] == bench.kernel_source_hash()
    assert bench.traffic_for("k_lp_tile", "wl") == rec["bytes_per_launch"]


def test_traffic_goes_null_when_the_kernel_source_changes(fake_root):
    rec = {"source_sha": bench.kernel_source_hash(), "bytes_per_launch": 1234}
    with open(fake_root / "profiles" / "traffic_k_lp_tile_wl.json", "w") as f:
        json.dump(rec, f)
    assert bench.traffic_for("k_lp_tile", "wl") == 1234
    with open(fake_root / "paper_1708_06127_amd" / "csrc" / "vc_kernels.hip", "a") as f:
        f.write("\n// edited\n")
    assert bench.traffic_for("k_lp_tile", "wl") is None
    assert bench.traffic_for("k_lp_tile", "other_workload") is None


def test_record_traffic_needs_the_copy_probe(fake_root):
    small = "void vc::(anonymous namespace)::k_lp_tile<false>(int const*)"
    big = "void vc::(anonymous namespace)::k_lp_tile_big<false>(int const*)"
    write_pmc(fake_root / "f.csv", "FETCH_SIZE", [(small, 1.0), (big, 1.0)])
    write_pmc(fake_root / "w.csv", "WRITE_SIZE", [(small, 1.0), (big, 1.0)])
    with pytest.raises(SystemExit):
        bench.record_traffic(str(fake_root / "f.csv"), str(fake_root / "w.csv"), "k_lp_tile", "wl", "cmd")


def test_roofline_picks_the_dominant_unit(fake_root):
    prof = {"k_lp_tile": {"launches": 4, "total_ms": 0.8, "bytes": 4 * 400e6},
            "k_first_tile": {"launches": 2, "total_ms": 0.3, "bytes": 2 * 300e6},
            "k_first_tile_level0": {"launches": 0, "total_ms": 0.0, "bytes": 0}}
    r = bench.roofline(prof, "wl")
    assert r["kernel"] == "k_lp_tile"
    assert r["avg_us"] == pytest.approx(200.0)
    assert r["achieved"] == pytest.approx(2000.0)  # 400 MB in 200 us
    assert r["frac"] == pytest.approx(2000.0 / bench.HBM_PEAK_GBS)
    assert r["traffic"] is None  # no record in the scratch tree
    assert bench.roofline({"k_lp_tile": {"launches": 0, "total_ms": 0.0, "bytes": 0}}, "wl") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_roofline_ignores_the_sweep_span(fake_root):
    prof = {"k_lp_tile": {"launches": 4, "total_ms": 0.8, "bytes": 4 * 400e6},
            "lp_contract_sweep": {"launches": 4, "total_ms": 2.4, "bytes": 4 * 1.0e9}}
    assert bench.roofline(prof, "wl")["kernel"] == "k_lp_tile"
    s = bench.sweep_roofline(prof)
    assert s["avg_us"] == pytest.approx(600.0)
    assert s["achieved"] == pytest.approx(1.0e9 / 600e-6 / 1e9, abs=0.1)
    assert s["frac"] == pytest.approx(s["achieved"] / bench.HBM_PEAK_GBS, abs=1e-4)
    assert s["algorithmic_bytes"] == 1_000_000_000
    assert bench.sweep_roofline({"k_lp_tile": prof["k_lp_tile"]}) is None


def test_median():
    assert bench.median([3.0, 1.0, 2.0]) == 2.0
    assert bench.median([4.0, 1.0, 2.0, 3.0]) == 2.5
    assert bench.median([5.0]) == 5.0


def test_cpu_child_times_the_oracle_on_the_planted_graph():
    env = dict(os.environ, OMP_NUM_THREADS="2")
    p = subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), "--cpu-child", "c1", "--cpu-budget", "1",
                        "--cpu-runs", "2"], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr
    rec = json.loads(p.stdout.strip().splitlines()[-1])
    assert rec["threads"] == 2 and 1 <= rec["runs"] <= 2 and rec["value"] > 0
