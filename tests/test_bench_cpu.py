"""CPU checks of bench.py's host logic: the single-GPU refusal, and the
parsing of rocprofv3 counter files into traffic records."""
import csv
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def _counter_dir(tmp_path, name, counter, rows):
    d = tmp_path / name / "host"
    d.mkdir(parents=True)
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kname, val in rows:
            w.writerow({"Kernel_Name": kname, "Counter_Name": counter, "Counter_Value": val})
    return str(tmp_path / name)


def test_traffic_records_separate_modes_and_widths(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    k = "void esmf::(anonymous namespace)::fock_mfma_kernel<{}>(esmf::UnitDesc const*, int, esmf::WorkItem const*, int)"
    fetch = _counter_dir(tmp_path, "f", "FETCH_SIZE", [
        (k.format("0, 1, 3, 4, 8"), 100.0), (k.format("0, 1, 3, 4, 8"), 300.0),
        (k.format("0, 1, 2, 4, 16"), 500.0), (k.format("2, 1, 4, 4, 8"), 50.0),
        ("some_other_kernel", 9e9)])
    write = _counter_dir(tmp_path, "w", "WRITE_SIZE", [
        (k.format("0, 1, 3, 4, 8"), 10.0), (k.format("0, 1, 3, 4, 8"), 30.0),
        (k.format("0, 1, 2, 4, 16"), 70.0), (k.format("2, 1, 4, 4, 8"), 5.0)])
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    bench.record_traffic(fetch, write, "wl")
    rec = json.load(open(prof / "traffic.json"))
    assert set(rec) == {"wl:fp64", "wl:fp64_wide", "wl:store32"}
    assert rec["wl:fp64"]["fetch_KiB_per_dispatch"] == 200.0 and rec["wl:fp64"]["dispatches"] == [2, 2]
    assert rec["wl:fp64_wide"]["write_KiB_per_dispatch"] == 70.0
    assert rec["wl:fp64"]["hbm_bytes_per_launch"] == 1024.0 * (bench.FETCH_SCALE * 200.0 + bench.WRITE_SCALE * 20.0)


def test_code_only_hash_ignores_comments():
    sys.path.insert(0, ROOT)
    import bench
    a = "int f(int x) {  // doubles x\n    return 2 * x; /* no\n overflow check */\n}\n"
    b = "int f(int x) {\n\n    return 2 * x;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(b.replace("2 *", "3 *"))


def test_cpu_baseline_is_one_full_oracle_build(oracle_mod):
    # the baseline times every unique screened quartet once (its chunks
    # partition the outer pairs), not a sample scaled up
    sys.path.insert(0, ROOT)
    import bench
    import workloads as wl
    c = wl.config2()
    _, nq = oracle_mod.count(c["centers"], c["alpha"], c["tau"])
    out = bench.cpu_baseline(c, nq)
    assert out["quartets_visited"] == nq
    assert out["sample"].startswith("full build")
    assert out["value"] == pytest.approx(1.0 / out["seconds_per_build"])
    assert out["cores"] >= 1 and out["cpu_model"]
    assert out["chain400_builds"] == 5 and out["chain400_median_s_per_build"] > 0
