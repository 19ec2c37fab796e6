"""Host-side logic of the benchmark (no GPU): the one-GPU guard, the
algorithmic byte model, and the counter summary behind roofline.traffic."""
import csv
import json

import bench


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_algorithmic_bytes_model():
    # per particle 7 reals read and 6 written; per cell E, B read and J read + written
    assert bench.algorithmic_bytes_per_push(1000, 10, 1) == 1000 * 52 + 10 * 48
    assert bench.algorithmic_bytes_per_push(1000, 10, 2, es=8) == 1000 * 104 + 10 * 96
    n, cells = 128**3 * 16, 128**3
    assert bench.algorithmic_bytes_per_push(n, cells, 1) == 1_845_493_760


def _write_csv(path, rows):
    path.mkdir(parents=True)
    with open(path / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counter_summary_and_traffic(tmp_path, monkeypatch):
    push = "void pic::k_push<1, false, false, 256, float>(pic::GridViewT<float>, ...)"
    other = "void pic::k_yee_b<float>(...)"
    copy = "__amd_rocclr_copyBuffer"
    _write_csv(tmp_path / "F", [dict(Kernel_Name=push, Counter_Name="FETCH_SIZE", Counter_Value=v) for v in (100, 300)]
               + [dict(Kernel_Name=other, Counter_Name="FETCH_SIZE", Counter_Value=9e9)])
    _write_csv(tmp_path / "W", [dict(Kernel_Name=push, Counter_Name="WRITE_SIZE", Counter_Value=v) for v in (50, 70)])
    _write_csv(tmp_path / "CF", [dict(Kernel_Name=copy, Counter_Name="FETCH_SIZE", Counter_Value=v)
                                 for v in (1000, 524288)])
    _write_csv(tmp_path / "CW", [dict(Kernel_Name=copy, Counter_Name="WRITE_SIZE", Counter_Value=1048576)])
    out = tmp_path / "summary.json"
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", str(out))
    assert bench.counter_summary(*(str(tmp_path / d) for d in ("F", "W", "CF", "CW"))) == 0
    d = json.loads(out.read_text())
    assert d["fetch_kib_per_dispatch"] == 200.0 and d["write_kib_per_dispatch"] == 60.0 and d["dispatches"] == 2
    assert d["fetch_scale"] == 0.5 and d["write_scale"] == 1.0
    assert d["k_push_sha256_16"] == bench.source_hash(bench.PUSH_SOURCES)
    # HBM bytes per launch: FETCH / 0.5 + WRITE / 1.0, in KiB
    assert bench.traffic_from_profile(d["particles"]) == (200.0 / 0.5 + 60.0) * 1024
    assert bench.traffic_from_profile(d["particles"] + 1) is None     # another workload
    d["k_push_sha256_16"] = "0" * 16                                   # the kernel changed since
    out.write_text(json.dumps(d))
    assert bench.traffic_from_profile(d["particles"]) is None


def test_cpu_baseline_legs(monkeypatch):
    # one thread on a sub-box, then the threaded oracle cycle on the full
    # (here: the small 16^3) workload, with the host described
    monkeypatch.setenv("OMP_NUM_THREADS", "2")
    out = bench.cpu_baseline(0, 8, 2, full=True, full_steps=1)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["value"] > 0
    assert out["host"]["nproc"] >= 1 and "CPU(s)" in out["host"]["lscpu"]
    a = out["all_cores"]
    assert a["cores"] == 2 and a["value"] > 0 and "16x16x16" in a["sample"]


def test_lds_byte_model():
    # gather reads (4 B) and in-line deposit atomics (8 B) per particle
    assert bench.lds_bytes_per_particle(1) == (48 * 4, 12 * 8)      # CIC: 6 x 8 reads, 12 atomics
    assert bench.lds_bytes_per_particle(2) == (162 * 4, 54 * 8)     # TSC: 6 x 27 reads, 54 atomics
    assert bench.lds_bytes_per_particle(3) == (384 * 4, 144 * 8)    # PCS: 6 x 64 reads, 3 x 16 x 3 atomics
    # Galerkin CIC: E_d reads 1 x 2 x 2 nodes, B_d 2 x 1 x 1
    assert bench.lds_bytes_per_particle(1, galerkin=True)[0] == (3 * 4 + 3 * 2) * 4
