#!/usr/bin/env python3
"""Particle-in-cell throughput on one MI355X.

One "step" is one full PIC cycle of the library (pic_step): zero J; per
supercell gather + relativistic Boris + move + Esirkepov deposit (fused
kernel); supercell migration; Yee B/2, E, B/2.  The default workload is the
128^3 CIC electron shear layer (16 particles per cell, 33.6M electrons,
+-0.2c counter-streaming along x, u_th = 0.01c, immobile ions, dt = 0.5,
particles re-sorted into supercell frames every step).  Inputs are synthetic
and seeded, generated on the GPU by pic_init, and resident in HBM before the
timed region starts.

Prints one JSON line: particle updates/s (value), ms per step, the roofline
of the dominant kernel (the fused particle kernel, HIP-event timed on the
handle's stream) and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
RATE_COUNTERS = os.path.join(ROOT, "profiles", "rate_exact_fp64_counters.json")
RATE_SOURCES = [os.path.join(ROOT, "paper_1606_02862_amd", "csrc", f)
                for f in ("k_ionize.hip", "ionize_internal.hpp", "pic_device.hpp", "pic_internal.hpp")]
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "push_shear128_counters.json")
PUSH_SOURCES = [os.path.join(ROOT, "paper_1606_02862_amd", "csrc", f)
                for f in ("k_push.hip", "pic_deposit.hpp", "pic_migrate.hpp", "pic_device.hpp", "pic_internal.hpp")]


def algorithmic_bytes_per_push(n_particles: int, n_cells: int, order: int, es: int = 4) -> int:
    """Bytes one particle-kernel launch must move (es = bytes per real): per
    particle 7 reals read (x, y, z, ux, uy, uz, w) and 6 written (x, y, z,
    ux, uy, uz); per cell E and B read once (6 reals) and J
    read-modify-written once (6 reals).  FP32: 52 B per particle, 48 B per cell."""
    return n_particles * 13 * es + n_cells * 12 * es


def algorithmic_bytes_per_step(n_particles: int, n_cells: int, es: int = 4) -> int:
    """Whole cycle: the particle kernel's bytes, J zeroed (3 reals per cell),
    and the three Yee passes (each reads 6 and writes 3 components, plus J
    read in the E pass: 30 reals per cell)."""
    return algorithmic_bytes_per_push(n_particles, n_cells, 1, es) + n_cells * (3 + 9 * 3 + 3) * es


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_particles: int):
    """HBM bytes per push launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs, scaled by the copy-kernel calibration; None if absent
    or if the particle kernel's source changed since they were taken."""
    try:
        with open(PROFILE_COUNTERS) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("k_push_sha256_16") != source_hash(PUSH_SOURCES) or d.get("particles") != n_particles:
        return None
    fetch = d["fetch_kib_per_dispatch"] * 1024 / d["fetch_scale"]
    write = d["write_kib_per_dispatch"] * 1024 / d["write_scale"]
    return fetch + write


def host_description():
    cpu = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                cpu = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return cpu, os.cpu_count()


def host_threads() -> int:
    """Threads for the all-cores leg: OMP_NUM_THREADS when set (the GPU host
    sets it to the CPU share of one GPU), else the CPUs this process may use."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def lscpu_summary() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
    except OSError:
        return ""
    keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz")
    return "; ".join(l.split(":", 1)[0].strip() + ": " + l.split(":", 1)[1].strip()
                     for l in out.splitlines() if l.split(":", 1)[0].strip() in keep)


def cpu_baseline(cfg_idx: int, box: int, steps: int, full: bool = True, full_steps: int = 3, **grid) -> dict:
    """The FP64 oracle on the host: one thread on a sub-box of the same
    workload (grid: the same shape / gather overrides as the GPU run), and,
    with full, the oracle's cycle with its particle loop split over all host
    threads (private current arrays) on the full-size workload, one warm-up
    cycle and full_steps timed ones."""
    import oracle
    cfg = workloads.config(cfg_idx, nx=box, ny=box, nz=box, **grid)
    st = oracle.init_state(cfg)
    n = sum(s.n for s in st.species if s.mobile)
    t0 = time.perf_counter()
    oracle.step(st, steps)
    dt = time.perf_counter() - t0
    del st
    cpu, ncpu = host_description()
    out = {"value": n * steps / dt, "unit": "particle updates/s", "cores": 1, "kind": "oracle",
           "sample": f"{box}^3 periodic sub-box of the same workload ({n} particles), {steps} PIC cycles, "
                     f"FP64 C oracle, single thread; host {cpu}, {ncpu} logical CPUs",
           "seconds": dt, "host": {"cpu": cpu, "nproc": ncpu, "lscpu": lscpu_summary()}}
    if full:
        cfg = workloads.config(cfg_idx, **grid)
        gc = cfg["grid"]
        st = oracle.init_state(cfg)
        n = sum(s.n for s in st.species if s.mobile)
        nt = host_threads()
        oracle.step_threads(st, 1, nt)
        t0 = time.perf_counter()
        used = oracle.step_threads(st, full_steps, nt)
        dt = time.perf_counter() - t0
        out["all_cores"] = {
            "value": n * full_steps / dt, "unit": "particle updates/s", "cores": used,
            "kind": "oracle cycle, particle loop split over threads (private current arrays)",
            "sample": f"the full {gc['nx']}x{gc['ny']}x{gc['nz']} workload ({n} particles), 1 warm-up and "
                      f"{full_steps} timed PIC cycles, FP64 C oracle on {used} threads",
            "seconds": dt}
    return out


def copy_calibration() -> int:
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters divided
    by 1 GiB give the scale that turns the counters into HBM bytes."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 4 * n, "repeats": 3}), flush=True)
    return 0


def dword_calibration() -> int:
    """A dword-per-lane copy of 1 GiB (the particle streams' access width,
    from the probe library), three times: its FETCH_SIZE / WRITE_SIZE per GiB
    give the counter scale for such streams."""
    import ctypes
    import torch
    from paper_1606_02862_amd import build as B
    lib = ctypes.CDLL(B.PROBE_LIB)
    lib.probe_copy_dword.restype = ctypes.c_int
    lib.probe_copy_dword.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    if lib.probe_copy_dword(src.data_ptr(), dst.data_ptr(), n, 3) != 0:
        raise SystemExit("dword copy failed")
    assert bool((dst == 1).all())
    print(json.dumps({"dword_copy_bytes_each_way": 4 * n, "repeats": 3}), flush=True)
    return 0


def _counter_rows(run_dir: str):
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    return rows


def counter_summary(fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str) -> int:
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of the default
    benchmark, then of --copy-calibration) into the counter summary that
    roofline.traffic is computed from, stamped with the particle kernel's
    source hash."""
    push = "k_push<1, false, false, 256, float>"

    def push_avg(run_dir, counter):
        v = [float(r["Counter_Value"]) for r in _counter_rows(run_dir)
             if push in r["Kernel_Name"] and r["Counter_Name"] == counter]
        if not v:
            raise SystemExit(f"no {counter} rows for {push} under {run_dir}")
        return sum(v) / len(v), len(v)

    def copy_max(run_dir, counter):
        v = [float(r["Counter_Value"]) for r in _counter_rows(run_dir)
             if "copy" in r["Kernel_Name"].lower() and r["Counter_Name"] == counter]
        if not v:
            raise SystemExit(f"no {counter} rows for a copy kernel under {run_dir}")
        return max(v)

    fetch, nd = push_avg(fetch_dir, "FETCH_SIZE")
    write, _ = push_avg(write_dir, "WRITE_SIZE")
    cf, cw = copy_max(copy_fetch_dir, "FETCH_SIZE"), copy_max(copy_write_dir, "WRITE_SIZE")
    cfg = workloads.config(1)
    gc = cfg["grid"]
    d = {"k_push_sha256_16": source_hash(PUSH_SOURCES),
         "particles": gc["nx"] * gc["ny"] * gc["nz"] * cfg["species"][0]["ppc"],
         "workload": cfg["workload"],
         "fetch_kib_per_dispatch": round(fetch, 1), "write_kib_per_dispatch": round(write, 1), "dispatches": nd,
         "fetch_scale": round(cf / 1048576.0, 4), "write_scale": round(cw / 1048576.0, 4),
         "copy_fetch_kib_per_gib": round(cf, 1), "copy_write_kib_per_gib": round(cw, 1)}
    with open(PROFILE_COUNTERS, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d), flush=True)
    return 0


def exact_rate_profile() -> int:
    """One exact-quadrature ionisation step on the 128^3 electron-carbon
    workload (2 PIC cycles first), for an FP64 counter pass over k_rate_exact."""
    import torch  # noqa: F401
    import paper_1606_02862_amd as P
    P.load()
    cfg = workloads.config(3)
    gc = cfg["grid"]
    with P.Pic(cfg) as pic:
        pic.step(2)
        r = pic.ionize("exact", staged=True)
    print(json.dumps({"ions_active": r["ions_active"], "rate_ms": r["rate_ms"],
                      "ions": gc["nx"] * gc["ny"] * gc["nz"] * cfg["species"][1]["ppc"]}), flush=True)
    return 0


def exact_rate_fp64(rate_ms: float, ions: int):
    """FP64 FLOP rate of k_rate_exact from the committed counter summary (FP64
    FLOPs per dispatch over the same ion population), or None if it is absent
    or the rate kernel's sources changed since."""
    try:
        with open(RATE_COUNTERS) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("sources_sha256_16") != source_hash(RATE_SOURCES) or d.get("ions") != ions:
        return None
    tflops = d["fp64_flops_per_dispatch"] / (rate_ms * 1e-3) / 1e12
    return {"fp64_flops_per_ion": d["fp64_flops_per_dispatch"] / ions, "achieved_tflops": tflops,
            "peak_tflops": FP64_PEAK_TFLOPS, "frac": tflops / FP64_PEAK_TFLOPS}


def rate_counter_summary(run_dir: str, ions: int) -> int:
    """Turn one rocprofv3 --pmc run of --exact-rate-profile (FP64 instruction
    counters of k_rate_exact) into the summary behind ionize.exact_rate_fp64:
    FP64 FLOPs per dispatch = 64 lanes x (ADD + MUL + TRANS + 2 FMA) wave
    instructions, stamped with the rate kernel's source hash."""
    rows = [r for r in _counter_rows(run_dir) if "k_rate_exact" in r["Kernel_Name"]]
    if not rows:
        raise SystemExit(f"no k_rate_exact rows under {run_dir}")
    c = {}
    for r in rows:
        c.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    avg = {k: sum(v) / len(v) for k, v in c.items()}
    inst = {k: avg.get(f"SQ_INSTS_VALU_{k}_F64", 0.0) for k in ("ADD", "MUL", "FMA", "TRANS")}
    flops = 64.0 * (inst["ADD"] + inst["MUL"] + inst["TRANS"] + 2.0 * inst["FMA"])
    d = {"sources_sha256_16": source_hash(RATE_SOURCES), "ions": ions, "kernel": "k_rate_exact",
         "fp64_wave_instructions": inst, "fp64_flops_per_dispatch": flops,
         "counter_FLOPS_FP64": avg.get("SQ_INSTS_VALU_FLOPS_FP64"),
         "counter_FLOPS_FP64_TRANS": avg.get("SQ_INSTS_VALU_FLOPS_FP64_TRANS"), "dispatches": len(c.get("SQ_INSTS_VALU_FMA_F64", []))}
    with open(RATE_COUNTERS, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d), flush=True)
    return 0


def ionize_leg(P, torch, repeats: int = 3, cpu: bool = True) -> dict:
    """Monte Carlo ionisation on the 128^3 electron-carbon workload: GPU time
    of the rate stage and of the whole step with the exact FP64 GL-64
    quadrature, with the BF16-MFMA surrogate (trained first on the GPU; SiLU
    as configured, and the same network with ReLU as a second line) and with
    the tabulated rate, and their rate errors against the exact quadrature."""
    import numpy as np
    cfg = workloads.config(3)
    gc = cfg["grid"]
    ncell = gc["nx"] * gc["ny"] * gc["nz"]
    pic = P.Pic(cfg)
    rep = pic.mlp_train(1, seed=workloads.MLP_TRAIN_SEED, **workloads.MLP_TRAIN)
    trained = pic.mlp_get_params(1)
    # the same network and recipe with ReLU hidden activations, on a second handle
    pic_relu = P.Pic(cfg)
    rep_relu = pic_relu.mlp_train(1, seed=workloads.MLP_TRAIN_SEED, **dict(workloads.MLP_TRAIN, activation="relu"))
    trained_relu = pic_relu.mlp_get_params(1)
    pic.step(2)
    out = {"workload": workloads.config(4)["workload"], "ions": ncell * cfg["species"][1]["ppc"],
           "electrons_initial": ncell * cfg["species"][0]["ppc"], "train": rep, "train_relu": rep_relu}

    def one_call(mode, staged):
        # a fresh handle per call: every mode and repeat ionises the same state
        # (same cells, charge states and Philox draws)
        h = P.Pic(cfg)
        if mode == "mlp":
            h.mlp_set_params(1, *trained)
        if mode == "mlp_relu":
            h.mlp_set_params(1, *trained_relu)
        if mode == "table":
            h.rate_eval("table", 1, [100.0], [1e21], [2])   # builds the table (once per handle)
        h.step(2)
        r = h.ionize("mlp" if mode == "mlp_relu" else mode, staged=staged)
        h.close()
        return r

    for mode in ("exact", "mlp", "table", "mlp_relu"):
        # staged: the rate stage timed on its own; fused (pic_ionize): the
        # whole step as one launch per supercell (the table runs staged)
        runs = [one_call(mode, True) for _ in range(repeats)]
        fused = [one_call(mode, False) for _ in range(repeats)]
        out[mode] = {"rate_ms": min(r["rate_ms"] for r in runs), "total_staged_ms": min(r["total_ms"] for r in runs),
                     "total_ms": min(r["total_ms"] for r in fused),
                     "ionized_per_call": [r["ionized"] for r in runs + fused], "fallback": fused[-1]["fallback"],
                     "ions_active": fused[-1]["ions_active"]}
    out["rate_stage_speedup"] = out["exact"]["rate_ms"] / out["mlp"]["rate_ms"]
    # the whole pic_ionize (cell moments + rate + draw/append), each mode fused
    out["whole_step_speedup"] = out["exact"]["total_ms"] / out["mlp"]["total_ms"]
    # the same with the three stages as separate launches
    out["whole_step_speedup_staged"] = out["exact"]["total_staged_ms"] / out["mlp"]["total_staged_ms"]
    # how efficient the exact baseline is: its FP64 rate against the FP64 peak
    out["exact_rate_fp64"] = exact_rate_fp64(out["exact"]["rate_ms"], out["ions"])
    out["rate_stage_ions_per_s"] = {m: out[m]["ions_active"] / (out[m]["rate_ms"] * 1e-3)
                                    for m in ("exact", "mlp", "table", "mlp_relu")}
    out["table_rate_stage_speedup"] = out["exact"]["rate_ms"] / out["table"]["rate_ms"]
    out["table_whole_step_speedup"] = out["exact"]["total_ms"] / out["table"]["total_ms"]
    out["mlp_relu_rate_stage_speedup"] = out["exact"]["rate_ms"] / out["mlp_relu"]["rate_ms"]
    out["mlp_relu_whole_step_speedup"] = out["exact"]["total_ms"] / out["mlp_relu"]["total_ms"]
    # error of the surrogate against the exact quadrature (its reference)
    T, ne, Z = workloads.loguniform_rate_inputs(workloads.MLP_HELDOUT_SEED, 1_000_000)
    ex = pic.rate_eval("exact", 1, T, ne, Z)
    ml = pic.rate_eval("mlp", 1, T, ne, Z)
    rel = np.abs(np.expm1(ml - ex))
    pz = np.array(workloads.CARBON_IONIZATION_EV)[Z]
    qz = np.array(workloads.CARBON_LOTZ_Q)[Z]
    z = pz / T
    vbar = 2.99792458e10 * np.sqrt(8 * T / (np.pi * 510998.95))
    prior = np.log(ne * vbar * 4.5e-14 * qz / (pz * T)) - z + np.log(np.log1p(1 / z))
    relp = np.abs(np.expm1(prior - ex))

    def stats(r):
        return {"median": float(np.median(r)), "p99": float(np.quantile(r, 0.99)), "max": float(r.max())}
    out["mlp_error_heldout"] = stats(rel)
    out["table_error_heldout"] = stats(np.abs(np.expm1(pic.rate_eval("table", 1, T, ne, Z) - ex)))
    out["prior_only_error_heldout"] = stats(relp)
    out["mlp_relu_error_heldout"] = stats(np.abs(np.expm1(pic_relu.rate_eval("mlp", 1, T, ne, Z) - ex)))
    # live population: every cell's (n_e, kT_e) with the charge states present
    ne_c, kT_c = pic.cell_moments(1)
    ok = (ne_c > 0) & (kT_c > 0)
    lt, ln = kT_c[ok], ne_c[ok]
    zz = np.full(lt.size, 2, dtype=np.int32)
    rl = np.abs(np.expm1(pic.rate_eval("mlp", 1, lt, ln, zz) - pic.rate_eval("exact", 1, lt, ln, zz)))
    out["mlp_error_live_cells_Z2"] = stats(rl)
    rr = np.abs(np.expm1(pic_relu.rate_eval("mlp", 1, lt, ln, zz) - pic.rate_eval("exact", 1, lt, ln, zz)))
    out["mlp_relu_error_live_cells_Z2"] = stats(rr)
    pic.close()
    pic_relu.close()
    if cpu:
        import oracle.ionize as oi
        Ts, ns, Zs = T[:200_000], ne[:200_000], Z[:200_000]
        t0 = time.perf_counter()
        oi.ln_rate_exact(Ts, ns, pz[:200_000], qz[:200_000])
        dt = time.perf_counter() - t0
        out["cpu_oracle_exact_rates_per_s"] = Ts.size / dt
    return out


def lds_bytes_per_particle(order: int, galerkin: bool = False) -> tuple[int, int]:
    """LDS bytes one particle moves in the particle kernel's in-line path:
    the field gather reads (6 components, (order+1) nodes per axis, one order
    lower along staggered axes with the Galerkin gather; 4 B each) and the
    Esirkepov deposit of a particle that keeps its first shape node (per
    current component (order+1)^2 lines of `order` nodes; 8-byte atomics)."""
    p = order + 1
    if galerkin:  # each component is staggered along one (E) or two (B) axes
        reads = 3 * (order * p * p) + 3 * (order * order * p)
    else:
        reads = 6 * p ** 3
    atomics = 3 * p * p * order
    return 4 * reads, 8 * atomics


def lds_peaks() -> dict:
    """Measured LDS bandwidth of the device (bytes/s): conflict-free
    ds_read_b64 and ds_add_u64 streams of the probe library."""
    import ctypes
    from paper_1606_02862_amd import build as B
    lib = ctypes.CDLL(B.PROBE_LIB)
    lib.probe_lds_bandwidth.restype = ctypes.c_double
    lib.probe_lds_bandwidth.argtypes = [ctypes.c_int, ctypes.c_int]
    return {"read": lib.probe_lds_bandwidth(0, 4000), "atomic": lib.probe_lds_bandwidth(1, 2000)}


def timed_kernels(P, torch, cfg: dict, warmup: int, steps: int) -> dict:
    """Per-kernel GPU times (pic_timing: HIP events around every launch on the
    handle's stream) over cycles warmup .. warmup + steps of a fresh handle of
    the workload, i.e. over the same cycles as the timed region."""
    pic = P.Pic(cfg)
    pic.step(warmup)
    torch.cuda.synchronize()
    pic.timing(1)
    pic.step(steps)
    tm = pic.timing(0)
    torch.cuda.synchronize()
    pic.close()
    return tm


def shape_leg(P, torch, cfg_idx: int, steps: int, warmup: int, peaks: dict) -> dict:
    """One workload's PIC cycle (the TSC workloads: 256x256x128 electrons and
    protons, and the 128^3 Kelvin-Helmholtz shear flow): updates/s, the
    particle kernel's time per launch, and its HBM and LDS rooflines."""
    cfg = workloads.config(cfg_idx)
    gc = cfg["grid"]
    ncell = gc["nx"] * gc["ny"] * gc["nz"]
    order = {"cic": 1, "tsc": 2, "pcs": 3}[gc["shape"]]
    mobile = [s for s in cfg["species"] if s["mobile"]]
    n = sum(ncell * s["ppc"] for s in mobile)
    pic = P.Pic(cfg)
    pic.step(warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(pic.stream)
    pic.step(steps)
    t1.record(pic.stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    pic.close()
    tm = timed_kernels(P, torch, cfg, warmup, steps)
    push_s = tm["push_ms"] / steps * 1e-3            # all species' particle kernels of one cycle
    hbm = sum(algorithmic_bytes_per_push(ncell * s["ppc"], ncell, order) for s in mobile)
    rd, at = lds_bytes_per_particle(order, gc.get("gather", "standard") == "galerkin")
    t_lds = n * rd / peaks["read"] + n * at / peaks["atomic"]
    return {"workload": cfg["workload"], "particles": n, "steps": steps, "ms_per_step": ms,
            "value": n / (ms * 1e-3), "unit": "particle updates/s",
            "push_ms_per_step": push_s * 1e3, "push_launches_per_step": tm["push_launches"] / steps,
            "roofline_hbm": {"achieved": hbm / push_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": hbm / push_s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_step": hbm},
            "roofline_lds": {"bytes_read_per_particle": rd, "bytes_atomic_per_particle": at,
                             "peak_read": peaks["read"] / 1e9, "peak_atomic": peaks["atomic"] / 1e9, "unit": "GB/s",
                             "t_min_ms": t_lds * 1e3, "frac": t_lds / push_s}}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=1,
                    help="workload preset (1: 128^3 CIC shear, 2: 256x256x128 TSC e+p, 5: 128^3 TSC KHI e+p)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-box", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=32)
    ap.add_argument("--no-cpu-full", action="store_true",
                    help="skip the all-cores oracle leg on the full-size workload")
    ap.add_argument("--no-ionize", action="store_true", help="skip the ionisation leg")
    ap.add_argument("--no-tsc", action="store_true", help="skip the TSC workload lines (256x256x128 e+p, 128^3 KHI)")
    ap.add_argument("--tsc-steps", type=int, default=10)
    ap.add_argument("--shape", choices=("cic", "tsc", "pcs"), help="override the workload's particle shape")
    ap.add_argument("--gather", choices=("standard", "galerkin"), help="override the field gather")
    ap.add_argument("--fp64", action="store_true",
                    help="the FP64 variant of the PIC cycle (the ionisation leg, FP32 only, is skipped)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--exact-rate-profile", action="store_true",
                    help="only one exact-quadrature ionisation step on the 128^3 carbon workload (FP64 counters)")
    ap.add_argument("--dword-calibration", action="store_true",
                    help="only run a 1 GiB copy with one dword per lane per access (HBM counter calibration)")
    ap.add_argument("--rate-counter-summary", nargs=2, metavar=("RUN_DIR", "IONS"),
                    help="write the FP64 counter summary of k_rate_exact from one rocprofv3 --pmc run")
    ap.add_argument("--counter-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the counter summary behind roofline.traffic from four rocprofv3 --pmc runs")
    args = ap.parse_args(argv)
    if args.copy_calibration:
        return copy_calibration()
    if args.dword_calibration:
        return dword_calibration()
    if args.exact_rate_profile:
        return exact_rate_profile()
    if args.counter_summary:
        return counter_summary(*args.counter_summary)
    if args.rate_counter_summary:
        return rate_counter_summary(args.rate_counter_summary[0], int(args.rate_counter_summary[1]))

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU; sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        return 2

    import torch

    import paper_1606_02862_amd as P
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    P.load()
    cfg = workloads.config(args.config)
    if args.fp64:
        cfg["grid"]["precision"] = "fp64"
    overridden = False
    for key in ("shape", "gather"):
        if getattr(args, key) and getattr(args, key) != cfg["grid"].get(key, "standard"):
            cfg["grid"][key] = getattr(args, key)
            cfg["workload"] += f", {key} {getattr(args, key)}"
            overridden = True
    es = 8 if args.fp64 else 4
    gc = cfg["grid"]
    ncell = gc["nx"] * gc["ny"] * gc["nz"]
    order = {"cic": 1, "tsc": 2, "pcs": 3}[gc["shape"]]
    n_particles = sum(ncell * s["ppc"] for s in cfg["species"] if s["mobile"])

    pic = P.Pic(cfg)
    stream = pic.stream
    pic.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: exactly `steps` cycles, HIP events on the handle's stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    pic.step(args.steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    ms_per_step = ms / args.steps

    moments = pic.moments()
    pic.close()
    # the same region again on a fresh handle (same seed, same warm-up), with
    # per-kernel HIP events for the roofline; the events cost 2-6 % of a
    # cycle, so they stay out of the region `value` is timed on
    tm = timed_kernels(P, torch, cfg, args.warmup, args.steps)

    push_avg_ms = tm["push_ms"] / max(tm["push_launches"], 1)
    per_launch = algorithmic_bytes_per_push(n_particles // max(1, sum(1 for s in cfg["species"] if s["mobile"])),
                                            ncell, order, es)
    achieved = per_launch / (push_avg_ms * 1e-3) / 1e9
    # the counter summary covers the default FP32 workload only
    traffic = None if (args.fp64 or overridden or args.config != 1) else traffic_from_profile(n_particles)
    step_bytes = algorithmic_bytes_per_step(n_particles, ncell, es)
    value = n_particles * args.steps / (ms * 1e-3)
    line = {
        "metric": "particle updates/s (gather+push+deposit) & % HBM peak; ionize step exact vs MLP",
        "value": value,
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp64 else "f32",
        "data": "synthetic (seeded Philox initial state generated on the GPU)",
        "config": {"workload": cfg["workload"], "grid": [gc["nx"], gc["ny"], gc["nz"]], "shape": gc["shape"],
                   "gather": gc.get("gather", "standard"),
                   "species": [{"name": s["name"], "ppc": s["ppc"], "mass": s["mass"]} for s in cfg["species"]],
                   "particles": n_particles, "supercell": [8, 8, 4], "dt": gc["dt"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_push (gather+Boris+Esirkepov)", "avg_launch_ms": push_avg_ms,
                     "algorithmic_bytes_per_launch": per_launch},
        "step_breakdown_ms": {"push": tm["push_ms"] / args.steps, "migrate": tm["migrate_ms"] / args.steps,
                              "fields": tm["field_ms"] / args.steps},
        "hbm_frac_whole_step": step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "checks": {"gauss_max_over_rho_max": moments["gauss_max"] / max(moments["rho_max"], 1e-30),
                   "particles_after": sum(moments["count"])},
    }
    peaks = lds_peaks()
    rd, at = lds_bytes_per_particle(order, gc.get("gather", "standard") == "galerkin")
    t_lds = n_particles * rd / peaks["read"] + n_particles * at / peaks["atomic"]
    line["roofline"]["lds"] = {"bytes_read_per_particle": rd, "bytes_atomic_per_particle": at,
                               "peak_read": peaks["read"] / 1e9, "peak_atomic": peaks["atomic"] / 1e9,
                               "unit": "GB/s", "t_min_ms": t_lds * 1e3, "frac": t_lds / (push_avg_ms * 1e-3)}
    if not args.no_tsc and not args.fp64 and args.config == 1 and not overridden:
        line["tsc"] = {"ep256": shape_leg(P, torch, 2, args.tsc_steps, 3, peaks),
                       "khi128": shape_leg(P, torch, 5, args.tsc_steps, 3, peaks)}
    if not args.no_ionize and not args.fp64:
        line["ionize"] = ionize_leg(P, torch, cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        over = {k: getattr(args, k) for k in ("shape", "gather") if getattr(args, k)}
        line["cpu_baseline"] = cpu_baseline(args.config, args.cpu_box, args.cpu_steps,
                                            full=not args.no_cpu_full and not args.fp64, **over)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
