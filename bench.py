#!/usr/bin/env python3
"""Throughput benchmark of the hybrid PIC/MCC hot path on one MI355X.

Workload (default): the single large discharge -- helium at 1 atm, 1 mm gap,
2,048 cells, 250 V at 13.56 MHz, 8,388,608 FP32 electron superparticles,
full-inertia ion fluid, re-sort every 16 steps -- with seeded synthetic
cross sections and initial load.  A step is one pass of the whole hot path
(field, ion fluid, push / MCC / deposit, emission, append, sort when due).

Before the timed region the autotuner takes --tune-steps real steps to pick
the launch shapes (they never change results), then the warmup runs at
least --warmup steps, up to a sort-interval boundary.  The timed region is
exactly --steps steps, whole intervals replayed from captured graphs and a
partial last interval launched kernel by kernel, with the particle state
resident in HBM, bracketed by device synchronisation.  value = particle-steps
(live electrons pushed, counted on the device) / seconds.

roofline: the fused electron kernel is timed with HIP events on the
library's stream over --profile-steps further real steps; its algorithmic
bytes are 36 B per FP32 particle-step (read cell, offset, three velocities
and id; write cell, offset, v_z) plus 8 B per collision (v_x, v_y).
traffic: HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
(profiles/), scaled by the same counters on a plain copy of known size;
null when the kernel source changed since they were taken.  copy_measured:
a 1 GiB device-to-device copy timed on the same GPU (read + write bytes per
second), the practical ceiling beside the published peak; frac_of_copy is
the kernel's rate against it.
cpu_baseline: the plain CPU oracle on this host for a bounded number of
steps of the same workload, on all usable cores and on one (host recorded).
fp32_vs_fp64: the error of FP32 particle arithmetic against FP64 per result,
by decision-locked replay on the CPU (the oracle's float run is the device's
bit for bit).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1508_02892_amd/csrc/k_electron.hip",
                  "paper_1508_02892_amd/csrc/hd_device.h",
                  "paper_1508_02892_amd/csrc/hd_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_electron_c1_traffic.md")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_copy_gbs(n_bytes=1 << 30, reps=5):
    """Device-to-device copy rate on this GPU (bytes read plus written per
    second, GB/s), the practical ceiling beside the published 8 TB/s."""
    import torch
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * n_bytes / (ms * 1e-3) / 1e9


def read_traffic():
    """HBM bytes per electron launch recorded from rocprofv3 counters, if the
    kernel is unchanged since they were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m_hash = re.search(r"source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


def workload(name: str):
    from paper_1508_02892_amd import workloads as W
    if name == "c1":
        return W.c1(), ("single large discharge: He 1 atm, 1 mm, 2048 cells, 250 V, "
                        "8,388,608 FP32 electrons, full ion fluid, sort every 16")
    if name == "c2":
        return W.c2(), ("complex chemistry: He + 0.5% O2-like, 1 mm, 1024 cells, 300 V, "
                        "4,194,304 FP32 electrons, 12 channels with attachment, 4 DD ion species")
    if name == "c0":
        return W.c0(), ("small plain discharge: He 1 atm, 0.5 mm, 256 cells, 150 V, "
                        "16,384 FP64 electrons, drift-diffusion ions")
    raise SystemExit("unknown workload " + name)


def host_info() -> dict:
    """The host's core count and CPU model (lscpu), for the CPU baseline."""
    info = {"nproc": os.cpu_count() or 0, "model": ""}
    try:
        sched = len(os.sched_getaffinity(0))
        info["usable_cores"] = sched
    except (AttributeError, OSError):
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return info


def cpu_baseline(p, steps: int, desc: str, threads: int = 0):
    """The plain oracle on this host: `steps` steps of the workload after its
    load, on all usable cores (the particle loop split over threads with
    per-thread integer grids, bitwise the single-thread run) and on one."""
    import oracle
    host = host_info()
    all_cores = threads or host.get("usable_cores") or host["nproc"] or 1
    rates = {}
    for t in sorted({1, all_cores}, reverse=True):
        oracle.set_threads(t)
        try:
            orc = oracle.Oracle(p)
            c0 = orc.counters()["pushed"]
            t0 = time.perf_counter()
            orc.step(steps)
            dt = time.perf_counter() - t0
            n = orc.counters()["pushed"] - c0
            rates[t] = (n / dt, n, dt)
        finally:
            oracle.set_threads(1)
        del orc
    v, n, dt = rates[all_cores]
    return {"value": v, "unit": "particle-steps/s", "cores": all_cores, "kind": "oracle",
            "sample": "%s; %d steps after the initial load (%d particle-steps, %.1f s), "
                      "%d threads" % (desc, steps, n, dt, all_cores),
            "single_thread_value": rates[1][0],
            "host": host}


def precision_leg() -> dict:
    """Error of the FP32 particle arithmetic against FP64, per result, by
    decision-locked replay on the CPU (the oracle's float run is bitwise the
    device's): the large discharge's geometry with 65,536 electrons, 64
    steps, each step from the float state and accumulated.  Normwise:
    max |x32 - x64| / max |x64|; element-wise with a floor of 1e-3 of the
    profile's largest value."""
    from oracle.replay_errors import replay_errors
    from paper_1508_02892_amd import workloads as W
    p = W.scaled(W.c1(), 1 << 16)
    th = os.cpu_count() or 1
    out = {"sample": "2,048 cells, full ion fluid, 65,536 electrons, 64 steps"}
    for name, per_step in (("per_step", True), ("accumulated", False)):
        r = replay_errors(p, 64, threads=min(th, 16), per_step=per_step)
        out[name] = {"normwise": r["normwise"], "elementwise": r["elementwise"],
                     "flips": r["flips"]}
    return out


C1_TABLE_STEPS = 200  # the first 200 steps of the single large discharge


def cpu_table(a):
    """The CPU oracle's rates on this host for the set of workloads the
    baseline plan names: the small plain discharge in full (FP64 particles,
    and in FP32), the single large discharge for a bounded number of steps,
    and one discharge of the batched sweep per size octave (100 steps each),
    each single-threaded and on all usable cores.  No GPU is used."""
    import oracle
    from paper_1508_02892_amd import workloads as W
    host = host_info()
    cores = host.get("usable_cores") or host["nproc"] or 1
    cases = [("small plain discharge, FP64, all 2,000 steps", W.c0(), W.C0_STEPS),
             ("small plain discharge, FP32 particles, all 2,000 steps", W.c0(precision=0),
              W.C0_STEPS),
             ("single large discharge, first %d steps" % C1_TABLE_STEPS, W.c1(), C1_TABLE_STEPS)]
    ps = W.c3()
    for lo in range(18, 23):
        pick = [p for p in ps if (1 << lo) <= p["n_macro"] < (1 << (lo + 1))]
        if pick:
            cases.append(("batched-sweep member with %d electrons (octave 2^%d), 100 steps"
                          % (pick[0]["n_macro"], lo), pick[0], 100))
    rows = []
    for name, p, steps in cases:
        row = {"workload": name, "electrons": int(p["n_macro"])}
        for t in (1, cores):
            oracle.set_threads(t)
            try:
                o = oracle.Oracle(p)
                c0 = o.counters()["pushed"]
                t0 = time.perf_counter()
                o.step(steps)
                dt = time.perf_counter() - t0
                row["threads_%d" % t] = (o.counters()["pushed"] - c0) / dt
            finally:
                oracle.set_threads(1)
            del o
        print("bench: %s: %s" % (name, row), file=sys.stderr, flush=True)
        rows.append(row)
    print(json.dumps({"cpu_oracle_particle_steps_per_s": rows, "host": host}), flush=True)


def launch_cfg(text: str) -> dict:
    """--launch "variant,electron_groups,sort_groups,append_groups[,sort_tile]" (0: default)."""
    v = [int(x) for x in text.split(",")]
    return dict(zip(["electron_variant", "electron_groups", "sort_groups", "append_groups",
                     "sort_tile"], v))


def batched(a):
    """Batched sweep: 64 independent discharges (64M electrons in total) in one
    launch per phase, against the same discharges as separate handles (one
    launch per discharge and phase, each on its own stream)."""
    import torch

    from paper_1508_02892_amd import hd, workloads as W
    ps = W.c3(n_discharges=a.discharges, total_electrons=a.total_electrons)
    print("bench: building batch of %d" % len(ps), file=sys.stderr, flush=True)
    b = hd.Batch(ps, device=0)
    # the batched sweep's launch shapes come from the autotuner (128 real
    # steps unless --tune-steps says otherwise), or from --launch
    if a.launch:
        b.set_launch(launch_cfg(a.launch))
        launch = b.get_launch()
    else:
        launch = b.autotune(a.tune_steps or 128)
    if a.copy_calib:  # a 1 GiB copy that scales the HBM counters of a profiled run
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    b.step(a.warmup)
    torch.cuda.synchronize()
    p0 = sum(b.moments(i)["pushed"] for i in range(len(ps)))
    t0 = time.perf_counter()
    b.step(a.steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    p1 = sum(b.moments(i)["pushed"] for i in range(len(ps)))
    value = (p1 - p0) / secs
    # the electron launch of the whole batch against the roofline, as for
    # the single discharge
    m1 = [b.moments(i) for i in range(len(ps))]
    kms = b.profile_steps(a.profile_steps)
    m2 = [b.moments(i) for i in range(len(ps))]
    n_push = sum(y["pushed"] - x["pushed"] for x, y in zip(m1, m2)) / a.profile_steps
    n_coll = sum(float(y["coll"].sum() - x["coll"].sum()) for x, y in zip(m1, m2)) / a.profile_steps
    alg_bytes = 36.0 * n_push + 8.0 * n_coll
    achieved = alg_bytes / (kms["electron"] * 1e-3) / 1e9
    b.close()
    del b
    sep = None
    if not a.no_separate:
        print("bench: separate handles", file=sys.stderr, flush=True)
        hs = [hd.Discharge(p, device=0) for p in ps]
        for h in hs:
            h.step(a.warmup)
        torch.cuda.synchronize()
        q0 = sum(h.moments()["pushed"] for h in hs)
        t0 = time.perf_counter()
        for h in hs:
            h.step(a.steps)
        torch.cuda.synchronize()
        s2 = time.perf_counter() - t0
        q1 = sum(h.moments()["pushed"] for h in hs)
        sep = {"value": (q1 - q0) / s2, "ms_per_step": s2 * 1e3 / a.steps}
        for h in hs:
            h.close()
    line = {
        "metric": "electron particle-steps/s (push+MCC+deposit), % HBM peak; p50/p99 job latency",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": secs * 1e3 / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched sweep: %d He discharges, gaps U(0.3,2) mm, 256-4096 "
                               "cells, 100-400 V, %d FP32 electrons in total, DD ions, one "
                               "launch per phase" % (len(ps), a.total_electrons)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_electron",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": kms["electron"]},
        "kernel_ms": kms,
        "one_launch_per_discharge": sep,
        "launch": launch,
    }
    print(json.dumps(line), flush=True)


def swarm(a):
    """Auxiliary ion swarm (Sec. II.C): 16 He+ swarms of 2^20 ions in fields
    log-spaced over 1e5 .. 1e7 V/m, 2 ns to the stationary drift, then 2 ns
    averaged; value = ion-steps/s of the averaged run."""
    import torch

    import numpy as np
    from paper_1508_02892_amd import hd, workloads as W
    p = W.swarm_bench()
    n_ion_steps = len(p["e0_V_m"]) * p["n_ions"]
    s = hd.Swarm(p, device=0)
    print("bench: swarm warmup %d steps" % W.SWARM_WARM, file=sys.stderr, flush=True)
    s.run(W.SWARM_WARM)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(W.SWARM_AVG, accumulate=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    res = s.results()
    e0 = 1.47e6
    table2 = [1e-3 * (1.18 - 0.185 * r["e0_V_m"] / e0) if r["e0_V_m"] < e0 else
              1e-3 * 0.94 * (e0 / r["e0_V_m"]) ** 0.3 for r in res]
    line = {
        "metric": "ion-steps/s (auxiliary ion Monte Carlo, accelerate + null-collision MCC)",
        "value": n_ion_steps * W.SWARM_AVG / secs, "unit": "ion-steps/s", "n_gpus": 1,
        "steps": W.SWARM_AVG, "warmup": W.SWARM_WARM, "ms_per_step": secs * 1e3 / W.SWARM_AVG,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ion swarm: He+ in He 1 atm 300 K, Q_m = Q_i + 2 Q_b, %d fields "
                               "1e5..1e7 V/m, %d ions each, dt 0.5 ps"
                               % (len(p["e0_V_m"]), p["n_ions"])},
        "mobility_vs_table2": [[r["e0_V_m"], r["mobility_m2_Vs"], t]
                               for r, t in zip(res, table2)],
        "nu_s": [r["nu_s"] for r in res],
        "table_overflow_per_collision": sum(r["overflow"] for r in res) /
        max(1, sum(r["collisions"] for r in res)),
    }
    if not a.no_cpu:
        import oracle
        q = dict(p, n_ions=4096)
        orc = oracle.Swarm(q)
        t1 = time.perf_counter()
        orc.run(W.SWARM_WARM)
        orc.run(W.SWARM_AVG, accumulate=True)
        dt = time.perf_counter() - t1
        n = 4096 * len(p["e0_V_m"]) * (W.SWARM_WARM + W.SWARM_AVG)
        line["cpu_baseline"] = {"value": n / dt, "unit": "ion-steps/s", "cores": 1,
                                "kind": "oracle",
                                "sample": "the same 16 fields with 4,096 ions each, %d steps "
                                          "(%d ion-steps, %.1f s), single thread"
                                          % (W.SWARM_WARM + W.SWARM_AVG, n, dt)}
    s.close()
    del np
    print(json.dumps(line), flush=True)


def served(a):
    """Served job stream: Poisson arrivals of discharge jobs drawn like the
    batched sweep, admitted by HBM budget into continuously batched slots;
    reports aggregate particle-steps/s and p50/p99 submit-to-result latency."""
    import numpy as np

    from paper_1508_02892_amd import hd, workloads as W

    def stream(rate):
        jobs = W.c4_jobs(rate_per_s=rate, duration_s=a.duration, seed=4,
                         size_scale=a.size_scale, steps_range=(a.min_steps, a.max_steps))
        srv = hd.Server(precision=0, max_slots=a.slots, max_cells=4096,
                        hbm_budget_bytes=int(a.budget_gb * 1e9))
        print("bench: serving %d jobs at %g/s" % (len(jobs), rate), file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        ids = []
        for j in jobs:
            wait = t0 + j["arrival_s"] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            ids.append(srv.submit(j["params"], j["steps"]))
        srv.drain(3600.0)
        wall = time.perf_counter() - t0
        lat = np.array([srv.poll(i)[1][1] for i in ids])
        st = srv.stats()
        srv.close()
        print("bench: %d jobs done in %.1f s" % (len(jobs), wall), file=sys.stderr, flush=True)
        return jobs, wall, lat, st

    jobs, wall, lat, st = stream(a.rate)
    sub = None
    if a.sub_rate > 0:
        j2, w2, l2, s2 = stream(a.sub_rate)
        sub = {"rate_jobs_per_s": a.sub_rate, "jobs": len(j2),
               "value": s2["particle_steps"] / w2, "wall_s": w2,
               "latency_s": {"p50": float(np.percentile(l2, 50)),
                             "p99": float(np.percentile(l2, 99)), "max": float(l2.max())}}
    line = {
        "metric": "electron particle-steps/s (push+MCC+deposit), % HBM peak; p50/p99 job latency",
        "value": st["particle_steps"] / wall, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": int(sum(j["steps"] for j in jobs)), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served job stream: Poisson arrivals %.3g jobs/s for %.0f s, "
                               "sizes log-uniform [2^18, 2^23] x %.3g electrons, %d-%d steps, "
                               "%d slots, %.0f GB budget"
                               % (a.rate, a.duration, a.size_scale, a.min_steps, a.max_steps,
                                  a.slots, a.budget_gb),
                   "jobs": len(jobs)},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "server": st,
        "sub_saturation": sub,
        "wall_s": wall,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--profile-steps", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=96)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ion", choices=["default", "dd", "full", "dd-fit", "full-fit"],
                    default="default",
                    help="override the ion model of the workload (diagnostic variants)")
    ap.add_argument("--power-w-m2", type=float, default=0.0,
                    help="enable power control (Eq 2.9) with this P_0 per electrode area")
    ap.add_argument("--power-alpha", type=float, default=0.05)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration runs)")
    ap.add_argument("--rate", type=float, default=20.0, help="served stream: jobs/s")
    ap.add_argument("--sub-rate", type=float, default=7.0,
                    help="served stream: a second, sub-saturation arrival rate (0: none)")
    ap.add_argument("--duration", type=float, default=20.0,
                    help="served stream: arrival window in seconds (the stated stream is 600 s)")
    ap.add_argument("--size-scale", type=float, default=1.0)
    ap.add_argument("--min-steps", type=int, default=2000)
    ap.add_argument("--max-steps", type=int, default=20000)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--discharges", type=int, default=64, help="batched sweep size")
    ap.add_argument("--total-electrons", type=int, default=1 << 26)
    ap.add_argument("--no-separate", action="store_true")
    ap.add_argument("--electrons", type=int, default=0,
                    help="override the superparticle count (diagnostic variants)")
    ap.add_argument("--launch", default="",
                    help="launch shape variant,electron_groups,sort_groups,append_groups "
                         "(0: default) instead of the autotuner")
    ap.add_argument("--tune-steps", type=int, default=0,
                    help="steps the autotuner may take (within the warmup); 0: no tuning")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: runs on one GPU only (got --gpus %d): independent discharges would "
              "be spread over GPUs one process each, which is not implemented" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.workload == "served":
        return served(a)
    if a.workload == "batched":
        return batched(a)
    if a.workload == "swarm":
        return swarm(a)
    if a.workload == "cpu":
        return cpu_table(a)

    import torch
    from paper_1508_02892_amd import hd

    torch.cuda.set_device(0)
    p, desc = workload(a.workload)
    if a.ion != "default":
        p["ion_model"], name = {
            "dd": (0, "drift-diffusion, constant mobility"),
            "full": (1, "full fluid, constant nu"),
            "dd-fit": (2, "drift-diffusion, mobility of Table 2"),
            "full-fit": (3, "full fluid, nu of Table 3")}[a.ion]
        desc += "; ion model overridden: %s" % name
    if a.power_w_m2 > 0:
        p["power_W_m2"], p["power_alpha"] = a.power_w_m2, a.power_alpha
        desc += "; power control P_0 = %g W/m^2, alpha = %g" % (a.power_w_m2, a.power_alpha)
    if a.electrons:
        from paper_1508_02892_amd import workloads as W
        p = W.scaled(p, a.electrons)
        desc += "; electrons overridden: %d" % a.electrons
    dev = hd.Discharge(p, device=0)
    if a.launch:
        dev.set_launch(launch_cfg(a.launch))
    elif a.tune_steps:
        print("bench: autotuning over %d steps" % a.tune_steps, file=sys.stderr, flush=True)
        dev.autotune(a.tune_steps)
    launch = dev.get_launch()
    if a.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # untimed warmup: at least the steps asked for, up to the next sort
    # interval boundary, so that the timed steps start with a captured
    # interval (the tuner's steps, if any, came before)
    se = int(p["sort_every"])
    done = dev.moments()["step"]
    warm = a.warmup + (-(done + a.warmup)) % se
    print("bench: warmup %d steps (asked %d; from step %d to an interval boundary)"
          % (warm, a.warmup, done), file=sys.stderr, flush=True)
    dev.step(warm)
    torch.cuda.synchronize()
    m0 = dev.moments()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev.step(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m1 = dev.moments()
    pushed = m1["pushed"] - m0["pushed"]
    secs = t1 - t0
    value = pushed / secs
    graph_steps = m1["graph_steps"] - m0["graph_steps"]
    sorts = (m1["step"] // se) - (m0["step"] // se)
    print("bench: timed %d steps in %.3f s (%d replayed from captured intervals, %d sorts)"
          % (a.steps, secs, graph_steps, sorts), file=sys.stderr, flush=True)

    kms = dev.profile_steps(a.profile_steps)
    m2 = dev.moments()
    n_push = (m2["pushed"] - m1["pushed"]) / a.profile_steps
    n_coll = float(m2["coll"].sum() - m1["coll"].sum()) / a.profile_steps
    fp32 = p["precision"] == 0
    per_particle = 36.0 if fp32 else 60.0
    per_coll = 8.0 if fp32 else 16.0
    alg_bytes = per_particle * n_push + per_coll * n_coll
    achieved = alg_bytes / (kms["electron"] * 1e-3) / 1e9
    # the recorded counters belong to the default workload in its default
    # launch shape only
    default_run = (a.workload == "c1" and a.ion == "default" and a.power_w_m2 <= 0
                   and not a.electrons and launch["electron_variant"] == 0)
    traffic = read_traffic() if default_run else None
    copy_gbs = measured_copy_gbs()
    line = {
        "metric": "electron particle-steps/s (push+MCC+deposit), % HBM peak; p50/p99 job latency",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": secs * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "electrons": int(p["n_macro"]), "cells": p["n_cells"],
                   "live_electrons_end": int(m1["n_live"]), "parallelism": "1 GPU",
                   "warmup_steps_run": warm, "timed_graph_steps": graph_steps,
                   "timed_sorts": sorts},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_electron", "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": kms["electron"], "copy_measured": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs},
        "kernel_ms": kms,
        "launch": launch,
    }
    if not a.no_cpu:
        print("bench: cpu baseline (%d oracle steps)" % a.cpu_steps, file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, a.cpu_steps, desc)
        line["fp32_vs_fp64"] = precision_leg()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
