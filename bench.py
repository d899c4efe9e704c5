#!/usr/bin/env python3
"""Throughput benchmark of the hybrid PIC/MCC hot path on one MI355X.

Workload (default): the single large discharge -- helium at 1 atm, 1 mm gap,
2,048 cells, 250 V at 13.56 MHz, 8,388,608 FP32 electron superparticles,
full-inertia ion fluid, re-sort every 16 steps -- with seeded synthetic
cross sections and initial load.  A step is one pass of the whole hot path
(field, ion fluid, push / MCC / deposit, emission, append, sort when due).

The timed region is --steps steps replayed from captured graphs with the
particle state resident in HBM, bracketed by device synchronisation.  value
= particle-steps (live electrons pushed, counted on the device) / seconds.

roofline: the fused electron kernel is timed with HIP events on the
library's stream over --profile-steps further real steps; its algorithmic
bytes are 36 B per FP32 particle-step (read cell, offset, three velocities
and id; write cell, offset, v_z) plus 8 B per collision (v_x, v_y).
traffic: HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
(profiles/), scaled by the same counters on a plain copy of known size;
null when the kernel source changed since they were taken.
cpu_baseline: the CPU oracle on this host, single thread, for a bounded
number of steps of the same workload.
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
    if name == "c0":
        return W.c0(), ("small plain discharge: He 1 atm, 0.5 mm, 256 cells, 150 V, "
                        "16,384 FP64 electrons, drift-diffusion ions")
    raise SystemExit("unknown workload " + name)


def cpu_baseline(p, steps: int, desc: str):
    import oracle
    orc = oracle.Oracle(p)
    c0 = orc.counters()["pushed"]
    t0 = time.perf_counter()
    orc.step(steps)
    dt = time.perf_counter() - t0
    n = orc.counters()["pushed"] - c0
    return {"value": n / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%s; %d steps after the initial load (%d particle-steps, %.1f s), "
                      "single thread" % (desc, steps, n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--profile-steps", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ion", choices=["default", "dd", "full"], default="default",
                    help="override the ion model of the workload (diagnostic variants)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration runs)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (got --gpus %d); the multi-GPU "
              "design is described in DESIGN.md and not measured" % a.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1508_02892_amd import hd

    torch.cuda.set_device(0)
    p, desc = workload(a.workload)
    if a.ion != "default":
        p["ion_model"] = 0 if a.ion == "dd" else 1
        desc += "; ion model overridden: %s" % ("drift-diffusion" if a.ion == "dd" else "full")
    dev = hd.Discharge(p, device=0)
    if a.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print("bench: warmup %d steps" % a.warmup, file=sys.stderr, flush=True)
    dev.step(a.warmup)
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
    print("bench: timed %d steps in %.3f s" % (a.steps, secs), file=sys.stderr, flush=True)

    kms = dev.profile_steps(a.profile_steps)
    m2 = dev.moments()
    n_push = (m2["pushed"] - m1["pushed"]) / a.profile_steps
    n_coll = float(m2["coll"].sum() - m1["coll"].sum()) / a.profile_steps
    fp32 = p["precision"] == 0
    per_particle = 36.0 if fp32 else 60.0
    per_coll = 8.0 if fp32 else 16.0
    alg_bytes = per_particle * n_push + per_coll * n_coll
    achieved = alg_bytes / (kms["electron"] * 1e-3) / 1e9
    traffic = read_traffic()
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
                   "live_electrons_end": int(m1["n_live"]), "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_electron", "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": kms["electron"]},
        "kernel_ms": kms,
    }
    if not a.no_cpu:
        print("bench: cpu baseline (%d oracle steps)" % a.cpu_steps, file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, a.cpu_steps, desc)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
