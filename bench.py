"""Benchmark: one step = the whole hot path on the 32^3-cell, 20,000-line,
50,000-point, 2^20-ray workload (Gaussian hot spot 400-1800 K, x_H2O
U[0.05, 0.2], 1 m cube), inputs resident on the GPU:

    compute_kappa (Eq. (1)-(2) line sum + Eq. (4) Planck table)
    -> trace_rays (Philox rays, integer traversal, Eq. (3) march, tallies)
    -> tally (energy balance, per-cell powers to the host)

Prints one JSON line.  `value` is ray-cell-nu updates per second of the whole
step; the line-sum rate, the march roofline and the FP64 CPU oracle timed on a
bounded sample are reported beside it.  One GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ray·cell·nu updates/s + line evals/s; "
          "surrogate vs plain at ≤1e-3 rel power")

# Algorithmic work per ray-cell-nu update of Eq. (3) with the Planck value
# read once per (cell, nu) from a table: x = kappa * (-l log2 e), t = 2^x,
# a = 1 - t, d = I - B, I -= d a, absorbed += I a, emitted += B a:
# 9 FP32 flops (an FMA counts 2) in 6 full-rate VALU issue slots, plus one
# base-2 exponential.
MARCH_FLOPS_PER_UPDATE = 9.0
MARCH_SLOTS_PER_UPDATE = 6.0
# MI355X: 256 CUs x 64 FP32 lanes x 2.4 GHz = 39.32e12 lane-slots/s (packed
# FP32 is not used).  The hardware exponential issues at half rate on gfx950
# (2 slots), as measured by paper_cs_0703028_amd/probe/alu_rates.hip.
LANE_SLOTS_PER_S = 256 * 64 * 2.4e9
TRANS_SLOTS = 2.0


def march_peak_updates_per_s():
    return LANE_SLOTS_PER_S / (MARCH_SLOTS_PER_UPDATE + TRANS_SLOTS)


def cpu_baseline(w, n_cells_sample=32, n_rays_sample=96):
    """Time the FP64 oracle on a bounded sample of the same workload and
    extrapolate linearly to the full step."""
    import numpy as np

    from oracle import oracle as O

    g, L = w.grid, w.lines
    rng = np.random.default_rng(0)
    cells = np.sort(rng.choice(g.n_cells, n_cells_sample, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    kap = O.kappa(g, L, cells)
    B = O.planck_rows(g, L, cells)
    t_kappa = time.perf_counter() - t0
    Os, Ds, _ = O.rays(w.seed, 0, n_rays_sample, g.nx, g.ny, g.nz)
    # the march's cost does not depend on the values: every visited cell
    # reads one of the sampled rows
    row = (np.arange(g.n_cells) % n_cells_sample).astype(np.int32)
    segs = 0
    for k in range(n_rays_sample):
        segs += len(O.segments(g.nx, g.ny, g.nz, g.cell_m * 100.0, Os[k], Ds[k])[0])
    t0 = time.perf_counter()
    O.march(g, L, Os, Ds, O.ray_weight(g, L, w.n_rays), kap, B, cell_row=row)
    t_march = time.perf_counter() - t0
    total_s = t_kappa * g.n_cells / n_cells_sample + t_march * w.n_rays / n_rays_sample
    updates_total = segs / n_rays_sample * w.n_rays * L.n_nu
    return {
        "value": updates_total / total_s,
        "unit": "ray·cell·nu updates/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle: kappa+Planck rows of {n_cells_sample} cells x {L.n_nu} nu "
                   f"({t_kappa:.2f} s, OpenMP over cells) and the march of rays 0..{n_rays_sample-1} "
                   f"x {L.n_nu} nu ({t_march:.2f} s, one thread), extrapolated linearly to "
                   f"{g.n_cells} cells and {w.n_rays} rays"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="plain_32cube")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the spectral-range sharding is described in the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_cs_0703028_amd import inputs as I
    from paper_cs_0703028_amd import rtlbl

    w = getattr(I, args.workload)()
    t = rtlbl.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(w.lines)
    kap, B = t.alloc_tables()

    def step():
        t.reset_tally()
        t.compute_kappa(rtlbl.KAPPA_PLAIN, kap, B)
        t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, rtlbl.TALLY_F32)
        return t.tally()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = t.stats()  # drains the warmup timers
    t.reset_tally()
    kappa_ms = march_ms = 0.0
    launches = updates = evals = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, e, bal = step()
        st = t.stats()
        kappa_ms += st["kappa_ms"]
        march_ms += st["march_ms"]
        launches += st["march_launches"]
        updates += st["updates"]
        evals += st["line_evals"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / args.steps * 1e3
    value = updates / dt
    kappa_ms_timed = kappa_ms
    peak = march_peak_updates_per_s()
    march_rate = updates / (march_ms * 1e-3)
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "ray·cell·nu updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": w.grid.n_cells, "lines": int(len(w.lines.nu)),
                   "n_nu": w.lines.n_nu, "rays": w.n_rays, "kappa_mode": "plain",
                   "tally": "f32 partials, f64 accumulators"},
        "line_evals_per_s": evals / (kappa_ms_timed * 1e-3) if kappa_ms_timed > 0 else None,
        "trace_updates_per_s": march_rate,
        "energy_balance_rel": float(abs(bal[0] + bal[1] - bal[2] - bal[3]) / (bal[0] + bal[1])),
        "roofline": {
            "bound": "alu",
            "kernel": "march_kernel",
            "achieved": march_rate * MARCH_FLOPS_PER_UPDATE / 1e12,
            "peak": peak * MARCH_FLOPS_PER_UPDATE / 1e12,
            "unit": "TFLOP/s",
            "frac": march_rate / peak,
            "traffic": None,
            "launches": launches,
            "avg_launch_ms": march_ms / launches if launches else None,
        },
    }
    t.close()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
