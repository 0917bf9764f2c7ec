"""Benchmark: one step = the whole hot path on the 32^3-cell, 20,000-line,
50,000-point, 2^20-ray workload (Gaussian hot spot 400-1800 K, x_H2O
U[0.05, 0.2], 1 m cube), inputs resident on the GPU:

    compute_kappa (Eq. (1)-(2) line sum)
    -> trace_rays (Philox rays, integer traversal, Eq. (3) march with the
       Eq. (4) Planck values formed in registers, per-cell tallies)
    -> tally (energy balance, per-cell powers to the host)

Prints one JSON line.  `value` is ray-cell-nu updates per second of the whole
step; the line-sum rate, the march roofline and the FP64 CPU oracle timed on a
bounded sample are reported beside it, and `forms` carries the precision,
batched and learned forms, each on its own workload.  One GPU only.
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
# read once per (cell, nu): x = kappa * (-l log2 e), t = 2^x, a = 1 - t,
# d = I - B, I -= d a, absorbed += I a, emitted += B a: 9 FP32 flops (an FMA
# counts 2) in 6 full-rate VALU issue slots, plus one base-2 exponential.
MARCH_FLOPS_PER_UPDATE = 9.0
MARCH_SLOTS_PER_UPDATE = 6.0
# MI355X: 256 CUs x 64 FP32 lanes x 2.4 GHz = 39.32e12 lane-slots/s (packed
# FP32 is not used).  The hardware exponential and reciprocal issue at half
# rate on gfx950 (2 slots), as measured by paper_cs_0703028_amd/probe/alu_rates.hip.
LANE_SLOTS_PER_S = 256 * 64 * 2.4e9
TRANS_SLOTS = 2.0
# Eq. (2) per in-window (cell, line, nu) triple, with the squared offset
# shared by the cells of a tile: g2 + d^2 (1 add), reciprocal, acc += A * rcp
# (1 FMA): 4 FP32 flops in 2 full-rate slots plus one half-rate reciprocal.
LINE_FLOPS_PER_EVAL = 4.0
LINE_SLOTS_PER_EVAL = 2.0 + TRANS_SLOTS
# MI355X published vector peaks: FP32 157.3 TFLOP/s counts packed (dual) FP32
# FMAs, which this build does not use; one FMA per lane and cycle is 78.6.
FP32_PUBLISHED_PEAK = 157.3e12
FP32_UNPACKED_FMA_PEAK = 78.6e12
BF16_DENSE_PEAK = 2.5e15
MLP_WEIGHTS = 4 * 512 + 512 * 512 + 512 * 512 + 512 * 256
TUNING_CACHE = os.path.join(ROOT, "paper_cs_0703028_amd", "tuning", "batch_tune.json")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "march_kernel_plain_32cube_hbm_counters.md")
MARCH_SOURCES = ("paper_cs_0703028_amd/csrc/march.hip", "paper_cs_0703028_amd/csrc/device_common.h",
                 "paper_cs_0703028_amd/csrc/rt_internal.h")


def measured_traffic():
    """HBM bytes per march launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None once the march sources differ from the profiled ones."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        h = hashlib.sha256()
        for s in MARCH_SOURCES:
            h.update(open(os.path.join(ROOT, s), "rb").read())
        fields = dict(line.split(": ", 1) for line in text.splitlines()
                      if line.startswith(("traffic_bytes_per_launch: ", "source_sha256: ")))
        if fields.get("source_sha256", "").strip() != h.hexdigest():
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def march_peak_updates_per_s():
    return LANE_SLOTS_PER_S / (MARCH_SLOTS_PER_UPDATE + TRANS_SLOTS)


def line_peak_evals_per_s():
    return LANE_SLOTS_PER_S / LINE_SLOTS_PER_EVAL


def cpu_baseline(w, n_cells_sample=256, n_rays_sample=768, n_cells_one=16):
    """Time the FP64 oracle on a bounded sample of the same workload and
    extrapolate linearly to the full step, on all host threads and on one.
    All threads: kappa and Planck rows of sampled cells (OpenMP over cells)
    and the march of one slice of rays per thread (the oracle's march called
    from a thread pool on disjoint rays; ctypes releases the interpreter
    lock).  One thread: fewer rows, and one slice of rays."""
    import concurrent.futures as cf

    import numpy as np

    from oracle import oracle as O

    g, L = w.grid, w.lines
    threads = O.num_threads()
    rng = np.random.default_rng(0)
    cells = np.sort(rng.choice(g.n_cells, n_cells_sample, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    kap = O.kappa(g, L, cells)
    B = O.planck_rows(g, L, cells)
    t_kappa = time.perf_counter() - t0
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.kappa(g, L, cells[:n_cells_one])
        O.planck_rows(g, L, cells[:n_cells_one])
        t_kappa_one = time.perf_counter() - t0
    finally:
        O.set_num_threads(threads)
    # the march's cost does not depend on the values: every visited cell
    # reads one of the sampled rows
    row = (np.arange(g.n_cells) % n_cells_sample).astype(np.int32)
    wgt = O.ray_weight(g, L, w.n_rays)
    slices = [O.rays(w.seed, k * n_rays_sample, n_rays_sample, g.nx, g.ny, g.nz)[:2]
              for k in range(threads)]
    segs = 0
    for Os, Ds in slices:
        for k in range(n_rays_sample):
            segs += len(O.segments(g.nx, g.ny, g.nz, g.cell_m * 100.0, Os[k], Ds[k])[0])
    seg_per_ray = segs / (threads * n_rays_sample)
    t0 = time.perf_counter()
    O.march(g, L, slices[0][0], slices[0][1], wgt, kap, B, cell_row=row)
    t_march_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda sl: O.march(g, L, sl[0], sl[1], wgt, kap, B, cell_row=row), slices))
    t_march = time.perf_counter() - t0
    updates_total = seg_per_ray * w.n_rays * L.n_nu
    total_s = (t_kappa * g.n_cells / n_cells_sample
               + t_march * w.n_rays / (threads * n_rays_sample))
    total_one = (t_kappa_one * g.n_cells / n_cells_one
                 + t_march_one * w.n_rays / n_rays_sample)
    return {
        "value": updates_total / total_s,
        "unit": "ray·cell·nu updates/s",
        "cores": threads,
        "kind": "oracle",
        "value_1core": updates_total / total_one,
        "sample": (f"FP64 oracle on {threads} threads: kappa+Planck rows of {n_cells_sample} cells "
                   f"x {L.n_nu} nu ({t_kappa:.2f} s, OpenMP over cells) and the march of "
                   f"{threads} x {n_rays_sample} rays x {L.n_nu} nu ({t_march:.2f} s, one slice of "
                   f"rays per thread); on one thread: {n_cells_one} rows ({t_kappa_one:.2f} s) and "
                   f"{n_rays_sample} rays ({t_march_one:.2f} s); both extrapolated linearly to "
                   f"{g.n_cells} cells and {w.n_rays} rays"),
    }


def _rel(g, o):
    import numpy as np
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    nz = o != 0
    return float(np.max(np.abs(g[nz] - o[nz]) / np.abs(o[nz]))) if nz.any() else 0.0


def form_precision(rtlbl, I):
    """Precision form on the 8^3 workload: compensated line sums, Planck
    table, FP64 partial sums; the error of each result against the FP64
    oracle, plus the 1 m isothermal slab against its closed form."""
    import numpy as np
    import torch

    from oracle import oracle as O
    w = I.plain_8cube()
    t = rtlbl.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(w.lines)
    kap, B = t.alloc_tables()

    def step():
        t.reset_tally()
        t.compute_kappa(rtlbl.KAPPA_COMPENSATED, kap, B)
        t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, rtlbl.TALLY_F64)
        return t.tally()

    step()
    torch.cuda.synchronize()
    t.stats()
    t0 = time.perf_counter()
    a, e, b = step()
    dt = time.perf_counter() - t0
    st = t.stats()
    ref = O.run(w.grid, w.lines, w.n_rays, seed=w.seed)
    n = w.lines.n_nu
    out = {
        "workload": w.name,
        "ms_per_step": dt * 1e3,
        "updates_per_s": st["updates"] / dt,
        "line_evals_per_s_kappa": st["line_evals"] / (st["kappa_ms"] * 1e-3),
        "err_vs_fp64_oracle_max_rel": {
            "kappa": _rel(kap.cpu().numpy()[:, :n], ref["kappa"]),
            "planck": _rel(B.cpu().numpy()[:, :n], ref["planck"]),
            "absorbed": _rel(a, ref["absorbed"]),
            "emitted": _rel(e, ref["emitted"]),
            "balance": _rel(b, ref["balance"]),
        },
        "energy_balance_residual": float(abs(b[0] + b[1] - b[2] - b[3]) / (b[0] + b[1])),
    }
    t.close()
    s = I.slab_1cell()
    t = rtlbl.Tracer(0)
    t.setup_grid(s.grid)
    t.setup_lines(s.lines)
    t.compute_kappa(rtlbl.KAPPA_COMPENSATED)
    U = 1 << 21
    ex = t.trace_explicit(np.array([[0, U // 2 + 1, U // 2 + 1]]), np.array([[1 << 20, 0, 0]]),
                          1.0, prec=rtlbl.TALLY_F64, want_exit=True)[0]
    t.close()
    k = O.kappa(s.grid, s.lines)[0]
    Bc = O.planck_rows(s.grid, s.lines)[0]
    nu = s.lines.nu0 + np.arange(s.lines.n_nu) * s.lines.dnu
    Bw = np.array([O.planck(v, s.grid.T_wall) for v in nu])
    tr = np.exp(-k * s.grid.cell_m * 100.0)
    closed = Bw * tr + Bc * (1 - tr)
    out["slab_1m_exit_radiance_max_rel_vs_closed_form"] = _rel(ex, closed)
    # the same slab with 1,024 random boundary rays, against the oracle
    t = rtlbl.Tracer(0)
    t.setup_grid(s.grid)
    t.setup_lines(s.lines)
    t.compute_kappa(rtlbl.KAPPA_COMPENSATED)
    t.trace_rays(s.seed, s.n_rays, 0, s.n_rays, rtlbl.TALLY_F64)
    a, e, b = t.tally()
    t.close()
    ref = O.run(s.grid, s.lines, s.n_rays, seed=s.seed)
    out["slab_1m_random_rays_err_vs_fp64_oracle_max_rel"] = {
        "absorbed": _rel(a, ref["absorbed"]), "emitted": _rel(e, ref["emitted"]),
        "balance": _rel(b, ref["balance"])}
    return out


def form_batched(rtlbl, I):
    """Batched form: 64 receiver cases (16^3-48^3 cells, 2^14-2^18 rays, 5,000
    lines, 20,000 points) in one graph launch, with the launch shape and
    tuning looked up in (or written to) the autotuner's cache."""
    import numpy as np
    import torch
    cases = I.batched_cases(64)
    t = rtlbl.Tracer(0)
    t.setup_lines(cases[0].lines)
    # room for the largest trial of either launch shape
    big = rtlbl.Tracer.default_tuning()
    big.chunk_points = 4 * rtlbl.MARCH_CHUNK
    big.blocks_per_cu = 4
    big.slots = 8
    big.mode = rtlbl.BATCH_PERSISTENT
    nbytes = t.batch_workspace_size(cases, big)
    big.mode = rtlbl.BATCH_CHUNKED  # one slab of 3072 points for every cell
    big.chunk_points = 2 * rtlbl.MARCH_CHUNK
    big.slots = 1
    nbytes = max(nbytes, t.batch_workspace_size(cases, big))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    best = t.batch_autotune(cases, rtlbl.KAPPA_PLAIN, ws, TUNING_CACHE)
    tune_s = time.perf_counter() - t0
    t.batch_prepare(cases, rtlbl.KAPPA_PLAIN, best, ws)
    t.batch_launch()
    t.batch_results()
    t.stats()
    t0 = time.perf_counter()
    t.batch_launch()
    res = t.batch_results()
    dt = time.perf_counter() - t0
    st = t.stats()
    t.close()
    bal = np.array([r[2] for r in res])
    # The same 64 cases one after another through the single-case calls
    # (compute_kappa into a full table, then trace_rays): the unfused
    # reference at these cases' own ray densities.
    u = rtlbl.Tracer(0)
    u.setup_lines(cases[0].lines)
    ld = u.required_pitch()
    kap = torch.empty((max(c.grid.n_cells for c in cases), ld), dtype=torch.float32,
                      device="cuda")
    worst = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, c in enumerate(cases):
        u.setup_grid(c.grid)
        u.compute_kappa(rtlbl.KAPPA_PLAIN, kap[:c.grid.n_cells], None)
        u.trace_rays(c.seed, c.n_rays)
        a_single = u.tally()[0]
        a_batch = res[k][0]
        m = a_single > 0
        worst = max(worst, float(np.max(np.abs(a_batch[m] - a_single[m]) / a_single[m])))
    unfused_s = time.perf_counter() - t0
    su = u.stats()
    u.close()
    del kap
    torch.cuda.empty_cache()
    return {
        "unfused_case_by_case": {
            "s_wall": unfused_s, "kappa_ms": su["kappa_ms"], "trace_ms": su["trace_ms"],
            "batched_speedup": unfused_s / dt,
            "absorbed_max_rel_diff_batched_vs_case_by_case": worst},
        "workload": "64 cases, 16^3-48^3 cells, 2^14-2^18 rays, 5,000 lines, 20,000 nu",
        "cells": int(sum(c.grid.n_cells for c in cases)),
        "rays": int(sum(c.n_rays for c in cases)),
        "ms_per_launch": dt * 1e3,
        "device_ms": st["batch_ms"],
        "updates": st["batch_updates"],
        "line_evals": st["batch_line_evals"],
        "updates_per_s": st["batch_updates"] / dt,
        "line_evals_per_s": st["batch_line_evals"] / dt,
        # the line sum and the march share the launch: each phase's rate over
        # its own VALU ceiling, and their sum (the share of the launch's VALU
        # capacity the algorithmic work fills)
        "frac_of_valu_ceiling": {
            "line_sum": st["batch_line_evals"] / dt / line_peak_evals_per_s(),
            "march": st["batch_updates"] / dt / march_peak_updates_per_s(),
            "both": (st["batch_line_evals"] / dt / line_peak_evals_per_s()
                     + st["batch_updates"] / dt / march_peak_updates_per_s())},
        "tuning": best.as_dict(),
        "tuning_s": tune_s,
        "energy_balance_residual_max": float(np.max(
            np.abs(bal[:, 0] + bal[:, 1] - bal[:, 2] - bal[:, 3]) / (bal[:, 0] + bal[:, 1]))),
    }


# the learned form's training: 2^16 states, batch 1024, Adam with a cosine
# decay from this initial step
LEARNED_EPOCHS = 80
LEARNED_LR = 2e-3


def form_learned(rtlbl, I, epochs=LEARNED_EPOCHS, n_lines=None, model_path=None):
    """Learned form on the 8^3 workload: train the MLP on 2^16 line-sum
    spectra, then take kappa from it (range check, sampled check, line-sum
    fallback) for the plain march; error and speed-up against the line sum.
    n_lines replaces the 500-line list by a denser one over the same
    1000-1100 cm^-1 (the line sum's cost grows with it, the network's does
    not).  model_path: load the network from there if the file exists,
    otherwise train and save it there (so that a profiled run need not
    train)."""
    import numpy as np
    import torch
    w = I.plain_8cube()
    if n_lines is not None:
        dense = I.line_list(n_lines, 1000.0, 1100.0, n_nu=w.lines.n_nu)
        w = I.with_lines(w, **vars(dense))
        w.name = f"plain_8cube_{n_lines}lines_10k_nu_1024rays"
    t = rtlbl.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(w.lines)
    t0 = time.perf_counter()
    if model_path and os.path.exists(model_path):
        t.surrogate_load(model_path)
        loss = None
    else:
        T, x, p = I.surrogate_samples(1 << 16, seed=0)
        loss = t.surrogate_train(T, x, p, I.SURROGATE_BOX, epochs=epochs, batch=1024,
                                 lr=LEARNED_LR, seed=0, check_cells=32, tolerance=5e-4)
        if model_path:
            t.surrogate_save(model_path)
    train_s = time.perf_counter() - t0 if loss is not None else None
    kap = torch.empty((w.grid.n_cells, t.required_pitch()), dtype=torch.float32, device="cuda")

    def run(mode, reps=5):
        best = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            t.compute_kappa(mode, kap, None)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - a)
        t.reset_tally()
        t.trace_rays(w.seed, w.n_rays)
        return best, t.tally()

    t_plain, (a0, e0, _) = run(rtlbl.KAPPA_PLAIN)
    t_sur, (a1, e1, _) = run(rtlbl.KAPPA_SURROGATE)
    st = t.surrogate_stats()
    # phase times from timing events, in calls of their own (the events
    # would slow the timed calls above); best of five each
    t.surrogate_time_phases(True)
    phases = []
    for _ in range(5):
        t.compute_kappa(rtlbl.KAPPA_SURROGATE, kap, None)
        s = t.surrogate_stats()
        phases.append((s["infer_ms"], s["check_ms"], s["fallback_ms"]))
    t.surrogate_time_phases(False)
    st["infer_ms"], st["check_ms"], st["fallback_ms"] = (min(v) for v in zip(*phases))
    t.close()
    ra = np.abs(a1 - a0)[a0 > 0] / a0[a0 > 0]
    re_ = np.abs(e1 - e0)[e0 > 0] / e0[e0 > 0]
    # the network's rows: every chunk but a last one the spectrum ends inside
    # (summed exactly in the same launch).  infer_ms times that whole launch,
    # whose line-sum blocks (the check's exact rows, the last chunk) run on
    # the CUs the network leaves free, so the rate is the launch's
    flops = 2.0 * MLP_WEIGHTS * w.grid.n_cells * (st["n_chunks"] - st["exact_chunks"])
    return {
        "workload": w.name,
        "train_s": train_s,
        "train_samples": 1 << 16,
        "epochs": epochs if loss is not None else None,
        "train_mse_normalised": loss,
        "kappa_ms_surrogate": t_sur * 1e3,
        "kappa_ms_plain_line_sum": t_plain * 1e3,
        "speedup_vs_plain": t_plain / t_sur,
        "mlp_infer_ms": st["infer_ms"],
        "mlp_check_ms": st["check_ms"],
        "mlp_fallback_ms": st["fallback_ms"],
        "mlp_tflops": flops / (st["infer_ms"] * 1e-3) / 1e12 if st["infer_ms"] > 0 else None,
        "mlp_frac_of_bf16_peak": (flops / (st["infer_ms"] * 1e-3) / BF16_DENSE_PEAK
                                  if st["infer_ms"] > 0 else None),
        "fallback_chunks": st["fallback_chunks"],
        "fallback_cells": st["fallback_cells"],
        "n_chunks": st["n_chunks"],
        "exact_chunks": st["exact_chunks"],
        "check_error_max": st["check_error"],
        "rel_err_vs_plain_max": {"absorbed": float(ra.max()), "emitted": float(re_.max())},
        "within_1e-3": bool(max(ra.max(), re_.max()) <= 1e-3),
    }


def form_two_gases(rtlbl, I, reps=3):
    """Eq. (2) with two absorbers on the 32^3 grid: the 20,000 H2O-like lines
    plus 10,000 CO2-like lines at their own mole fractions.  The kappa table
    is the sum of the two line sums; reported: line evaluations per second of
    compute_kappa against the line-sum VALU ceiling."""
    import torch
    w = I.plain_32cube_two_gases()
    t = rtlbl.Tracer(0)
    t.setup_workload(w)
    kap = torch.empty((w.grid.n_cells, t.required_pitch()), dtype=torch.float32, device="cuda")
    t.compute_kappa(rtlbl.KAPPA_PLAIN, kap, None)          # warm-up
    torch.cuda.synchronize()
    s0 = t.stats()
    for _ in range(reps):
        t.compute_kappa(rtlbl.KAPPA_PLAIN, kap, None)
    torch.cuda.synchronize()
    s1 = t.stats()
    ms = (s1["kappa_ms"] - s0["kappa_ms"]) / reps
    evals = (s1["line_evals"] - s0["line_evals"]) / reps
    rate = evals / (ms * 1e-3)
    t.close()
    del kap
    torch.cuda.empty_cache()
    return {"workload": w.name, "lines": [int(len(w.lines.nu)), int(len(w.gases[0].lines.nu))],
            "kappa_ms": ms, "line_evals": evals, "line_evals_per_s": rate,
            "frac_of_line_sum_ceiling": rate / line_peak_evals_per_s()}


def form_table16(rtlbl, I, reps=3):
    """The paper's own kappa formulation (16 tabulated points per line,
    multiply-adds only) on the 32^3 workload beside the plain line sum: the
    compute_kappa time of each, and how far the per-cell absorbed power of the
    same 2^20 rays moves when the march reads the 16-point kappa."""
    import numpy as np
    import torch
    w = I.plain_32cube()
    t = rtlbl.Tracer(0)
    t.setup_workload(w)
    kap = torch.empty((w.grid.n_cells, t.required_pitch()), dtype=torch.float32, device="cuda")
    out = {}
    tallies = {}
    for name, mode in (("plain", rtlbl.KAPPA_PLAIN), ("table16", rtlbl.KAPPA_TABLE16)):
        t.compute_kappa(mode, kap, None)                 # warm-up
        torch.cuda.synchronize()
        s0 = t.stats()
        for _ in range(reps):
            t.compute_kappa(mode, kap, None)
        s1 = t.stats()
        out[f"kappa_ms_{name}"] = (s1["kappa_ms"] - s0["kappa_ms"]) / reps
        t.reset_tally()
        t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, rtlbl.TALLY_F32)
        tallies[name] = t.tally()[0]
    a0, a1 = tallies["plain"], tallies["table16"]
    m = a0 > 0
    rel = np.abs(a1[m] - a0[m]) / a0[m]
    out.update({
        "workload": w.name,
        "speedup_over_plain_line_sum": out["kappa_ms_plain"] / out["kappa_ms_table16"],
        "absorbed_rel_diff_vs_plain": {"max": float(rel.max()), "median": float(np.median(rel))},
        "total_absorbed_rel_diff": float(abs(a1.sum() - a0.sum()) / a0.sum()),
    })
    t.close()
    del kap
    torch.cuda.empty_cache()
    return out


def form_adaptive(rtlbl, I, eps_list=(1e-3, 1e-4, 3e-5, 1e-5, 1e-6),
                  wing_eps_list=(1e-2, 3e-3, 1e-3, 1e-4), reps=3):
    """Adaptive line windows (the paper's announced next version: points per
    line set by the local temperature and the line's intensity) on the 32^3
    workload beside the plain line sum: for each tolerance eps, the
    compute_kappa time (band means, windows and windowed sum), the fraction
    of line evaluations kept, and how far the per-cell absorbed power of the
    same 2^20 rays moves from the plain sum's.  The same for the windows with
    their wing return (the dropped points' Lorentz mass spread over the
    band, an extension), at the tolerances listed for it."""
    import numpy as np
    import torch
    w = I.plain_32cube()
    t = rtlbl.Tracer(0)
    t.setup_workload(w)
    kap = torch.empty((w.grid.n_cells, t.required_pitch()), dtype=torch.float32, device="cuda")

    def timed(mode):
        t.compute_kappa(mode, kap, None)                 # warm-up
        torch.cuda.synchronize()
        t.reset_tally()
        for _ in range(reps):
            t.compute_kappa(mode, kap, None)
        s = t.stats()
        return s["kappa_ms"] / reps, s["line_evals"] / reps

    def absorbed():
        t.reset_tally()
        t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, rtlbl.TALLY_F32)
        return t.tally()[0]

    ms0, ev0 = timed(rtlbl.KAPPA_PLAIN)
    a0 = absorbed()
    m = a0 > 0
    def rows(mode, tolerances):
        out = []
        for eps in tolerances:
            t.set_line_tolerance(eps)
            ms, ev = timed(mode)
            a1 = absorbed()
            rel = np.abs(a1[m] - a0[m]) / a0[m]
            out.append({
                "eps": eps,
                "kappa_ms": ms,
                "evals_kept": ev / ev0,
                "speedup_over_plain_line_sum": ms0 / ms,
                "absorbed_rel_diff_vs_plain": {"max": float(rel.max()),
                                               "median": float(np.median(rel))},
                "total_absorbed_rel_diff": float(abs(a1.sum() - a0.sum()) / a0.sum()),
            })
        return out

    res = {"workload": w.name, "kappa_ms_plain": ms0, "line_evals_plain": ev0,
           "tolerances": rows(rtlbl.KAPPA_ADAPTIVE, eps_list),
           "wing_return": rows(rtlbl.KAPPA_ADAPTIVE_WINGS, wing_eps_list)}
    t.close()
    del kap
    torch.cuda.empty_cache()
    return res


def form_arith(rtlbl, I):
    """FP32 arithmetic of the device (the paper's Table 2 experiments), in
    brief: which basic operations are correctly rounded on random operands,
    the outcome of the near-tie vectors 1.5 - 2^-i, and the largest error in
    ulp of the hardware exp2, log2, rcp, rsq and sqrt instructions over 2^22
    normal operands each.  References are binary64 (for +, -, *, / the
    binary64 result rounded to binary32 is the correctly rounded one)."""
    import numpy as np
    import torch
    t = rtlbl.Tracer(0)
    rng = np.random.default_rng(5)
    n = 1 << 22

    def run(op, *xs):
        ts = [torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda() for x in xs]
        out = t.arith_eval(op, *ts)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def f64(x):
        return np.asarray(x, np.float32).astype(np.float64)

    def ulp(v):
        v = np.abs(v)
        return np.where(v < 2.0 ** -126, 2.0 ** -149, np.ldexp(1.0, np.frexp(v)[1] - 24))

    def wide(k):
        return (rng.choice([-1.0, 1.0], k) * np.ldexp(rng.uniform(1, 2, k), rng.integers(-60, 60, k))).astype(np.float32)

    x, y = wide(n), wide(n)
    exact = {"add": f64(x) + f64(y), "sub": f64(x) - f64(y), "mul": f64(x) * f64(y),
             "div": f64(x) / f64(y)}
    rounded = {op: bool(np.array_equal(run(op, x, y).view(np.uint32),
                                       v.astype(np.float32).view(np.uint32)))
               for op, v in exact.items()}
    i = np.arange(1, 41)
    ties = run("sub", np.full(40, 1.5, np.float32), np.ldexp(1.0, -i).astype(np.float32))
    pos = np.ldexp(rng.uniform(1, 2, n), rng.integers(-125, 125, n)).astype(np.float32)
    e2 = rng.uniform(-125.0, 127.9, n).astype(np.float32)
    refs = {"exp2": (e2, np.exp2(f64(e2))), "log2": (pos, np.log2(f64(pos))),
            "rcp": (pos, 1.0 / f64(pos)), "rsq": (pos, 1.0 / np.sqrt(f64(pos))),
            "sqrt": (pos, np.sqrt(f64(pos)))}
    max_ulp = {}
    for op, (a, r) in refs.items():
        max_ulp[op] = round(float(np.max(np.abs(f64(run(op, a)) - r) / ulp(r))), 4)
    t.close()
    return {
        "correctly_rounded": rounded,
        "one_point_five_minus_2^-i": {"i<=23": "exact" if all(
            ties[k - 1] == np.float32(1.5 - 2.0 ** -k) for k in range(1, 24)) else "inexact",
            "i=24": float(ties[23]), "i>=25": float(ties[24])},
        "max_ulp": max_ulp,
        "operands": n,
    }


def form_spectral_shard(rtlbl, I, n_shards=8, steps=3):
    """One GPU's share of the 32^3 workload split by wavenumber over n_shards
    GPUs (shard boundaries on march chunks; the shard keeps only the lines
    that reach its range): the largest shard with all 2^20 rays, timed as the
    headline step.  The split run would take about the slowest shard's time
    plus one all-reduce of 0.5 MB of tallies, which is not measured here."""
    import torch
    w = I.plain_32cube()
    bounds = I.spectral_shard_bounds(w.lines.n_nu, n_shards, rtlbl.lib.rt_march_chunk())
    lo, hi = max(bounds, key=lambda b: b[1] - b[0])
    s = I.spectral_shard(w, lo, hi)
    t = rtlbl.Tracer(0)
    t.setup_grid(s.grid)
    t.setup_lines(s.lines)
    kap = torch.empty((s.grid.n_cells, t.required_pitch()), dtype=torch.float32, device="cuda")

    def step():
        t.reset_tally()
        t.compute_kappa(rtlbl.KAPPA_PLAIN, kap, None)
        t.trace_rays(s.seed, s.n_rays, 0, s.n_rays, rtlbl.TALLY_F32)
        return t.tally()

    step()
    torch.cuda.synchronize()
    t.stats()
    kappa_ms = march_ms = updates = evals = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        st = t.stats()
        kappa_ms += st["kappa_ms"]
        march_ms += st["march_ms"]
        updates += st["updates"]
        evals += st["line_evals"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    t.close()
    del kap
    torch.cuda.empty_cache()
    return {"workload": s.name, "n_shards": n_shards, "shard_points": hi - lo,
            "shard_bounds": bounds, "lines": int(len(s.lines.nu)), "rays": s.n_rays,
            "ms_per_step": dt * 1e3, "updates_per_s": updates / steps / dt,
            "kappa_ms_per_step": kappa_ms / steps, "march_ms_per_step": march_ms / steps,
            "march_updates_per_s": updates / (march_ms * 1e-3),
            "line_evals_per_s": evals / (kappa_ms * 1e-3)}


def run_forms(rtlbl, I, args):
    out = {}
    ep = args.learned_epochs
    for name, fn in (("precision", form_precision), ("batched", form_batched),
                     ("learned", lambda r, i: form_learned(r, i, epochs=ep,
                                                           model_path=args.learned_model)),
                     ("learned_dense_lines",
                      lambda r, i: form_learned(r, i, epochs=ep, n_lines=20000)),
                     ("two_gases", form_two_gases), ("table16", form_table16),
                     ("spectral_shard", form_spectral_shard),
                     ("adaptive", form_adaptive), ("arith", form_arith)):
        if name not in args.forms.split(","):
            continue
        try:
            out[name] = fn(rtlbl, I)
        except Exception as exc:  # a failing form must not hide the headline
            out[name] = {"error": repr(exc)}
        print(f"# form {name} done", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--forms", default="precision,batched,learned,learned_dense_lines,two_gases,table16,"
                                       "spectral_shard,adaptive,arith",
                    help="comma-separated subset of the forms to run")
    ap.add_argument("--workload", default="plain_32cube")
    ap.add_argument("--no-headline", action="store_true",
                    help="run only the forms (for profiling one form); no headline record")
    ap.add_argument("--learned-epochs", type=int, default=LEARNED_EPOCHS,
                    help="training epochs of the learned forms")
    ap.add_argument("--learned-model", default=None,
                    help="the 8^3 learned form's network: loaded from this file if it "
                         "exists, else trained and saved there (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device once (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the spectral-range sharding is described in the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 1 << 30, "copy_probe_bytes_written": 1 << 30}))
        return

    from paper_cs_0703028_amd import inputs as I
    from paper_cs_0703028_amd import rtlbl

    if args.no_headline:
        rec = {"forms": run_forms(rtlbl, I, args)}
        print(json.dumps(rec), flush=True)
        return

    w = getattr(I, args.workload)()
    t = rtlbl.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(w.lines)
    kap = torch.empty((w.grid.n_cells, t.required_pitch()), dtype=torch.float32, device="cuda")

    def step():
        t.reset_tally()
        t.compute_kappa(rtlbl.KAPPA_PLAIN, kap, None)
        t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, rtlbl.TALLY_F32)
        return t.tally()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t.stats()
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
    print(f"# headline done: {dt / args.steps * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    t.close()
    del kap
    torch.cuda.empty_cache()
    peak = march_peak_updates_per_s()
    traffic = measured_traffic()
    march_rate = updates / (march_ms * 1e-3)
    line_rate = evals / (kappa_ms * 1e-3)
    rec = {
        "metric": METRIC,
        "value": updates / dt,
        "unit": "ray·cell·nu updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": w.grid.n_cells, "lines": int(len(w.lines.nu)),
                   "n_nu": w.lines.n_nu, "rays": w.n_rays, "kappa_mode": "plain",
                   "tally": "f32 partials, exact fixed-point accumulators"},
        "kappa_ms_per_step": kappa_ms / args.steps,
        "march_ms_per_step": march_ms / args.steps,
        "line_evals_per_s": line_rate,
        "line_sum_alu": {"achieved": line_rate * LINE_FLOPS_PER_EVAL / 1e12,
                         "peak": line_peak_evals_per_s() * LINE_FLOPS_PER_EVAL / 1e12,
                         "unit": "TFLOP/s", "frac": line_rate / line_peak_evals_per_s(),
                         "frac_of_published_fp32_peak":
                             line_rate * LINE_FLOPS_PER_EVAL / FP32_PUBLISHED_PEAK,
                         "frac_of_unpacked_fp32_fma_peak":
                             line_rate * LINE_FLOPS_PER_EVAL / FP32_UNPACKED_FMA_PEAK},
        "trace_updates_per_s": march_rate,
        "energy_balance_rel": float(abs(bal[0] + bal[1] - bal[2] - bal[3]) / (bal[0] + bal[1])),
        "roofline": {
            "bound": "alu",
            "kernel": "march_kernel",
            "achieved": march_rate * MARCH_FLOPS_PER_UPDATE / 1e12,
            "peak": peak * MARCH_FLOPS_PER_UPDATE / 1e12,
            "unit": "TFLOP/s",
            "frac": march_rate / peak,
            # the same achieved rate against MI355X's published FP32 vector
            # peak (packed FMAs), and against one FMA per lane and cycle
            "published_fp32_peak": FP32_PUBLISHED_PEAK / 1e12,
            "frac_of_published_fp32_peak":
                march_rate * MARCH_FLOPS_PER_UPDATE / FP32_PUBLISHED_PEAK,
            "frac_of_unpacked_fp32_fma_peak":
                march_rate * MARCH_FLOPS_PER_UPDATE / FP32_UNPACKED_FMA_PEAK,
            "peak_derivation": ("256 CUs x 64 lanes x 2.4 GHz = 39.32e12 lane-slots/s; an update "
                                "takes 6 full-rate slots and one base-2 exponential issued at "
                                "half rate (2 slots, profiles/alu_rates_probe.md): 8 slots, "
                                "9 flops"),
            "traffic": traffic,
            "traffic_unit": "bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
            # those bytes over the launch time: the rate past L2 (Infinity
            # Cache and HBM), against 8 TB/s of HBM
            "traffic_gbs": (traffic / (march_ms / launches * 1e-3) / 1e9
                            if traffic and launches else None),
            "launches": launches,
            "avg_launch_ms": march_ms / launches if launches else None,
        },
    }
    if not args.no_forms:
        rec["forms"] = run_forms(rtlbl, I, args)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
