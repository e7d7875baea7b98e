#!/usr/bin/env python
"""Benchmark of the lattice Boltzmann hot path on one MI355X.

Workload (the value line): D3Q19 MRT, FP32 deviation storage, 128^3 periodic
box, one fixed sphere of radius 16.2 at a seed-drawn sub-grid offset, body
force for Re = 20, quadratic interpolated bounce-back with momentum-exchange
force and torque every step.  A step is the whole per-step path: the fused
stream-collide sweep, the bounce-back/force kernel and the per-solid force
reduction.  MLUPS counts every lattice cell.

Also reported (same JSON line): the FP64 and FP16 forms of that workload,
the direct-forcing IBM form (5 forcing iterations per step), the 256^3 box
with 64 spheres (working set far beyond the 256 MB Infinity Cache), the
other bounce-back schemes (Yu's, Zhao & Yong's single-node one) on both
boxes, the IBM with the 3- and 2-point delta functions, a free sphere
settling under gravity (its link set rebuilt every step), the achievable HBM
copy bandwidth, 512 lattices with translating spheres stepped as one batch,
the request trace served for a bounded window at the trace's own rate
(saturated) and at a rate below capacity, and the FP64 CPU oracle timed on a
bounded sample of the value workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline (D3Q19 FP32 vs FP64); served solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0
STORE_BYTES = {"F64": 8, "F32": 4, "F16": 2}
# the timed run records HIP events around every PROFILE_EVERY-th sweep launch
# (events on every launch add host and dispatch work to each step)
PROFILE_EVERY = 8


def sweep_source_hash():
    src = os.path.join(ROOT, "paper_1906_05445_amd", "csrc", "kernels_sweep.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def traffic_for(key, cells):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (calibrated on a copy kernel), if they were taken on the
    current sweep source; otherwise None.  The roofline's "traffic" is these
    bytes over the same average launch duration as "achieved"."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    if data.get("sweep_source_sha256_16") != sweep_source_hash():
        return None
    ent = data.get("workloads", {}).get(key)
    if not ent or ent.get("cells") != cells:
        return None
    return ent["bytes_per_launch"]


def run_case(case, steps, warmup, key, torch, lbm):
    Q = 19 if case.lattice == "D3Q19" else 9
    gpu = lbm.Lattice(case.lattice, case.collision, case.storage, case.shape, case.tau, g=case.g,
                      g_fluid_only=case.g_fluid_only, max_solids=max(1, len(case.solids)))
    gpu.set_solids(case.solids, case.method, n_iter=case.ibm_iters, retraction=case.retraction, delta=case.delta)
    N = gpu.N
    gpu.step(warmup)
    torch.cuda.synchronize()
    gpu.profile(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpu.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms, launches = gpu.profile_read()
    gpu.profile(False)
    if not gpu.check():
        raise RuntimeError(f"{key}: populations diverged")
    F = gpu.force_torque()
    tune = gpu.autotune_info()
    wall = t1 - t0
    # readouts after the timed run: fluid cells, and the Reynolds number at its end
    # (superficial velocity = mean fluid velocity times the fluid fraction, over the
    # sphere diameter and the viscosity) against the one its body force was set for
    _, u, types = gpu.macros()
    fluid = types != 1
    nfluid = int(fluid.sum())
    re_at_end = None
    if case.meta.get("Re") is not None and case.solids:
        nu = (case.tau - 0.5) / 3.0
        gdir = int(np.argmax(np.abs(case.g)))
        u_sup = float(u[gdir][fluid].sum()) / N
        re_at_end = u_sup * 2.0 * case.solids[0]["radius"] / nu
    per_cell = 2 * Q * STORE_BYTES[case.storage] + 1  # pull Q, push Q, one flag byte
    timing = f"HIP events around the sweep launches of the timed run (one span per call, or every {PROFILE_EVERY}th)"
    if launches > 0:
        avg_s = sweep_ms / 1e3 / launches
    else:  # a run shorter than the tuner times no sweep: the step average stands in
        avg_s = wall / steps
        timing = "no sweep timed (run shorter than the sweep tuner): whole-step average"
    achieved = N * per_cell / avg_s / 1e9
    traffic_bytes = traffic_for(key, N)
    traffic = None if traffic_bytes is None else traffic_bytes / avg_s / 1e9
    out = {
        "mlups": N * steps / wall / 1e6,
        "mflups_fluid": nfluid * steps / wall / 1e6,
        "ms_per_step": wall / steps * 1e3,
        "cells": N,
        "fluid_cells": nfluid,
        "re_target": case.meta.get("Re"),
        "re_at_end": re_at_end,
        "solids": len(case.solids),
        "method": case.method,
        "storage": case.storage,
        "sweep_avg_us": avg_s * 1e6,
        "sweep_launches_timed": launches,
        "sweep_timing": timing,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": N * per_cell, "traffic_bytes_per_launch": traffic_bytes},
        "drag_x": float(F[0, 0]),
        "autotune": tune,
    }
    if case.meta.get("U_set") is not None:  # free solid: its vertical velocity at the end vs the Stokes target
        out["settling_velocity_at_end"] = float(gpu.solid_state()[0, 2 + 3])
        out["settling_velocity_stokes"] = -case.meta["U_set"]
    gpu.close()
    del gpu
    torch.cuda.empty_cache()
    return out


def copy_probe(torch, lbm, nbytes=4 << 30, reps=20, warm=3):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    for _ in range(warm if reps > 1 else 0):
        lbm.lbm_copy_probe(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        lbm.lbm_copy_probe(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms / 1e3) / 1e9


def run_batch(torch, lbm, W, steps, warmup, count=512):
    """512 independent lattices with translating spheres, advanced as one batch."""
    cases = W.moving_sphere_batch(count)
    fps = [lbm.Batch.footprint(c.lattice, c.collision, c.storage, c.shape, c.tau, max_solids=1) for c in cases]
    pool = lbm.lbm_batch_table_bytes(count) + sum((f + 255) // 256 * 256 for f in fps) + (1 << 20)
    t_setup = time.perf_counter()
    b = lbm.Batch("D3Q19", "F32", max_slots=count, pool_bytes=pool)
    members = []
    for c in cases:
        m = b.admit(c.collision, c.storage, c.shape, c.tau, g=c.g, max_solids=1)
        if m is None:
            raise RuntimeError("batch pool too small")
        m.set_solids(c.solids, c.method)
        members.append(m)
    setup_s = time.perf_counter() - t_setup
    N = sum(m.N for m in members)
    b.step(warmup)  # the first steps also tune the sweep's launch shape
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    wall = time.perf_counter() - t0
    tune = b.tune_info()
    tune["candidates"] = b.tune_table()
    sweep_us = b.time_sweep(10)
    ok = all(m.check() for m in members[:: max(1, count // 16)])
    if not ok:
        raise RuntimeError("batch: populations diverged")
    per_cell = 2 * 19 * STORE_BYTES["F32"] + 1
    achieved = N * per_cell / (sweep_us * 1e-6) / 1e9
    out = {
        "lattices": count,
        "cells": N,
        "steps": steps,
        "mlups": N * steps / wall / 1e6,
        "ms_per_step": wall / steps * 1e3,
        "setup_s": setup_s,
        "pool_GB": pool / 1e9,
        "sweep_us_per_step": sweep_us,
        "roofline_sweep": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_step": N * per_cell},
        "tune": tune,
        "note": "whole step: sweep, bounce-back + force, reclassification, refill and link rebuild of every lattice",
    }
    b.close()
    del b
    torch.cuda.empty_cache()
    return out


def run_serving(torch, lbm, W, seconds, rate, count, pool_gb, max_slots):
    """The request trace served for a bounded wall time (see paper_1906_05445_amd/serving.py)."""
    from paper_1906_05445_amd import serving as S

    trace = W.request_trace(count=count, rate=50.0, seed=5)
    for e in trace:  # same requests, arrival times rescaled to the requested rate
        e["arrival"] *= 50.0 / rate
    reqs = S.requests_from_trace(trace)
    srv = S.Server(pool_bytes=int(pool_gb * 1e9), max_slots=max_slots, check_every=100, tol=1e-6, step_cap=200000)
    st = srv.run(reqs, wall_limit=seconds)
    srv.close()
    torch.cuda.empty_cache()
    st.update({"rate_req_per_s": rate, "window_s": seconds, "pool_GB": pool_gb, "max_slots": max_slots,
               "criterion": "|F(t)-F(t-100)|/|F(t)| < 1e-6, cap 2e5 steps"})
    return st


def run_precision(torch, lbm, W, steps):
    """Per-sphere drag of the 256^3 64-sphere workload stored in FP32 and FP16, against FP64 storage on the same
    GPU (the FP64 path matches the FP64 oracle to 1e-12)."""
    drag = {}
    for storage in ("F64", "F32", "F16"):
        case = W.sphere_pack(storage=storage)
        gpu = lbm.Lattice(case.lattice, case.collision, storage, case.shape, case.tau, g=case.g,
                          max_solids=len(case.solids))
        gpu.set_solids(case.solids, case.method)
        gpu.step(steps)
        drag[storage] = gpu.force_torque()[:, 0].copy()
        gpu.close()
        del gpu
        torch.cuda.empty_cache()
    ref = drag["F64"]
    out = {"steps": steps, "spheres": int(ref.size), "mean_drag_f64": float(ref.mean())}
    for storage, tol in (("F32", 2e-4), ("F16", 1e-1)):
        rel = abs(drag[storage] - ref) / abs(ref)
        out[storage] = {"max_rel_drag_err": float(rel.max()), "mean_rel_drag_err": float(rel.mean()),
                        "rel_err_of_mean_drag": float(abs(drag[storage].mean() - ref.mean()) / abs(ref.mean())),
                        "tolerance": tol, "within_tolerance": bool(rel.max() <= tol)}
    return out


def run_batch_vs_plain(torch, lbm, W, steps, count=8):
    """Drag of lattices stepped as an FP32 batch against the same lattices stepped alone in FP64."""
    cases = W.moving_sphere_batch(count, seed=11, edge=(32, 64))
    fps = [lbm.Batch.footprint(c.lattice, c.collision, "F32", c.shape, c.tau, max_solids=1) for c in cases]
    b = lbm.Batch("D3Q19", "F32", max_slots=count, pool_bytes=lbm.lbm_batch_table_bytes(count) + sum(fps) + (1 << 24))
    members = []
    for c in cases:
        m = b.admit(c.collision, "F32", c.shape, c.tau, g=c.g, max_solids=1)
        m.set_solids(c.solids, c.method)
        members.append(m)
    b.step(steps)
    errs = []
    for c, m in zip(cases, members):
        ref = lbm.Lattice(c.lattice, c.collision, "F64", c.shape, c.tau, g=c.g, max_solids=1)
        ref.set_solids(c.solids, c.method)
        ref.step(steps)
        f64 = ref.history()[:, 0, :3]
        f32 = m.history()[:, 0, :3]
        scale = np.abs(f64).max()
        errs.append(float(np.abs(f32 - f64).max() / scale))
        ref.close()
    b.close()
    torch.cuda.empty_cache()
    return {"lattices": count, "steps": steps, "max_rel_force_err": max(errs), "per_lattice": errs,
            "tolerance": 5e-4, "within_tolerance": bool(max(errs) <= 5e-4),
            "measure": "max over the retained steps (the last 8192) and components of "
                       "|F_batch,FP32 - F_alone,FP64| / max |F_alone,FP64|"}


def cpu_baseline(case, steps):
    """The FP64 oracle (single-threaded C) on a bounded sample of the value workload."""
    from oracle import Oracle

    o = Oracle(case.lattice, case.collision, case.shape, case.tau, g=case.g)
    o.set_solids(case.solids, case.method)
    t0 = time.perf_counter()
    o.step(steps)
    wall = time.perf_counter() - t0
    N = case.shape[0] * case.shape[1] * case.shape[2]
    return {"value": N * steps / wall / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the 128^3 one-sphere workload (quadratic IBB), FP64, one host thread",
            "seconds": wall}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--primary-only", action="store_true", help="measure only the value workload")
    ap.add_argument("--cases", default="all",
                    help="comma list of extras: single (the other single-lattice cases), schemes (Yu and "
                         "Zhao-Yong bounce-back; or one of its keys), copy, batch, precision, serving")
    ap.add_argument("--batch-steps", type=int, default=2000, help="steps of the 512-lattice batch (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="wall time of each serving window (0: skip)")
    ap.add_argument("--precision-steps", type=int, default=10000,
                    help="steps of the FP32/FP16 vs FP64 drag comparison (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run the copy kernel once over this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU (a lattice is not split across GPUs here); --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1906_05445_amd import lbm
    from paper_1906_05445_amd import workloads as W

    torch.cuda.set_device(0)
    K, Wm = args.steps, args.warmup
    primary_case = W.sphere_box(storage="F32", method="QUADRATIC")
    primary = run_case(primary_case, K, Wm, "sphere128_f32_quadratic", torch, lbm)
    print(f"# sphere128 F32 IBB: {primary['mlups']:.0f} MLUPS, sweep {primary['sweep_avg_us']:.1f} us, "
          f"{primary['roofline']['achieved']:.0f} GB/s, policy {primary['autotune'].get('policy')}",
          file=sys.stderr, flush=True)
    extras = {}
    want = set()
    if not args.primary_only:
        want = ({"single", "schemes", "copy", "batch", "precision", "serving"} if args.cases == "all"
                else set(args.cases.split(",")))
    if "single" in want:
        k2 = max(K // 2, 100)
        for key, case in [("sphere128_f64_quadratic", W.sphere_box(storage="F64", method="QUADRATIC")),
                          ("sphere128_f16_quadratic", W.sphere_box(storage="F16", method="QUADRATIC")),
                          ("sphere128_f32_ibm", W.sphere_box(storage="F32", method="IBM")),
                          ("pack256_f32_quadratic", W.sphere_pack(storage="F32")),
                          ("pack256_f64_quadratic", W.sphere_pack(storage="F64")),
                          ("pack256_f16_quadratic", W.sphere_pack(storage="F16"))]:
            k = k2 if "256" not in key else max(K // 8, 50)
            extras[key] = run_case(case, k, max(Wm // 4, 64), key, torch, lbm)
            extras[key]["steps"] = k
            print(f"# {key}: {extras[key]['mlups']:.0f} MLUPS, {extras[key]['roofline']['achieved']:.0f} GB/s, "
                  f"policy {extras[key]['autotune'].get('policy')}",
                  file=sys.stderr, flush=True)
    # the other two bounce-back schemes the paper compares: Yu's (five populations per link)
    # and Zhao & Yong's single-node scheme; the 256^3 pack has gaps of 2 lattice units
    # where the multi-node schemes fall back; the IBM with the 3- and 2-point deltas of
    # the same comparison, each at the retraction the paper finds best for it
    for key, (ctor, kw) in [("sphere128_f32_yu", (W.sphere_box, {"method": "YU"})),
                            ("sphere128_f32_zhao_yong", (W.sphere_box, {"method": "ZHAO_YONG"})),
                            ("pack256_f32_yu", (W.sphere_pack, {"method": "YU"})),
                            ("pack256_f32_zhao_yong", (W.sphere_pack, {"method": "ZHAO_YONG"})),
                            ("sphere128_f32_ibm_delta3", (W.sphere_box, {"method": "IBM", "delta": 3,
                                                                          "retraction": 0.3})),
                            ("sphere128_f32_ibm_delta2", (W.sphere_box, {"method": "IBM", "delta": 2,
                                                                          "retraction": 0.2})),
                            ("settle128_f32_free", (W.settling_sphere, {})),
                            ("settle128_f32_free_ibm", (W.settling_sphere, {"method": "IBM"}))]:
        if "schemes" in want or key in want:
            case = ctor(storage="F32", **kw)
            k = max(K // 2, 100) if "256" not in key else max(K // 8, 50)
            extras[key] = run_case(case, k, max(Wm // 4, 64), key, torch, lbm)
            extras[key]["steps"] = k
            print(f"# {key}: {extras[key]['mlups']:.0f} MLUPS, {extras[key]['roofline']['achieved']:.0f} GB/s",
                  file=sys.stderr, flush=True)
    if "copy" in want:
        extras["hbm_copy_GBps"] = copy_probe(torch, lbm)
    if args.batch_steps > 0 and "batch" in want:
        extras["batch512_moving_f32"] = run_batch(torch, lbm, W, args.batch_steps, 40)  # tuning: 36 steps
        bb = extras["batch512_moving_f32"]
        print(f"# batch512: {bb['mlups']:.0f} MLUPS, sweep {bb['roofline_sweep']['achieved']:.0f} GB/s",
              file=sys.stderr, flush=True)
    if args.precision_steps > 0 and "precision" in want:
        extras["precision_pack256_vs_f64"] = run_precision(torch, lbm, W, args.precision_steps)
        extras["batch_f32_vs_plain_f64"] = run_batch_vs_plain(torch, lbm, W, args.precision_steps)
        pr = extras["precision_pack256_vs_f64"]
        print(f"# precision: FP32 max drag err {pr['F32']['max_rel_drag_err']:.2e}, FP16 "
              f"{pr['F16']['max_rel_drag_err']:.2e}; batch FP32 vs FP64 "
              f"{extras['batch_f32_vs_plain_f64']['max_rel_force_err']:.2e}", file=sys.stderr, flush=True)
    if args.serve_seconds > 0 and "serving" in want:
        extras["serving_saturated"] = run_serving(torch, lbm, W, args.serve_seconds, 50.0, 256, 32.0, 16)
        extras["serving_subsaturated"] = run_serving(torch, lbm, W, args.serve_seconds, 0.1, 256, 32.0, 16)
        for k in ("serving_saturated", "serving_subsaturated"):
            sv = extras[k]
            print(f"# {k}: {sv['completed']} solves in {sv['wall_s']:.1f} s, p50 {sv['latency_p50_s']} s, "
                  f"p99 {sv['latency_p99_s']} s", file=sys.stderr, flush=True)
    if args.copy_calibration > 0:
        copy_probe(torch, lbm, nbytes=args.copy_calibration << 20, reps=1)
    cpu = cpu_baseline(W.sphere_box(storage="F64", method="QUADRATIC"), args.cpu_steps) if args.cpu_steps > 0 else None
    line = {
        "metric": METRIC,
        "value": primary["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": primary["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sphere128: D3Q19 MRT, 128^3 periodic, one sphere R=16.2 (seed 2), Re=20 "
                               "body force, quadratic IBB + momentum-exchange force, FP32 deviation storage",
                   "cells": primary["cells"], "parallelism": "single GPU"},
        "roofline": primary["roofline"],
        "mflups_fluid": primary["mflups_fluid"],
        "sweep_vs_copy": (None if "hbm_copy_GBps" not in extras else
                          {"copy_GBps": extras["hbm_copy_GBps"],
                           "frac": primary["roofline"]["achieved"] / extras["hbm_copy_GBps"],
                           "note": "sweep algorithmic GB/s over the copy kernel's measured GB/s"}),
        "cpu_baseline": cpu,
        "flow": {"re_target": primary["re_target"], "re_at_end": primary["re_at_end"],
                 "note": "the body force is a Stokes estimate for re_target; from rest, the mean flow of "
                         "the periodic box relaxes over about L^2/(3 nu) (5e4 steps at 128^3, tau 0.8), "
                         "so a run of a few thousand steps ends in its start-up transient"},
        "sweep_avg_us": primary["sweep_avg_us"],
        "sweep_timing": primary["sweep_timing"],
        "autotune": primary["autotune"],
        "extras": extras,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
