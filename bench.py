#!/usr/bin/env python
"""Benchmark of the lattice Boltzmann hot path on one MI355X.

Workload of the value line (the precision configuration, the largest single
lattice): D3Q19 MRT, FP32 deviation storage, 256^3 periodic box, 64 fixed
spheres of radius 8 at seed-drawn positions (random sequential addition,
gaps >= 2), body force for Re = 10, quadratic interpolated bounce-back with
the momentum-exchange force and torque of every sphere at every step.  A step
is the whole per-step path: the fused stream-collide sweep that also applies
the bounce-back of the links and the per-sphere force reduction.  MLUPS counts
every lattice cell.  The same workload in FP64 and FP16 deviation storage is
summarised in the line as well.

The last stdout line is one compact JSON object (the contract).  Every other
measurement goes to stderr (one "# key: ..." line each) and, in full, to the
JSON file --extras-out: the 128^3 one-sphere workload (FP32 / FP64 / FP16,
quadratic IBB and the direct-forcing IBM), the other bounce-back schemes, the
IBM with the 3- and 2-point deltas, a general-rate MRT run, free spheres
settling under gravity, the HBM copy yardstick, 512 lattices with translating
spheres as one batch, the FP32/FP16 drag error against FP64 storage, the
request trace served at saturation and below it, and the FP64 CPU oracle on a
bounded sample of the value workload (one thread and all cores).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--extras all|none|k1,k2]
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
STORE_BYTES = {"F64": 8, "F32": 4, "F16": 2, "F16_SR": 2}
# the sweep tuner of a new lattice takes 8 + 4 x 12 steps; warm-up always runs past it
TUNER_STEPS = 64
# extra runs record HIP events around every PROFILE_EVERY-th sweep launch where the
# sweeps of a call are not back to back (events on every launch add work to each step)
PROFILE_EVERY = 8
ALL_EXTRAS = ("single", "schemes", "open", "copy", "batch", "precision", "serving", "cpu")


T_START = time.perf_counter()


def log(msg):
    """A progress line on stderr, with the seconds since the start of the run."""
    print(f"{msg}  [{time.perf_counter() - T_START:.0f} s]", file=sys.stderr, flush=True)


SWEEP_SOURCES = ("sweep_core.hpp", "kernels_sweep.hip", "lbm_ibb.hpp", "lbm_device.hpp", "lbm_args.hpp")


def sweep_source_hash():
    """Hash of the sources the sweep kernel is compiled from."""
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1906_05445_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(key, cells):
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs (scaled by the same counters on a copy kernel), if they were taken on the
    current sweep source; otherwise None."""
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


def run_case(case, steps, warmup, key, torch, lbm, rates=None):
    """Warm up past the sweep tuner, then time exactly `steps` steps in one lbm_step
    call: HIP events on the lattice's stream around the call (whole-step time), the
    host clock around it (synchronised on both sides), and the library's events
    around the sweep launches (sweep-kernel time)."""
    Q = 19 if case.lattice == "D3Q19" else 9
    gpu = lbm.Lattice(case.lattice, case.collision, case.storage, case.shape, case.tau, g=case.g, rates=rates,
                      g_fluid_only=case.g_fluid_only, max_solids=max(1, len(case.solids)),
                      boundary=case.boundary, inflow=case.inflow)
    gpu.set_solids(case.solids, case.method, n_iter=case.ibm_iters, retraction=case.retraction, delta=case.delta)
    # body-force workloads start from the uniform flow of their periodic-array estimate (as served
    # solves do), so that the timed steps run near the driven flow instead of in the start from rest
    from paper_1906_05445_amd.serving import initial_velocity

    u0 = (case.inflow, 0.0, 0.0) if case.inflow else initial_velocity(case)
    if u0 is not None:
        gpu.set_equilibrium(1.0, u0)
    N = gpu.N
    w = max(warmup, TUNER_STEPS)
    gpu.step(w)
    while gpu.autotune_info()["policy"] is None:  # a tuner that needs longer
        gpu.step(TUNER_STEPS)
        w += TUNER_STEPS
    torch.cuda.synchronize()
    gpu.profile(True, every=PROFILE_EVERY)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(gpu.stream)
    gpu.step(steps)
    e1.record(gpu.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_s = e0.elapsed_time(e1) / 1e3 / steps
    sweep_ms, launches = gpu.profile_read()
    gpu.profile(False)
    if not gpu.check():
        raise RuntimeError(f"{key}: populations diverged")
    F = gpu.force_torque()
    tune = gpu.autotune_info()
    _, u, types = gpu.macros()
    fluid = types != 1
    nfluid = int(fluid.sum())
    re_at_end = None
    if case.meta.get("Re") is not None and case.solids and not case.inflow:
        # superficial velocity (mean fluid velocity x fluid fraction) over the diameter and viscosity
        nu = (case.tau - 0.5) / 3.0
        gdir = int(np.argmax(np.abs(case.g)))
        re_at_end = float(u[gdir][fluid].sum()) / N * 2.0 * case.solids[0]["radius"] / nu
    per_cell = 2 * Q * STORE_BYTES[case.storage] + 1  # pull Q, push Q, one flag byte
    achieved = N * per_cell / step_s / 1e9
    sweep_s = sweep_ms / 1e3 / launches if launches > 0 else None
    traffic_bytes = traffic_for(key, N)
    out = {
        "mlups": N * steps / wall / 1e6,
        "mflups_fluid": nfluid * steps / wall / 1e6,
        "ms_per_step": wall / steps * 1e3,
        "event_ms_per_step": step_s * 1e3,
        "steps": steps,
        "warmup": w,
        "cells": N,
        "fluid_cells": nfluid,
        "re_target": case.meta.get("Re"),
        "re_at_end": re_at_end,
        "solids": len(case.solids),
        "method": case.method,
        "storage": case.storage,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic_bytes is None or sweep_s is None else traffic_bytes / sweep_s / 1e9,
                     "basis": f"{per_cell} B/cell x {N} cells per step over the whole-step time (HIP events "
                              f"around the {steps} timed steps)"},
        "sweep_kernel": None if sweep_s is None else {
            "avg_us": sweep_s * 1e6, "launches_timed": launches,
            "achieved_GBps": N * per_cell / sweep_s / 1e9, "frac": N * per_cell / sweep_s / 1e9 / HBM_PEAK_GBS},
        "drag_x_solid0": float(F[0, 0]) if len(F) else None,
        "autotune_policy": tune.get("policy"),
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


def run_open_sphere(torch, lbm, W, steps, chunk=1000, tol=None, **kw):
    """The sphere of Sec. 3.4 (uniform inflow, stress-free sides, convective outflow) from a uniform
    stream: whole-step throughput, and the drag coefficient at the end with its change over the last
    chunk, beside the standard correlation (a sanity reference).  tol: stop once C_D changes by less
    than tol (relative) over a chunk, else after `steps`."""
    case = W.open_sphere(**kw)
    gpu = lbm.Lattice(case.lattice, case.collision, case.storage, case.shape, case.tau, max_solids=1,
                      max_links=4_000_000, max_lagrangian=1024, boundary=case.boundary, inflow=case.inflow)
    gpu.set_solids(case.solids, case.method)
    gpu.set_equilibrium(1.0, (case.inflow, 0.0, 0.0))
    gpu.step(TUNER_STEPS)
    torch.cuda.synchronize()
    nu = (case.tau - 0.5) / 3.0
    Re = case.meta["Re"]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cd = []
    ms = 0.0
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        e0.record(gpu.stream)
        gpu.step(k)
        e1.record(gpu.stream)
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        done += k
        cd.append(W.drag_coefficient(float(gpu.force_torque()[0, 0]), Re, nu))
        if len(cd) % 5 == 0:
            log(f"#   {case.name}: {done} steps, C_D {cd[-1]:.5f}")
        if tol is not None and len(cd) > 1 and abs(cd[-1] - cd[-2]) <= tol * abs(cd[-1]):
            break
    ok = gpu.check()
    gpu.close()
    N = case.shape[0] * case.shape[1] * case.shape[2]
    ref = W.schiller_naumann(Re)
    return {"workload": case.name, "shape": list(case.shape), "D": case.meta["D"], "Re": Re, "U_in": case.inflow,
            "tau": case.tau, "method": case.method, "storage": case.storage, "steps": done,
            "mlups": N * done / (ms / 1e3) / 1e6, "finite": bool(ok),
            "C_D": cd[-1], "C_D_rel_change_last_chunk": abs(cd[-1] - cd[-2]) / abs(cd[-1]) if len(cd) > 1 else None,
            "C_D_history_per_chunk": [round(x, 5) for x in cd], "chunk": chunk,
            "C_D_schiller_naumann": ref, "rel_diff_to_correlation": cd[-1] / ref - 1.0}


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
    sweep_us = b.time_sweep(10)
    if not all(m.check() for m in members[:: max(1, count // 16)]):
        raise RuntimeError("batch: populations diverged")
    per_cell = 2 * 19 * STORE_BYTES["F32"] + 1
    out = {
        "lattices": count, "cells": N, "steps": steps, "mlups": N * steps / wall / 1e6,
        "ms_per_step": wall / steps * 1e3, "setup_s": setup_s, "pool_GB": pool / 1e9,
        "step_frac": N * per_cell / (wall / steps) / 1e9 / HBM_PEAK_GBS,
        "sweep_us_per_step": sweep_us,
        "sweep_frac": N * per_cell / (sweep_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "tune": tune,
        "note": "whole step: sweep, bounce-back + force, reclassification, refill and link rebuild of every lattice",
    }
    b.close()
    del b
    torch.cuda.empty_cache()
    return out


def run_serving(torch, lbm, W, rate, seconds, min_completed, step_cap, count=256, pool_gb=32.0, max_slots=16):
    """The request trace served until min_completed requests have finished or `seconds`
    have passed (see paper_1906_05445_amd/serving.py)."""
    from paper_1906_05445_amd import serving as S

    trace = W.request_trace(count=count, rate=50.0, seed=5)
    for e in trace:  # same requests, arrival times rescaled to the requested rate
        e["arrival"] *= 50.0 / rate
    reqs = S.requests_from_trace(trace)
    srv = S.Server(pool_bytes=int(pool_gb * 1e9), max_slots=max_slots, check_every=100, tol=1e-6,
                   step_cap=step_cap)
    st = srv.run(reqs, wall_limit=seconds, stop_after=min_completed, log=lambda m: log(f"#   {m}"))
    srv.close()
    torch.cuda.empty_cache()
    done = [r for r in reqs if r.finished is not None]
    st.update({"rate_req_per_s": rate, "window_limit_s": seconds, "stop_after": min_completed, "pool_GB": pool_gb,
               "max_slots": max_slots, "criterion": f"|F(t)-F(t-100)|/|F(t)| < 1e-6, cap {step_cap} steps",
               "start": "uniform flow at the periodic-array estimate of the mean velocity",
               "per_request": [{"edge": r.case.shape[0], "Re": round(r.case.meta["Re"], 2), "method": r.case.method,
                                "steps": r.steps, "converged": r.converged, "latency_s": round(r.latency, 3),
                                "last_change": float(r.change) if r.change >= 0 else None}
                               for r in done]})
    # how far the capped solves were from the criterion when they stopped
    ch = sorted(float(r.change) for r in done if not r.converged and r.change >= 0)
    st["capped_last_change_p50"] = ch[len(ch) // 2] if ch else None
    st["capped_last_change_max"] = ch[-1] if ch else None
    return st


def run_precision(torch, lbm, W, steps):
    """Per-sphere drag of the 256^3 64-sphere workload stored in FP32 and FP16, against FP64
    storage on the same GPU (the FP64 path matches the FP64 oracle to 1e-12)."""
    drag = {}
    for storage in ("F64", "F32", "F16", "F16_SR"):
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
    # tolerances of the 10k-step comparison: FP32 2e-4; FP16 to nearest 1e-1 (it lags: per-step increments
    # below half an FP16 unit are lost); FP16 with stochastic rounding 2e-3
    for storage, tol in (("F32", 2e-4), ("F16", 1e-1), ("F16_SR", 2e-3)):
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
        errs.append(float(np.abs(f32 - f64).max() / np.abs(f64).max()))
        ref.close()
    b.close()
    torch.cuda.empty_cache()
    return {"lattices": count, "steps": steps, "max_rel_force_err": max(errs), "per_lattice": errs,
            "tolerance": 5e-4, "within_tolerance": bool(max(errs) <= 5e-4),
            "measure": "max over the retained steps (the last 8192) and components of "
                       "|F_batch,FP32 - F_alone,FP64| / max |F_alone,FP64|"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, steps1, stepsN, threads):
    """The FP64 oracle (plain C, literal form, OpenMP over its per-cell loops) on a
    bounded sample of the value workload: steps1 steps on one thread, then stepsN
    steps on `threads` threads, from the same state."""
    from oracle import Oracle

    t0 = time.perf_counter()
    o = Oracle(case.lattice, case.collision, case.shape, case.tau, g=case.g, threads=threads)
    o.set_solids(case.solids, case.method)
    setup = time.perf_counter() - t0
    N = case.shape[0] * case.shape[1] * case.shape[2]
    o.set_threads(1)
    t0 = time.perf_counter()
    o.step(steps1)
    w1 = time.perf_counter() - t0
    o.set_threads(threads)
    t0 = time.perf_counter()
    o.step(stepsN)
    wN = time.perf_counter() - t0
    del o
    return {"value": N * stepsN / wN / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{stepsN} steps of the value workload (256^3, 64 spheres, quadratic IBB, FP64) on "
                      f"{threads} threads; {steps1} steps on one thread",
            "value_1thread": N * steps1 / w1 / 1e6, "cpu": cpu_model(), "nproc": os.cpu_count(),
            "seconds": w1 + wN, "setup_s": setup}


def compact(d, keys):
    return {k: (round(d[k], 4) if isinstance(d.get(k), float) else d.get(k)) for k in keys}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--extras", default="all", help="all, none, or a comma list of " + ",".join(ALL_EXTRAS))
    ap.add_argument("--extras-out", default=os.path.join("bench_out", "bench_extras.json"))
    ap.add_argument("--batch-steps", type=int, default=500, help="steps of the 512-lattice batch")
    ap.add_argument("--precision-steps", type=int, default=10000, help="steps of the FP32/FP16 vs FP64 comparison")
    ap.add_argument("--serve-seconds", type=float, default=200.0, help="limit of the saturated serving window")
    ap.add_argument("--serve-min", type=int, default=32, help="completions that end the saturated window")
    ap.add_argument("--serve-cap", type=int, default=60000,
                    help="step cap of a solve (a capped solve is reported as capped, with its drag at the cap)")
    ap.add_argument("--open-steps", type=int, default=20000, help="steps of the open-domain sphere (Sec. 3.4)")
    ap.add_argument("--cpu-steps", default="1,3", help="oracle sample: steps on one thread, steps on all threads")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU (a lattice is not split across GPUs), so "
                                   "--gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1906_05445_amd import lbm
    from paper_1906_05445_amd import workloads as W

    torch.cuda.set_device(0)
    K, Wm = args.steps, args.warmup
    want = set(ALL_EXTRAS) if args.extras == "all" else (set() if args.extras == "none" else
                                                          set(args.extras.split(",")))

    def wanted(group, key):  # a whole group, or one case by its key
        return group in want or key in want
    extras = {}

    def extra(key, value, summary):
        extras[key] = value
        log(f"# {key}: {summary}")

    # ---- the value workload, FP32, and its FP64 / FP16 forms
    prim = run_case(W.sphere_pack(storage="F32", drive="array"), K, Wm, "pack256_f32_quadratic", torch, lbm)
    log(f"# pack256 F32: {prim['mlups']:.0f} MLUPS, step {prim['event_ms_per_step'] * 1e3:.1f} us, "
        f"{prim['roofline']['achieved']:.0f} GB/s ({prim['roofline']['frac']:.3f}), policy {prim['autotune_policy']}")
    forms = {}
    for st in ("F64", "F16", "F16_SR"):
        r = run_case(W.sphere_pack(storage=st, drive="array"), K, Wm, f"pack256_{st.lower()}_quadratic", torch, lbm)
        forms[st] = r
        log(f"# pack256 {st}: {r['mlups']:.0f} MLUPS, {r['roofline']['achieved']:.0f} GB/s "
            f"({r['roofline']['frac']:.3f})")

    # ---- everything else: stderr + the extras file
    k2 = max(K, 100)
    for key, (ctor, kw) in [("sphere128_f32_quadratic", (W.sphere_box, {"storage": "F32"})),
                            ("sphere128_f64_quadratic", (W.sphere_box, {"storage": "F64"})),
                            ("sphere128_f16_quadratic", (W.sphere_box, {"storage": "F16"})),
                            ("sphere128_f32_ibm", (W.sphere_box, {"storage": "F32", "method": "IBM"})),
                            ("sphere128_f64_ibm", (W.sphere_box, {"storage": "F64", "method": "IBM"}))]:
        if wanted("single", key):
            r = run_case(ctor(drive="array", **kw), k2, Wm, key, torch, lbm)
            extra(key, r, f"{r['mlups']:.0f} MLUPS, step frac {r['roofline']['frac']:.3f}")
    if wanted("single", "sphere128_f32_mrt_general_rates"):
        # general relaxation rates (every MRT row its own rate): the sparse-M relaxation
        rates = [0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, 1.0 / 0.8, 1.4, 1.0 / 0.8, 1.4, 1.0 / 0.8,
                 1.0 / 0.8, 1.0 / 0.8, 1.98, 1.98, 1.98]
        r = run_case(W.sphere_box(storage="F32", method="QUADRATIC", drive="array"), k2, Wm, "sphere128_f32_mrt_rates", torch, lbm,
                     rates=rates)
        extra("sphere128_f32_mrt_general_rates", r, f"{r['mlups']:.0f} MLUPS, step frac {r['roofline']['frac']:.3f}")
    for key, (ctor, kw) in [("sphere128_f32_yu", (W.sphere_box, {"method": "YU", "drive": "array"})),
                            ("sphere128_f32_zhao_yong", (W.sphere_box, {"method": "ZHAO_YONG", "drive": "array"})),
                            ("pack256_f32_yu", (W.sphere_pack, {"method": "YU", "drive": "array"})),
                            ("pack256_f32_zhao_yong", (W.sphere_pack, {"method": "ZHAO_YONG", "drive": "array"})),
                            ("sphere128_f32_ibm_delta3", (W.sphere_box, {"method": "IBM", "delta": 3, "drive": "array",
                                                                          "retraction": 0.3})),
                            ("sphere128_f32_ibm_delta2", (W.sphere_box, {"method": "IBM", "delta": 2, "drive": "array",
                                                                          "retraction": 0.2})),
                            ("settle128_f32_free", (W.settling_sphere, {})),
                            ("settle128_f32_free_ibm", (W.settling_sphere, {"method": "IBM"}))]:
        if not wanted("schemes", key):
            continue
        r = run_case(ctor(storage="F32", **kw), k2, Wm, key, torch, lbm)
        extra(key, r, f"{r['mlups']:.0f} MLUPS, step frac {r['roofline']['frac']:.3f}")
    if "open" in want and args.open_steps > 0:
        # Sec. 3.4's sphere, D = 16 (Zhao-Yong's sufficient resolution is about 14 at Re_p = 20)
        op = run_open_sphere(torch, lbm, W, args.open_steps)
        ch = op["C_D_rel_change_last_chunk"]
        extra("open_sphere_re20_f32_zhao_yong", op,
              f"{op['mlups']:.0f} MLUPS, C_D {op['C_D']:.4f} (change "
              f"{'n/a' if ch is None else format(ch, '.1e')} over the last {op['chunk']} steps; "
              f"Schiller-Naumann {op['C_D_schiller_naumann']:.4f})")
        key = "open_sphere_f32_quadratic"
        if wanted("open", key):
            r = run_case(W.open_sphere(method="QUADRATIC"), k2, Wm, key, torch, lbm)
            extra(key, r, f"{r['mlups']:.0f} MLUPS, step frac {r['roofline']['frac']:.3f}")
    if "open_resolution" in want:
        # Sec. 3.4's resolution question for Zhao-Yong at Re_p = 20: D = 16, 32 and 48 (the paper's largest:
        # 1152 x 576 x 576, 3.8e8 cells) at the viscosity of the D = 16 case (the paper keeps nu fixed), each
        # run until C_D changes by less than 1e-5 over 1000 steps
        res = {}
        for D, cap in ((16, 30000), (32, 50000), (48, 60000)):
            r = run_open_sphere(torch, lbm, W, cap, tol=1e-5, D=float(D), nu=0.04)
            res[f"D{D}"] = r
            log(f"# open sphere D = {D}: C_D {r['C_D']:.5f} after {r['steps']} steps, {r['mlups']:.0f} MLUPS")
        hi = res["D48"]["C_D"]
        extra("open_sphere_resolution_re20_zhao_yong",
              {"runs": res, "rel_diff_to_D48": {k: v["C_D"] / hi - 1.0 for k, v in res.items()}},
              ", ".join(f"{k}: {v['C_D'] / hi - 1.0:+.4f}" for k, v in res.items()) + " relative to D48")
    copy_gbps = None
    if "copy" in want:
        c = copy_probe(torch, lbm)
        copy_gbps = c
        extra("hbm_copy_GBps", c, f"{c:.0f} GB/s")
    if "batch" in want and args.batch_steps > 0:
        bb = run_batch(torch, lbm, W, args.batch_steps, 40)  # tuning: 36 steps
        extra("batch512_moving_f32", bb, f"{bb['mlups']:.0f} MLUPS, step frac {bb['step_frac']:.3f}, "
                                         f"sweep frac {bb['sweep_frac']:.3f}")
    precision = None
    if "precision" in want and args.precision_steps > 0:
        pr = run_precision(torch, lbm, W, args.precision_steps)
        precision = pr
        extra("precision_pack256_vs_f64", pr, f"FP32 max drag err {pr['F32']['max_rel_drag_err']:.2e}, "
                                              f"FP16 {pr['F16']['max_rel_drag_err']:.2e} (nearest), "
                                              f"{pr['F16_SR']['max_rel_drag_err']:.2e} (stochastic rounding)")
        bp = run_batch_vs_plain(torch, lbm, W, args.precision_steps)
        extra("batch_f32_vs_plain_f64", bp, f"max rel force err {bp['max_rel_force_err']:.2e}")
    serving = None
    if "serving" in want and args.serve_seconds > 0:
        sat = run_serving(torch, lbm, W, 50.0, args.serve_seconds, args.serve_min, args.serve_cap)
        extra("serving_saturated", sat, f"{sat['completed']} done ({sat['converged']} converged) in "
                                        f"{sat['wall_s']:.1f} s, p50 {sat['latency_p50_s']} s, p99 {sat['latency_p99_s']} s")
        # below capacity: arrivals at half the measured saturated completion rate
        rate = max(0.5 * sat["solves_per_s"], 0.02)
        sub = run_serving(torch, lbm, W, rate, 60.0, None, args.serve_cap)
        extra("serving_subsaturated", sub, f"{sub['completed']} done at {rate:.3f} req/s, p50 "
                                           f"{sub['latency_p50_s']} s, p99 {sub['latency_p99_s']} s")
        serving = {"n": sat["latency_n"], "converged": sat["converged"], "capped": sat["capped"],
                   "step_cap": args.serve_cap, "capped_change_p50": sat["capped_last_change_p50"],
                   "p50_s": sat["latency_p50_s"], "p99_s": sat["latency_p99_s"],
                   "solves_per_s": round(sat["solves_per_s"], 4), "offered_req_per_s": 50.0,
                   "sub_rate_req_per_s": round(rate, 4), "sub_n": sub["latency_n"], "sub_p50_s": sub["latency_p50_s"],
                   "sub_p99_s": sub["latency_p99_s"]}
    cpu = None
    if "cpu" in want:
        s1, sN = (int(x) for x in args.cpu_steps.split(","))
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(W.sphere_pack(storage="F64", drive="array"), s1, sN, threads)
        extras["cpu_baseline"] = cpu
        log(f"# cpu_baseline: {cpu['value']:.2f} MLUPS on {threads} threads, {cpu['value_1thread']:.2f} on one")
    if args.extras_out:
        d = os.path.dirname(args.extras_out)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.extras_out, "w") as fh:
            json.dump({"primary": prim, "f64": forms["F64"], "f16": forms["F16"], "extras": extras}, fh, indent=1)

    rf = prim["roofline"]
    line = {
        "metric": METRIC,
        "value": prim["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": prim["warmup"],
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "pack256: D3Q19 MRT 256^3 periodic, 64 fixed spheres R=8 (seed 3, gaps>=2), Re=10 "
                               "body force, quadratic IBB + Eq.17 force/torque, FP32 deviation storage",
                   "cells": prim["cells"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(rf["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(rf["frac"], 4), "traffic": None if rf["traffic"] is None else round(rf["traffic"], 1),
                     "basis": "153 B/cell/step over HIP-event whole-step time",
                     "sweep_kernel_frac": None if prim["sweep_kernel"] is None else
                     round(prim["sweep_kernel"]["frac"], 4),
                     # the measured yardstick next to the published peak: the library's copy kernel
                     "copy_GBps": None if copy_gbps is None else round(copy_gbps, 1),
                     "frac_of_copy": None if copy_gbps is None else round(rf["achieved"] / copy_gbps, 4)},
        "f64": {"mlups": round(forms["F64"]["mlups"], 1), "frac": round(forms["F64"]["roofline"]["frac"], 4)},
        "f16": {"mlups": round(forms["F16"]["mlups"], 1), "frac": round(forms["F16"]["roofline"]["frac"], 4)},
        "f16_sr": {"mlups": round(forms["F16_SR"]["mlups"], 1), "frac": round(forms["F16_SR"]["roofline"]["frac"], 4),
                   "drag_err_10k": None if precision is None else round(precision["F16_SR"]["max_rel_drag_err"], 6),
                   "f16_nearest_drag_err_10k": None if precision is None else
                   round(precision["F16"]["max_rel_drag_err"], 5)},
        "serving": serving,
        "cpu_baseline": None if cpu is None else {
            "value": round(cpu["value"], 3), "unit": "MLUPS", "cores": cpu["cores"], "kind": "oracle",
            "sample": cpu["sample"], "value_1thread": round(cpu["value_1thread"], 3), "cpu": cpu["cpu"],
            "nproc": cpu["nproc"]},
        "extras_file": args.extras_out or None,
    }
    print(json.dumps(line, separators=(",", ":")))


if __name__ == "__main__":
    main()
