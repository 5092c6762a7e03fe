"""Throughput of the HOFKS hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--forms a,b]

Primary workload (``value``): the 2D-2V perturbed gas, 256^2 cells x 32^2
velocities, plain FP64, tau = 1e-3, periodic; a step is one HOFKS time step
(Euler sub-steps, relaxation + shift + moment sums, per-cell update).  The
timed region starts with the state resident in HBM.  ``value`` counts cell-
velocity updates per second.  The roofline object refers to the kinetic
kernel, whose algorithmic traffic is one read and one write of every piece
per step (16 B per cell-velocity in FP64, 8 B in FP32), timed with hipEvents
on the library's stream.  Extra forms (FP32 precision form, ...) are reported
under ``forms``.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "cell·velocity updates/s and % HBM peak, FP32/batched/MLP vs plain FP64"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kinetic_gas2d_fp64_traffic.txt")
# sources of the dominant kernel (k_kinetic2w and the helpers it includes)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1212_0204_amd", "csrc", f)
                  for f in ("kernels.hpp", "kinetic2w.hpp")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(ng, unr):
    """HBM bytes per launch of the kinetic kernel in configuration (ng, unr)
    from the committed rocprofv3 counter passes (FETCH_SIZE and WRITE_SIZE,
    scaled by the copy kernel), or None when the kernel source has changed
    since they were taken or the configuration was not profiled"""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals, rows = {}, {}
    for line in open(TRAFFIC_FILE):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "config":
            rows[(int(f[1]), int(f[2]))] = (float(f[3]), float(f[4]))
        else:
            vals[f[0]] = f[1]
    if vals.get("source_hash") != kernel_source_hash() or (ng, unr) not in rows:
        return None
    fk, wk = rows[(ng, unr)]
    return 1024.0 * (fk * float(vals["fetch_scale"]) + wk * float(vals["write_scale"]))


def run_solver(wl, steps, warmup, precision, scheme=0, dt=None, strang=False):
    import torch
    import workloads as W
    from paper_1212_0204_amd import Solver

    fields = W.initial_fields(wl)
    s = Solver(wl.d, wl.n, wl.dx, wl.nv, wl.dv, bc=wl.bc, precision=precision, scheme=scheme,
               tau=wl.tau, dt=dt, strang=strang)
    s.set_state_macro(*fields)
    tuned = s.autotune(steps=3)  # launch configuration picked by timing
    if warmup:
        s.set_state_macro(*fields)
        s.step(warmup)
        s.sync()
    # the Euler and update launch groups in a pass of their own: their events
    # on both streams lengthen the step by a few percent
    s.set_state_macro(*fields)
    s.kernel_timing(enable=True, groups=(0, 2))
    s.step(steps)
    gms, gcnt = s.kernel_timing(enable=False)
    # the timed pass records events around the kinetic launches only
    s.set_state_macro(*fields)
    s.kernel_timing(enable=True, groups=(1,))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms, cnt = s.kernel_timing(enable=False)
    s.sync()  # raises on a non-physical state or sub-step overflow
    substeps, _ = s.counters()
    cv = wl.cv * steps
    bpcv = 8 if precision else 16
    kin_ms = kms[1] / max(cnt[1], 1)
    achieved = bpcv * wl.cv / (kin_ms * 1e-3) / 1e9
    out = {
        "steps": steps,
        "cv_per_s": cv / (ms * 1e-3),
        "ms_per_step": ms / steps,
        "dt": s.dt,
        "kernel_ms_per_step": {"euler": gms[0] / max(gcnt[0], 1), "kinetic": kin_ms,
                               "cell_update": gms[2] / max(gcnt[2], 1)},
        "euler_substeps_last_step": substeps,
        "kinetic_GBps": achieved,
        "kinetic_hbm_frac": achieved / HBM_PEAK_GBPS,
        "step_hbm_frac": bpcv * cv / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        # the kinetic launch of the step against the HBM roofline: one read
        # and one write of every piece, over its average duration in the
        # step (hipEvents around each launch on its stream)
        "roofline": {"bound": "hbm", "kernel": "kinetic launch (relaxation, shift, moment sums)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "algorithmic_bytes_per_launch": bpcv * wl.cv},
        "tuned": {"wavefronts_per_block": tuned[0], "loads_ahead": tuned[1],
                  "euler_before_kinetic": bool(tuned[2])},
    }
    del s
    torch.cuda.empty_cache()
    return out


def run_batch(steps, warmup):
    """the batched form: 512 independent shock tubes (seed 4), FP32 pieces,
    an Euler launch and a kinetic launch side by side, then the update
    launch, per step, replayed from a captured graph"""
    import numpy as np
    import torch
    import workloads as W
    from paper_1212_0204_amd import Batch

    tubes = W.batched_tubes()
    fields = [np.concatenate(a) for a in zip(*[
        (r, uu[0], th) for r, uu, th in (W.sod_tube(t.nx, left=t.left, right=t.right)
                                          for t in tubes)])]
    b = Batch([(t.nx, t.dx, t.nv, t.dv, t.tau) for t in tubes])
    b.set_state_macro(*fields)
    tuned = b.autotune(steps=4)
    b.set_state_macro(*fields)
    b.step(warmup)
    b.sync()
    b.set_state_macro(*fields)
    b.kernel_timing(enable=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    b.kernel_timing(enable=False)
    b.sync()
    flags = b.tube_flags()
    flagged = int((flags != 0).sum())
    # throughput of the tubes whose results are valid: a tube that met a
    # non-physical state is no longer advanced and none of its steps count
    ok = flags == 0
    cv_ok = int((b.nx * b.nvs)[ok].sum()) * steps
    out = {"workload": "batch512_tubes_seed4_fp32", "tubes": len(tubes), "cv_per_step": b.ncv,
           "steps": steps, "cv_per_s": cv_ok / (ms * 1e-3), "ms_per_step": ms / steps,
           "hbm_frac": 8 * cv_ok / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
           # the whole step (Euler and kinetic launches side by side, then the
           # update) against the HBM roofline: the pieces' 8 B per
           # cell-velocity over the step time, valid tubes only
           "roofline": {"bound": "hbm", "kernel": "whole step (k_batch_euler beside k_batch_kinetic, "
                                                  "then k_batch_update)",
                        "achieved": 8 * cv_ok / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": 8 * cv_ok / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                        "algorithmic_bytes_per_step": 8 * int((b.nx * b.nvs)[ok].sum())},
           "tuned": {"cells_per_item": tuned[0], "euler_part": tuned[1]},
           "flagged_tubes": flagged,
           # cold-side velocity resolution of each tube: dv / sqrt(theta_min)
           "dv_over_cold_thermal_speed": dict(zip(
               ("min", "median", "max"),
               (float(x) for x in np.percentile(
                   [t.dv / math.sqrt(min(t.left[2] / t.left[0], t.right[2] / t.right[0]))
                    for t in tubes], [0, 50, 100]))))}
    del b
    torch.cuda.empty_cache()
    return out


def run_closure(warmup=2):
    """the learned-closure form on the 512^2 disk (FP32 pieces, tau = 1e-4,
    100 steps).  The network is first trained with the library's kernels on
    snapshots of nine 128^2 runs (same dx); then the plain FP32 run and the
    closure run (threshold 1e-3) are timed from the same initial state.
    Effective cv/s counts every cell and velocity of every step."""
    import torch
    import workloads as W
    from paper_1212_0204_amd import Solver
    from paper_1212_0204_amd.mlp import ClosureNet, collect_snapshots

    t0 = time.perf_counter()
    x, t = collect_snapshots(W.closure_runs(seed=21, count=9), steps_at=[1, 3, 6, 10, 16, 24])
    net = ClosureNet(seed=0)
    scale, losses, used = net.fit_closure(x, t, steps=4000, log_every=3999)
    nsamp = int(x.shape[0])
    del x, t
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    wl = W.DISK_2D
    fields = W.initial_fields(wl)
    zero = ClosureNet(sigma=0.0)  # N^ = 0: the closure form without the network

    def timed(closure, tau=wl.tau, netw=None, steps=wl.steps):
        netw = netw or net
        s = Solver(wl.d, wl.n, wl.dx, wl.nv, wl.dv, bc=wl.bc, precision=1, tau=tau)
        s.set_state_macro(*fields)
        if closure:  # tune the kernel that the closure steps launch
            s.closure_enable(netw, threshold=1e-3)
        tuned = s.autotune(steps=3)
        for phase in ("warmup", "groups", "timed"):
            s.set_state_macro(*fields)
            if closure:
                s.closure_enable(netw, threshold=1e-3)
            if phase == "warmup":
                s.step(warmup)
                s.sync()
                continue
            if phase == "groups":  # the other launch groups, in a pass of their own
                s.kernel_timing(enable=True, groups=(0, 2, 3))
                s.step(steps)
                gms, gcnt = s.kernel_timing(enable=False)
                continue
            s.kernel_timing(enable=True, groups=(1,))
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.step(steps)
            e1.record(s.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            kms, cnt = s.kernel_timing(enable=False)
        U = s.read_moments()
        cs, kin = s.closure_stats()
        del s
        torch.cuda.empty_cache()
        per = [k / max(c, 1) for k, c in zip(gms, gcnt)]
        per[1] = kms[1] / max(cnt[1], 1)
        return ms, U, kin / max(cs * wl.nc, 1), per, tuned

    ms_p, Up, _, per_p, tuned_p = timed(False)
    ms_c, Uc, frac, per_c, tuned_c = timed(True)
    cv = wl.cv * wl.steps
    l1 = lambda a, b: float(np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum())
    dt = wl.dx / wl.dv
    # a relaxation time where the pieces carry a fifth of U^{n+1} (lambda =
    # exp(-dt/tau) ~ 0.21), so that the network's estimate matters: the
    # trained network against N^ = 0 at the same tau.  40 steps (t = 0.31):
    # at this tau the plain scheme itself meets a non-physical state near
    # step 51, when the blast waves of the periodic images meet.
    tau_mid, steps_mid = 5e-3, 40
    ms_pm, Upm, _, _, _ = timed(False, tau_mid, steps=steps_mid)
    ms_cm, Ucm, frac_m, per_m, _ = timed(True, tau_mid, steps=steps_mid)
    ms_zm, Uzm, frac_z, _, _ = timed(True, tau_mid, zero, steps=steps_mid)
    cvm = wl.cv * steps_mid
    mid = {"tau": tau_mid, "lambda": math.exp(-dt / tau_mid), "steps": steps_mid,
           "l1_density_error_vs_plain_fp32": l1(Ucm, Upm),
           "l1_density_error_zero_network": l1(Uzm, Upm),
           "kinetic_cell_fraction": frac_m, "kinetic_cell_fraction_zero_network": frac_z,
           "cv_per_s": cvm / (ms_cm * 1e-3), "ms_per_step": ms_cm / steps_mid,
           "plain_fp32_ms_per_step": ms_pm / steps_mid, "speedup_vs_plain_fp32": ms_pm / ms_cm,
           "closure_network_ms_per_step": per_m[3]}
    return {"workload": wl.name, "steps": wl.steps, "tau": wl.tau, "threshold": 1e-3,
            "lambda": math.exp(-dt / wl.tau), "mid_tau": mid,
            "cv_per_s": cv / (ms_c * 1e-3), "ms_per_step": ms_c / wl.steps,
            "plain_fp32_cv_per_s": cv / (ms_p * 1e-3), "plain_fp32_ms_per_step": ms_p / wl.steps,
            "speedup_vs_plain_fp32_same_workload": ms_p / ms_c,
            "l1_density_error_vs_plain_fp32": float(np.abs(Uc[0] - Up[0]).sum() / np.abs(Up[0]).sum()),
            "kinetic_cell_fraction": frac,
            "kernel_ms_per_step": {"euler": per_c[0], "kinetic": per_c[1], "cell_update": per_c[2],
                                   "closure_network": per_c[3]},
            "plain_kernel_ms_per_step": {"euler": per_p[0], "kinetic": per_p[1], "cell_update": per_p[2]},
            "tuned": {"wavefronts_per_block": tuned_c[0], "loads_ahead": tuned_c[1]},
            "plain_tuned": {"wavefronts_per_block": tuned_p[0], "loads_ahead": tuned_p[1]},
            "training": {"seconds_incl_snapshots": train_s, "samples": nsamp, "used": used,
                         "adam_steps": 4000, "loss_first_last": [losses[0][1], losses[-1][1]],
                         "output_scales": [float(v) for v in scale]}}


def copy_probe(mb, reps=5):
    """a plain device-to-device copy of known size (torch's copy kernel): the
    reachable HBM bandwidth, and the reference for scaling the FETCH_SIZE /
    WRITE_SIZE counters of the profiled kernels"""
    import torch
    n = mb * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * n * 4
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_read": n * 4, "bytes_written": n * 4, "ms": ms,
            "GBps": moved / (ms * 1e-3) / 1e9}


def stream_probe(mb, reps=5):
    """the library's streaming probe (16-byte non-temporal accesses, no
    arithmetic): read, write and copy bandwidth of `mb` MiB"""
    import ctypes
    import torch
    from paper_1212_0204_amd import _lib
    L = _lib.lib()
    nbytes = mb * (1 << 20)
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {}
    for mode, name, moved in ((0, "read", nbytes), (1, "write", nbytes), (2, "copy", 2 * nbytes)):
        src = ctypes.c_void_p(a.data_ptr())
        dst = ctypes.c_void_p((sink if mode == 0 else b).data_ptr())
        assert L.hofks_stream_probe(mode, src, dst, nbytes, st) == 0
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            L.hofks_stream_probe(mode, src, dst, nbytes, st)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_GBps"] = moved / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    out["bytes"] = nbytes
    return out


def fp32_error_sample():
    """per-moment error of the FP32 precision form against the FP64 oracle on
    a reduced grid of the 3D workload (16^3 cells x 24^3 velocities, dv =
    1/2, the workload's field recipe), 3 steps, at the workload's tau and at
    lambda = 1/2 where the FP32 pieces carry half of U^{n+1}"""
    import workloads as W
    from oracle import Oracle
    from paper_1212_0204_amd import Solver
    wl = W.GAS_3D
    n, dx = (16, 16, 16), 1.0 / 16
    fields = W.perturbed_gas(16, 3, 0.1, 0.1, 4, (3, 33))
    out = {}
    for label, tau in (("workload_tau", wl.tau), ("lambda_half", (dx / wl.dv) / math.log(2.0))):
        o = Oracle(3, n, dx, wl.nv, wl.dv, bc=wl.bc, tau=tau)
        s = Solver(3, n, dx, wl.nv, wl.dv, bc=wl.bc, tau=tau, precision=1)
        o.init_macro(*fields)
        s.set_state_macro(*fields)
        o.step(3)
        s.step(3)
        U, Uo = s.read_moments(), o.U
        rho = Uo[0]
        u = Uo[1:4] / rho
        th = (2.0 * Uo[4] - rho * (u ** 2).sum(0)) / (3 * rho)
        c = np.sqrt(5.0 / 3.0 * th)
        sc = [np.abs(rho).max()] + [np.abs(rho).max() * c.max()] * 3 + [np.abs(Uo[4]).max()]
        out[label] = {"lambda": o.lam, "moment_errors": [float(np.abs(U[r] - Uo[r]).max() / sc[r])
                                                         for r in range(5)]}
        del s
    out["sample"] = "16^3 cells x 24^3 velocities, 3 steps, normwise per moment (rho, rho u, E)"
    return out


def batch_oracle_rate(count=32, steps=10):
    """the oracle on the first `count` tubes of the batched workload for
    `steps` steps (one tube after the other, OpenMP over cells)"""
    import workloads as W
    from oracle import Oracle, OracleError
    tubes = W.batched_tubes()[:count]
    t0 = time.perf_counter()
    cv = 0
    for t in tubes:
        o = Oracle(1, (t.nx,), t.dx, t.nv, t.dv, bc=(1,), tau=t.tau)
        r, uu, th = W.sod_tube(t.nx, left=t.left, right=t.right)
        o.init_macro(r, uu, th)
        try:
            o.step(steps)
        except OracleError:
            continue
        cv += t.nx * t.nv * steps
    el = time.perf_counter() - t0
    return {"value": cv / el, "sample": f"first {count} tubes of the 512-tube batch, {steps} steps "
                                        f"each ({el:.1f} s)"}


def cpu_baseline(wl, budget_s=12.0, single_s=6.0):
    """the oracle on the host cores, on the same workload: as many whole steps
    of the full grid as fit in ~budget_s (at least one) with all threads,
    then ~single_s with one thread."""
    import workloads as W
    from oracle import Oracle, max_threads, set_threads

    def timed(budget):
        o = Oracle(wl.d, wl.n, wl.dx, wl.nv, wl.dv, bc=wl.bc, tau=wl.tau)
        o.init_macro(*W.initial_fields(wl))
        t0 = time.perf_counter()
        n = 0
        while True:
            o.step(1)
            n += 1
            if time.perf_counter() - t0 > budget:
                break
        return n, time.perf_counter() - t0

    cores = max_threads()
    n, el = timed(budget_s)
    set_threads(1)
    n1, el1 = timed(single_s)
    set_threads(cores)
    return {"value": wl.cv * n / el, "unit": "cell-velocity updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{wl.name}: {n} full steps of the {wl.nc}-cell x {wl.nvel}-velocity grid "
                      f"from the initial state ({el:.1f} s, OpenMP over cells, plain FP64 C)",
            "single_thread": {"value": wl.cv * n1 / el1, "cores": 1,
                              "sample": f"{n1} full steps ({el1:.1f} s)"},
            "batched_tubes": batch_oracle_rate(),
            "fp32_form_vs_oracle": fp32_error_sample()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms",
                    default="sod_1d,fp32_3d,fp64_3d,batched,closure,weno_2d,offlattice_2d,strang_2d")
    ap.add_argument("--copy-probe-mb", type=int, default=1024,
                    help="size of a plain device copy timed after the run (0: skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: --gpus must be 1"}))
        sys.exit(2)

    import torch
    import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    wl = W.GAS_2D
    prim = run_solver(wl, args.steps, args.warmup, precision=0)
    forms = {}
    for name in [f for f in args.forms.split(",") if f]:
        if name == "fp32_3d":
            forms[name] = dict(workload=W.GAS_3D.name, **run_solver(W.GAS_3D, W.GAS_3D.steps, 2, 1))
        elif name == "fp64_3d":
            forms[name] = dict(workload=W.GAS_3D.name.replace("fp32", "fp64"),
                               **run_solver(W.GAS_3D, W.GAS_3D.steps, 2, 0))
        elif name == "batched":
            forms[name] = run_batch(500, 16)
        elif name == "closure":
            forms[name] = run_closure()
        elif name == "sod_1d":
            forms[name] = dict(workload=W.SOD_1D.name, **run_solver(W.SOD_1D, W.SOD_1D.steps, 5, 0))
        elif name == "weno_2d":
            forms[name] = dict(workload=wl.name + "_weno", scheme=3, **run_solver(wl, 50, 3, 0, 3))
        elif name == "offlattice_2d":
            # the paper's regime: max |v_k| dt / dx = 1 (no Euler sub-cycling)
            dt = wl.dx / ((wl.nv // 2) * wl.dv)
            forms[name] = dict(workload=wl.name + "_offlattice_cfl1", kinetic_cfl=1.0,
                               **run_solver(wl, 200, 5, 0, dt=dt))
        elif name == "strang_2d":
            forms[name] = dict(workload=wl.name + "_strang", **run_solver(wl, 200, 5, 0, strang=True))
    if "fp32_3d" in forms and "fp64_3d" in forms:
        forms["fp32_3d"]["speedup_vs_fp64_same_workload"] = (
            forms["fp32_3d"]["cv_per_s"] / forms["fp64_3d"]["cv_per_s"])
    for f in forms.values():
        f["speedup_vs_plain_fp64_2d"] = f["cv_per_s"] / prim["cv_per_s"]

    line = {
        "metric": METRIC,
        "value": prim["cv_per_s"],
        "unit": "cell-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": list(wl.n), "velocities_per_axis": wl.nv,
                   "dv": wl.dv, "tau": wl.tau, "bc": "periodic", "hbm_step_frac": prim["step_hbm_frac"]},
        "roofline": {"bound": "hbm", "achieved": prim["kinetic_GBps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": prim["kinetic_hbm_frac"],
                     "traffic": profiled_traffic(prim["tuned"]["wavefronts_per_block"],
                                                 prim["tuned"]["loads_ahead"]),
                     "traffic_unit": "bytes per launch",
                     "kernel": "k_kinetic2w (2D FP64, two cells per lane)",
                     "algorithmic_bytes_per_launch": 16 * wl.cv},
        "kernel_ms_per_step": prim["kernel_ms_per_step"],
        "forms": forms,
    }
    if args.copy_probe_mb:
        line["copy_probe"] = copy_probe(args.copy_probe_mb)
        line["stream_probe"] = stream_probe(args.copy_probe_mb)
        line["roofline"]["frac_of_measured_copy"] = (
            prim["kinetic_GBps"] / line["stream_probe"]["copy_GBps"])
        for f in forms.values():
            if "roofline" in f:
                f["roofline"]["frac_of_measured_copy"] = (
                    f["roofline"]["achieved"] / line["stream_probe"]["copy_GBps"])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
