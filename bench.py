#!/usr/bin/env python
"""Throughput of the thermocapillary projection step on one MI355X.

A step is one pass of the whole path (WENO5-RK3 transport of alpha and T,
geometry and CSF force, momentum predictor, MG-PCG pressure solve with FP64
refinement, projection, FP64 diagnostics) over the 256^3 melt-pool workload
(cell 2.5 um, density ratio 7500, moving 200 W Gaussian heat flux), all
inputs resident in HBM.  The primary line is the FP32-stencil path with FP64
iterative refinement at a divergence residual <= 1e-8; the plain FP64 path at
the same accuracy is reported beside it.

Prints ONE JSON line.  Options: --steps K --warmup W --gpus 1 --workload i
--kernel FAMILY (kernel family for the roofline entry) --no-cpu --no-fp64
--no-adjoint --no-species --no-rk3p --no-nphase.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def algorithmic_bytes(family: str, c: dict, precision: int) -> float:
    """Bytes one launch of a kernel family must move (each value once)."""
    N = c["nx"] * c["ny"] * c["nz"]
    w = 4 if precision == 1 else 8
    nfaces_per_cell = 3 if c["dim"] == 3 else 2
    if family == "smooth":
        # finest-level Jacobi sweep: x, b, alpha (face weights recomputed) read, x' written
        return N * w * (3 + 1)
    if family == "spmv":
        # finest-level SpMV fused with d <- z + beta d: z, d, alpha read; d' written
        # (K d' is not stored)
        return N * w * (3 + 1)
    if family == "update":
        # x += alpha d, r -= alpha K d (K d recomputed), first Jacobi sweep:
        # x, r, d, alpha read; x, r, z1 written
        return N * w * (4 + 3)
    if family == "transport":
        # averaged over the three stages: alpha, T, one velocity per axis,
        # base alpha/T (stages 2, 3), outputs alpha, T
        return N * w * (2 + nfaces_per_cell + 2 * 2 / 3 + 2)
    if family == "species":
        # one species stage, averaged over the three: c, one velocity per
        # axis, base c (stages 2, 3), output c
        return N * w * (1 + nfaces_per_cell + 2 / 3 + 1)
    if family == "predictor":
        # per component launch: alpha, sigma*kappa, M_d, u, v, w, u*_d (write)
        return N * w * (3 + nfaces_per_cell + 1)
    if family == "resid64":
        return N * 8 * (3 + nfaces_per_cell + 1)
    raise ValueError(family)


def kernel_source_hash() -> str:
    """Hash of every device source; counter summaries taken on other sources
    are not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_09671_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(family: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"counters_{family}_{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def cpu_baseline(c: dict, dt: float, rtol: float):
    """One step of the same workload on the host cores with the FP64 oracle."""
    from oracle import pyoracle as O
    from paper_2209_09671_amd import inputs as I
    st = I.initial_state(c)
    t0 = time.perf_counter()
    _, info, status = O.step(c, st, 0.0, dt, 1, rtol=rtol)
    sec = time.perf_counter() - t0
    N = c["nx"] * c["ny"] * c["nz"]
    return {"value": N / sec / 1e6, "unit": "Mcell-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"1 step of the {c['nx']}x{c['ny']}x{c['nz']} workload from its initial state, "
                      f"FP64 oracle, pressure rtol {rtol:g} ({sec:.1f} s, {info['cg_iters']} CG iterations)"}


def run_gpu(c, st, precision, steps, warmup, family=None, family_steps=5):
    """Warm-up, then `steps` timed steps without instrumentation; with a
    kernel family, `family_steps` further steps in a second timed region
    with HIP events around that family's launches (their average duration),
    so that the events do not perturb the throughput."""
    import torch
    from paper_2209_09671_amd import tcf
    g = tcf.Grid(c, precision=precision)
    g.set_state(st)
    dt = c["dt"]
    for _ in range(warmup):
        g.step(dt, 1)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    iters, refs, worst_res, worst_div = 0, 0, 0.0, 0.0
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        info = g.step(dt, 1)
        iters += info["cg_iters"]
        refs += info["refine_iters"]
        worst_res = max(worst_res, info["p_relres"])
        worst_div = max(worst_div, info["div_rel"])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    kms, kn = 0.0, 0
    if family:
        g.profile(family)
        for _ in range(family_steps):
            g.step(dt, 1)
        torch.cuda.synchronize()
        kms, kn = g.profile_read()
    g.close()
    del g
    torch.cuda.empty_cache()
    return dict(wall=wall, ev_ms=ev_ms, iters=iters / max(steps, 1), refs=refs / max(steps, 1),
                relres=worst_res, div=worst_div, kernel_ms=kms, kernel_launches=kn, info=info)


def adjoint_timing(c, st, steps, every):
    """Seconds per adjoint step (FP64): gradient of the melt-pool kinetic
    energy 1/2 h^3 sum_f rho_f u_f^2 after `steps` steps with respect to
    dsigma/dT and the initial T, checkpoints every `every` steps; the time
    includes the forward recomputation of each checkpoint segment."""
    import torch
    from paper_2209_09671_amd import tcf
    dv = lambda x: None if x is None else torch.as_tensor(x, dtype=torch.float64, device="cuda")
    a0, u0, v0, w0 = dv(st["alpha"]), dv(st["u"]), dv(st["v"]), dv(st["w"])
    s = torch.tensor(c["dsigma_dT"], dtype=torch.float64, requires_grad=True)
    T0 = dv(st["T"]).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, T, u, v, w = tcf.TcfRollout.apply(s, T0, c, a0, u0, v0, w0, steps, every)
    rho = c["rho1"] + a.clamp(0, 1) * (c["rho2"] - c["rho1"])
    h3 = c["h"] ** 3
    ke = 0.5 * h3 * ((0.5 * (rho[:, :, 1:] + rho[:, :, :-1]) * u[:, :, 1:-1] ** 2).sum()
                     + (0.5 * (rho[:, 1:, :] + rho[:, :-1, :]) * v[:, 1:-1, :] ** 2).sum())
    if w.numel():
        ke = ke + 0.5 * h3 * (0.5 * (rho[1:] + rho[:-1]) * w[1:-1] ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ke.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"value": round((t2 - t1) / steps, 5), "unit": "s/step", "precision": "fp64",
           "steps": steps, "checkpoint_every": every, "forward_s_per_step": round((t1 - t0) / steps, 5),
           "loss": "1/2 h^3 sum_f rho_f u_f^2 (melt-pool kinetic energy)",
           "dL_dsigmaT": float(s.grad), "grad_T0_norm": float(T0.grad.norm())}
    del a, T, u, v, w, T0
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--kernel", default="smooth")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--inner-rtol", type=float, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=10)
    ap.add_argument("--no-species", action="store_true")
    ap.add_argument("--no-rk3p", action="store_true")
    ap.add_argument("--no-nphase", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this path runs on one GPU; runs on several GPUs are not supported "
              "(the step is measured on one GPU's share of the grid)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2209_09671_amd import inputs as I

    c = I.config(args.workload)
    c["p_rtol"] = args.rtol
    if args.inner_rtol:
        c["inner_rtol"] = args.inner_rtol
    st = I.initial_state(c)
    N = c["nx"] * c["ny"] * c["nz"]
    wl = c["name"]

    r32 = run_gpu(c, st, 1, args.steps, args.warmup, args.kernel)
    sec = r32["ev_ms"] / 1e3
    value = N * args.steps / sec / 1e6
    fp64 = None
    if not args.no_fp64:
        r64 = run_gpu(c, st, 0, args.steps, args.warmup)
        fp64 = {"value": N * args.steps / (r64["ev_ms"] / 1e3) / 1e6, "unit": "Mcell-steps/s",
                "ms_per_step": r64["ev_ms"] / args.steps, "cg_iters_per_step": r64["iters"],
                "max_div_rel": r64["div"], "max_p_relres": r64["relres"]}

    roof = None
    if r32["kernel_launches"]:
        avg_ms = r32["kernel_ms"] / r32["kernel_launches"]
        ab = algorithmic_bytes(args.kernel, c, 1)
        ach = ab / (avg_ms / 1e3) / 1e9
        traffic = measured_traffic(args.kernel, re.sub(r"\^\d", "", wl).replace("-", ""))
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": args.kernel, "avg_launch_ms": round(avg_ms, 5),
                "launches": r32["kernel_launches"], "algorithmic_bytes_per_launch": ab}

    species = None
    if not args.no_species:
        # solutal Marangoni: the same workload carrying a species field (a
        # seeded Gaussian bump of concentration) with sigma = sigma(T, c)
        cs = I.with_species(c, -0.05, "blob")
        rs = run_gpu(cs, dict(st, c=I.species_field(cs)), 1, args.steps, args.warmup, "species")
        avg = rs["kernel_ms"] / max(rs["kernel_launches"], 1)
        ab = algorithmic_bytes("species", c, 1)
        species = {"value": round(N * args.steps / (rs["ev_ms"] / 1e3) / 1e6, 3), "unit": "Mcell-steps/s",
                   "ms_per_step": round(rs["ev_ms"] / args.steps, 4),
                   "added_ms_per_step": round((rs["ev_ms"] - r32["ev_ms"]) / args.steps, 4),
                   "cg_iters_per_step": round(rs["iters"], 2), "max_div_rel": rs["div"],
                   "dsigma_dc": cs["dsigma_dc"], "species_field": "blob",
                   "species_stage": {"kernel": "k_transport2 (species only)", "avg_launch_ms": round(avg, 5),
                                     "launches": rs["kernel_launches"], "algorithmic_bytes_per_launch": ab,
                                     "achieved_GBs": round(ab / (avg / 1e3) / 1e9, 1)}}

    rk3p = None
    if not args.no_rk3p:
        # the time-accurate integrator: SSP-RK3 over the whole state with a
        # projection in every stage (three pressure solves per step)
        rr = run_gpu(dict(c, integrator=1), st, 1, args.steps, args.warmup)
        rk3p = {"value": round(N * args.steps / (rr["ev_ms"] / 1e3) / 1e6, 3), "unit": "Mcell-steps/s",
                "ms_per_step": round(rr["ev_ms"] / args.steps, 4), "cg_iters_per_step": round(rr["iters"], 2),
                "refine_iters_per_step": round(rr["refs"], 2), "max_div_rel": rr["div"],
                "max_p_relres": rr["relres"], "integrator": "SSP-RK3, projection in every stage"}

    nphase = None
    if not args.no_nphase:
        # N-phase VOF: gas, a liquid pool and solid metal (three phases,
        # per-pair surface tension) on the same grid and beam
        cn = I.meltpool_phases(c)
        rn = run_gpu(cn, I.phase_state(cn), 1, args.steps, args.warmup)
        nphase = {"value": round(N * args.steps / (rn["ev_ms"] / 1e3) / 1e6, 3), "unit": "Mcell-steps/s",
                  "ms_per_step": round(rn["ev_ms"] / args.steps, 4), "cg_iters_per_step": round(rn["iters"], 2),
                  "max_div_rel": rn["div"], "phases": "gas, liquid metal, solid metal"}

    adj = None
    if not args.no_adjoint:
        ca = dict(c, precision=0)
        adj = adjoint_timing(ca, st, args.adjoint_steps, max(1, args.adjoint_steps // 2))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(c, c["dt"], args.rtol)

    out = {
        "metric": "Mcell-steps/s (FP32 stencils + FP64 refinement, divergence residual <= 1e-8)",
        "value": round(value, 3),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ev_ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl, "cells": N, "grid": [c["nx"], c["ny"], c["nz"]], "h_m": c["h"],
                   "dt_s": c["dt"], "precision": "fp32 stencils/inner solve, fp64 refinement",
                   "pressure_guess": f"extrapolated in time, order {c.get('p_extrapolate', 2)}",
                   "p_rtol": args.rtol, "cg_iters_per_step": round(r32["iters"], 2),
                   "refine_iters_per_step": round(r32["refs"], 2), "max_p_relres": r32["relres"],
                   "max_div_rel": r32["div"]},
        "fp64_same_accuracy": fp64,
        "wall_ms_per_step": round(r32["wall"] * 1e3 / args.steps, 4),
        "adjoint": adj,
        "solutal_species": species,
        "time_accurate_rk3": rk3p,
        "nphase_3": nphase,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
