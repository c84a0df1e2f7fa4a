#!/usr/bin/env python
"""Throughput of the thermocapillary projection step on one MI355X.

A step is one pass of the whole path (WENO5-RK3 transport of alpha and T,
geometry and CSF force, momentum predictor, MG-PCG pressure solve with FP64
refinement, projection, FP64 diagnostics) over the 256^3 melt-pool workload
(cell 2.5 um, density ratio 7500, moving 200 W Gaussian heat flux), all
inputs resident in HBM.  The primary line is the FP32-stencil path with FP64
iterative refinement at a divergence residual <= 1e-8; the plain FP64 path at
the same accuracy is reported beside it.

The timed steps follow a spin-up (--spinup, default 200 steps from rest):
the beam has then heated the melt surface and driven a Marangoni flow (CFL
~0.12 at step 200), and the pressure solve needs the iterations of the
developed flow (7 CG iterations and 2 refinements per step instead of 4 and
1 from rest).  With no phase change the surface temperature keeps rising and
the flow passes the explicit CFL limit near step 330, so the window stays
below that.  Then --warmup W untimed and --steps K timed steps.

Prints ONE JSON line.  Options: --steps K --warmup W --gpus 1 --spinup S
--cpu-steps C --no-cpu --no-fp64 --no-kernels --no-adjoint --no-species
--no-rk3p --no-nphase.  `--trace-summary CSV` prints the per-kernel table of
the last --trace-steps steps of a rocprofv3 kernel trace instead (with
--trace-adjoint: the backward sweep of --trace-steps adjoint steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# kernel families timed with HIP events (tcf_profile), in the order tried
FAMILIES = ("transport", "smooth2", "smooth", "update", "spmv", "predictor", "resid64", "project", "geometry")
KERNEL_NAMES = {"transport": "k_transport2<float,3,1>", "smooth": "k0_smooth<float,3,false>",
                "smooth2": "k0_smooth2<float,true,8>",
                "update": "k0_update_smooth<float,3>", "spmv": "k0_spmv_upd<float,3>",
                "predictor": "k_pred2_f<float,3,0..2> (the three components)", "resid64": "k0_resid64<float,3>",
                "project": "k_project_diag<float,3>", "geometry": "k_geometry_z<float>",
                "species": "k_transport2<float,3,0>"}


def algorithmic_bytes(family: str, c: dict) -> float:
    """Bytes one launch of a kernel family of the FP32 path must move (each
    value read or written once; face arrays counted as N values)."""
    N = c["nx"] * c["ny"] * c["nz"]
    w = 4
    nf = 3 if c["dim"] == 3 else 2
    if family == "smooth":
        # finest-level Jacobi sweep: x, b, alpha (face weights recomputed) read, x' written
        return N * w * (3 + 1)
    if family == "smooth2":
        # both post-smoothing sweeps in one pass: x, b, alpha and the coarse
        # correction (1/8) read, x'' written
        return N * w * (3 + 1 / 8 + 1)
    if family == "spmv":
        # d <- z + beta d with d'.K d': z, d, alpha read; d' written (K d' not stored)
        return N * w * (3 + 1)
    if family == "update":
        # x += alpha d, r -= alpha K d (K d recomputed), first sweep: x, r, d, alpha / x, r, z1
        return N * w * (4 + 3)
    if family == "transport":
        # per stage, averaged over the three: alpha, T, one velocity per axis,
        # base alpha and T (stages 2, 3) read; alpha, T written
        return N * w * (2 + nf + 2 * 2 / 3 + 2)
    if family == "species":
        return N * w * (1 + nf + 2 / 3 + 1)
    if family == "predictor":
        # one timed launch is the three (two) component kernels; per component:
        # alpha, sigma*kappa, M_d and the nf velocities read; u*_d written
        return N * w * nf * (3 + nf + 1)
    if family == "resid64":
        # FP64 refinement residual: b, p (FP64), alpha read; r (FP64) written
        return N * (8 + 8 + w + 8)
    if family == "project":
        # alpha, p (FP64), u*, v*, w* read; u, v, w written in FP64 and FP32
        return N * (w + 8 + nf * w) + N * nf * (8 + w)
    if family == "geometry":
        # alpha, T read; sigma*kappa and the nf components of M written
        return N * w * (2 + 1 + nf)
    raise ValueError(family)


def step_bytes_per_cell(n_it: float, n_ref: float, precision: int) -> float:
    """The path's algorithmic HBM bytes per cell-step: 42 + 26 n_it values
    (transport stages 25, predictor with the divergence 9, projection 8, and
    per CG iteration the SpMV, the vector updates and one V(2,2) cycle's
    finest-level sweeps with the coarse levels' share) of w bytes, plus in
    the FP32 path the FP64 words of u, v, w, p and the right-hand side, and
    per refinement the FP64 residual pass."""
    if precision == 1:
        return (42 + 26 * n_it) * 4 + (8 + 28 * n_ref)
    return (42 + 26 * n_it) * 8


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
    they were taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"counters_{family}_{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def measured_valu_busy(kernel: str, workload: str):
    """Fraction of the SIMD cycles a kernel issues VALU work in, from the
    committed SQ counter summary, if it was taken on the current kernel
    sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"sq_valu_{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    want = kernel.replace(" ", "")
    for line in txt.splitlines():
        cells = [x.strip() for x in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0].replace(" ", "") == want and cells[4].endswith("%"):
            return float(cells[4][:-1]) / 100.0
    return None


def host_cpu():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(c: dict, rtol: float, steps: int):
    """The FP64 oracle on the host cores: the first `steps` steps of the
    same workload from its initial state."""
    from oracle import pyoracle as O
    from paper_2209_09671_amd import inputs as I
    st = I.initial_state(c)
    t0 = time.perf_counter()
    _, info, status = O.step(c, st, 0.0, c["dt"], steps, rtol=rtol)
    sec = time.perf_counter() - t0
    N = c["nx"] * c["ny"] * c["nz"]
    model, ncpu = host_cpu()
    return {"value": N * steps / sec / 1e6, "unit": "Mcell-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"first {steps} steps of the {c['nx']}x{c['ny']}x{c['nz']} workload from its initial state "
                      f"(FP64 oracle, pressure rtol {rtol:g}, {sec:.1f} s; {info['cg_iters']} CG iterations in "
                      f"the last step)",
            "cpu_model": model, "nproc": ncpu, "status": status}


def run_gpu(c, st, precision, spinup, warmup, steps, families=(), family_steps=None):
    """Spin-up, warm-up, then `steps` timed steps without instrumentation;
    then, per kernel family, the first `family_steps` (default: all) steps of
    the timed window again, from its saved start state (the replay is
    bitwise the timed run, so every family is measured on the same steps,
    with the window's launches per step), with HIP events around that
    family's launches (their average duration), so that the events do not
    perturb the throughput."""
    import torch
    from paper_2209_09671_amd import tcf
    g = tcf.Grid(c, precision=precision)
    g.set_state(st)
    dt = c["dt"]
    sp_it = sp_ref = 0
    sp_cfl = 0.0
    for _ in range(spinup):
        info = g.step(dt, 1)
        sp_it += info["cg_iters"]
        sp_ref += info["refine_iters"]
        sp_cfl = max(sp_cfl, info["cfl_max"])
    for _ in range(warmup):
        g.step(dt, 1)
    start = g.get_fields() if families else None
    if start is not None and c.get("species"):
        start["c"] = g.get_species()
    if start is not None and c.get("nphases", 0) > 2:
        start["alpha3"], start["alpha4"] = g.get_phases()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    iters, refs, worst_res, worst_div, cfl = 0, 0, 0.0, 0.0, 0.0
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        info = g.step(dt, 1)
        iters += info["cg_iters"]
        refs += info["refine_iters"]
        worst_res = max(worst_res, info["p_relres"])
        worst_div = max(worst_div, info["div_rel"])
        cfl = max(cfl, info["cfl_max"])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    fams = {}
    nfam = steps if family_steps is None else min(family_steps, steps)
    for fam in families:
        g.set_state(start, start["t"])
        g.profile(fam)
        for _ in range(nfam):
            g.step(dt, 1)
        torch.cuda.synchronize()
        kms, kn = g.profile_read()
        g.profile(None)
        fams[fam] = (kms, kn, nfam)
    del start
    g.close()
    del g
    torch.cuda.empty_cache()
    return dict(wall=wall, ev_ms=ev_ms, iters=iters / max(steps, 1), refs=refs / max(steps, 1),
                relres=worst_res, div=worst_div, cfl=cfl, info=info, fams=fams,
                spinup=dict(steps=spinup, cg_iters_per_step=round(sp_it / max(spinup, 1), 2),
                            refine_iters_per_step=round(sp_ref / max(spinup, 1), 2), max_cfl=round(sp_cfl, 4)))


def kernel_table(r, c):
    rows = {}
    for fam, (kms, kn, nst) in r["fams"].items():
        if not kn:
            continue
        avg = kms / kn
        ab = algorithmic_bytes(fam, c)
        ach = ab / (avg / 1e3) / 1e9
        rows[fam] = {"kernel": KERNEL_NAMES.get(fam, fam), "avg_launch_ms": round(avg, 5),
                     "launches_per_step": round(kn / nst, 2), "ms_per_step": round(kms / nst, 4),
                     "algorithmic_bytes_per_launch": ab, "achieved_GBs": round(ach, 1),
                     "frac": round(ach / HBM_PEAK_GBS, 4)}
    return rows


def adjoint_timing(c, spin, steps, every):
    """Seconds per adjoint step (FP64): gradient of the melt-pool kinetic
    energy 1/2 h^3 sum_f rho_f u_f^2 after `steps` steps, started from the
    state after `spin` steps, with respect to dsigma/dT and that state's T;
    checkpoints every `every` steps; the time includes the forward
    recomputation of each checkpoint segment."""
    import torch
    from paper_2209_09671_amd import inputs as I
    from paper_2209_09671_amd import tcf
    g = tcf.Grid(c, precision=0)
    g.set_state(I.initial_state(c))
    for _ in range(spin):
        g.step(c["dt"], 1)
    f = g.get_fields()
    g.close()
    t_start = f["t"]
    a0, u0, v0, w0, p0 = f["alpha"], f["u"], f["v"], f["w"], f["p"]
    s = torch.tensor(c["dsigma_dT"], dtype=torch.float64, requires_grad=True)
    T0 = f["T"].clone().requires_grad_(True)
    del f
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, T, u, v, w = tcf.TcfRollout.apply(s, T0, c, a0, u0, v0, w0, steps, every, t_start, p0)
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
           "steps": steps, "checkpoint_every": every, "window": f"steps {spin}..{spin + steps}",
           "forward_s_per_step": round((t1 - t0) / steps, 5),
           "loss": "1/2 h^3 sum_f rho_f u_f^2 (melt-pool kinetic energy)",
           "dL_dsigmaT": float(s.grad), "grad_T_norm": float(T0.grad.norm())}
    del a, T, u, v, w, T0, a0, u0, v0, w0, p0
    torch.cuda.empty_cache()
    return out


def trace_summary(path, nsteps, marker="k_transport2<float, 3, 1>", per_step=3, adjoint=False):
    """Markdown table of the kernels of the last `nsteps` steps of a
    rocprofv3 kernel trace (CSV); a step is found by its `per_step`
    launches of `marker` (the transport stages).  With `adjoint`, the window
    is the backward sweep instead (first to last adjoint kernel, recomputed
    forward segments included), over `nsteps` adjoint steps.  Needs no GPU."""
    import collections
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    if adjoint:
        idx = [i for i, r in enumerate(rows) if "::ka_" in r[2]]
        win = rows[idx[0]:idx[-1] + 1]
    else:
        idx = [i for i, r in enumerate(rows) if marker in r[2]]
        win = rows[idx[-nsteps * per_step]:]
    t0, t1 = win[0][0], win[-1][1]
    agg = collections.defaultdict(lambda: [0, 0.0])
    for a, b, n in win:
        n = n.replace("void ", "").replace("tcf::(anonymous namespace)::", "").split("(")[0]
        agg[n][0] += 1
        agg[n][1] += (b - a) / 1e3
    tot = sum(v[1] for v in agg.values())
    what = f"the backward sweep of {nsteps} adjoint steps" if adjoint else f"the last {nsteps} steps"
    out = [f"Window: {what}, {len(win)} dispatches, span {(t1 - t0) / 1e6:.3f} ms "
           f"({(t1 - t0) / 1e6 / nsteps:.3f} ms/step), kernel time {tot / 1e3 / nsteps:.3f} ms/step.", "",
           "| kernel | calls/step | avg us | ms/step | % |", "|---|---:|---:|---:|---:|"]
    for n, (c, us) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| {n} | {c / nsteps:.2f} | {us / c:.2f} | {us / 1e3 / nsteps:.3f} | {100 * us / tot:.1f} |")
    return "\n".join(out)


def leg_summary(r, N, steps):
    return {"value": round(N * steps / (r["ev_ms"] / 1e3) / 1e6, 3), "unit": "Mcell-steps/s",
            "ms_per_step": round(r["ev_ms"] / steps, 4), "cg_iters_per_step": round(r["iters"], 2),
            "refine_iters_per_step": round(r["refs"], 2), "max_div_rel": r["div"], "max_p_relres": r["relres"],
            "max_cfl": round(r["cfl"], 4), "spinup": r["spinup"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--spinup", type=int, default=200)
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--inner-rtol", type=float, default=None)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=None)
    ap.add_argument("--adjoint-spinup", type=int, default=50)
    ap.add_argument("--no-species", action="store_true")
    ap.add_argument("--no-rk3p", action="store_true")
    ap.add_argument("--no-nphase", action="store_true")
    ap.add_argument("--trace-summary", default=None,
                    help="print the per-kernel table of the last --trace-steps steps of a rocprofv3 "
                         "kernel trace CSV and exit (no GPU)")
    ap.add_argument("--trace-steps", type=int, default=20)
    ap.add_argument("--trace-adjoint", action="store_true",
                    help="with --trace-summary: tabulate the adjoint's backward sweep (--trace-steps steps)")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(args.trace_summary, args.trace_steps, adjoint=args.trace_adjoint))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this path runs on one GPU; runs on several GPUs are not supported "
              "(the step is measured on one GPU's share of the grid)", file=sys.stderr)
        sys.exit(2)

    from paper_2209_09671_amd import inputs as I

    c = I.config(args.workload)
    c["p_rtol"] = args.rtol
    if args.inner_rtol:
        c["inner_rtol"] = args.inner_rtol
    st = I.initial_state(c)
    N = c["nx"] * c["ny"] * c["nz"]
    wl = c["name"]
    K, W, S = args.steps, args.warmup, args.spinup
    window = f"steps {S + W + 1}..{S + W + K} of a run from rest"

    r32 = run_gpu(c, st, 1, S, W, K, () if args.no_kernels else FAMILIES)
    sec = r32["ev_ms"] / 1e3
    value = N * K / sec / 1e6
    ms = r32["ev_ms"] / K
    fp64 = None
    if not args.no_fp64:
        r64 = run_gpu(c, st, 0, S, W, K)
        fp64 = leg_summary(r64, N, K)
        b64 = step_bytes_per_cell(r64["iters"], 0, 0)
        fp64["step_hbm"] = {"bytes_per_cell_step": b64,
                            "achieved_GBs": round(N * b64 / (fp64["ms_per_step"] / 1e3) / 1e9, 1),
                            "frac": round(N * b64 / (fp64["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

    kernels = kernel_table(r32, c)
    roof = None
    if kernels:
        # the kernel family that takes the most time per step
        dom = max(kernels, key=lambda f: kernels[f]["ms_per_step"])
        k = kernels[dom]
        workload_tag = re.sub(r"\^\d", "", wl).replace("-", "")
        roof = {"bound": "hbm", "achieved": k["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": k["frac"], "traffic": measured_traffic(dom, workload_tag),
                "kernel": dom, "kernel_name": k["kernel"], "avg_launch_ms": k["avg_launch_ms"],
                "launches_per_step": k["launches_per_step"], "ms_per_step": k["ms_per_step"],
                "algorithmic_bytes_per_launch": k["algorithmic_bytes_per_launch"],
                "valu_busy": measured_valu_busy(k["kernel"], workload_tag)}
    b32 = step_bytes_per_cell(r32["iters"], r32["refs"], 1)
    step_hbm = {"model": "(42 + 26 n_it) 4 + (8 + 28 n_ref) B per cell-step",
                "bytes_per_cell_step": round(b32, 1),
                "achieved_GBs": round(N * b32 / (ms / 1e3) / 1e9, 1),
                "frac": round(N * b32 / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

    species = None
    if not args.no_species:
        # solutal Marangoni: the same workload carrying a species field (a
        # seeded Gaussian bump of concentration) with sigma = sigma(T, c)
        cs = I.with_species(c, -0.05, "blob")
        rs = run_gpu(cs, dict(st, c=I.species_field(cs)), 1, S, W, K, ("species",))
        species = leg_summary(rs, N, K)
        species.update(added_ms_per_step=round(species["ms_per_step"] - ms, 4), dsigma_dc=cs["dsigma_dc"],
                       species_field="blob", species_stage=kernel_table(rs, c).get("species"))

    rk3p = None
    if not args.no_rk3p:
        # the time-accurate integrator: SSP-RK3 over the whole state with a
        # projection in every stage (three pressure solves per step)
        rk3p = leg_summary(run_gpu(dict(c, integrator=1), st, 1, S, W, K), N, K)
        rk3p["integrator"] = "SSP-RK3, projection in every stage"

    nphase = None
    if not args.no_nphase:
        # N-phase VOF: gas, a liquid pool and solid metal (three phases,
        # per-pair surface tension) on the same grid and beam
        cn = I.meltpool_phases(c)
        nphase = leg_summary(run_gpu(cn, I.phase_state(cn), 1, S, W, K), N, K)
        nphase["phases"] = "gas, liquid metal, solid metal"

    adj = None
    if not args.no_adjoint:
        ca = dict(c, precision=0)
        n_adj = args.adjoint_steps or c.get("adjoint_steps", 200)
        adj = adjoint_timing(ca, args.adjoint_spinup, n_adj, c.get("checkpoint_every", 25))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(c, args.rtol, args.cpu_steps)

    out = {
        "metric": "Mcell-steps/s (FP32 stencils + FP64 refinement, divergence residual <= 1e-8)",
        "value": round(value, 3),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl, "cells": N, "grid": [c["nx"], c["ny"], c["nz"]], "h_m": c["h"],
                   "dt_s": c["dt"], "window": window, "spinup_steps": S,
                   "precision": "fp32 stencils/inner solve, fp64 refinement",
                   "pressure_guess": f"extrapolated in time, order {c.get('p_extrapolate', 2)}",
                   "p_rtol": args.rtol, "cg_iters_per_step": round(r32["iters"], 2),
                   "refine_iters_per_step": round(r32["refs"], 2), "max_p_relres": r32["relres"],
                   "max_div_rel": r32["div"], "max_cfl": round(r32["cfl"], 4), "spinup": r32["spinup"]},
        "fp64_same_accuracy": fp64,
        "wall_ms_per_step": round(r32["wall"] * 1e3 / K, 4),
        "step_hbm": step_hbm,
        "kernels": kernels,
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
