"""Finite-difference check of the adjoint on the 3D droplet workload.

96^3 droplet (radius 0.25 at (0.5, 0.5, 0.4), sigma_T = 0.2, T = z), 200 FP64
steps of 1e-4 s, checkpoints every 20 steps.  Loss: squared distance of the
final alpha centroid from a seeded target plus 1e-3 h^3 sum u_f^2.  The
gradient with respect to dsigma/dT and the initial T field comes from
TcfRollout (tcf_step_backward); it is compared with central finite
differences of the forward path along dsigma/dT and along 16 seeded smooth
T-directions (Richardson-combined steps for T).  Pass if
|g - g_FD| <= 1e-5 max(|g_FD|, 1e-3 ||grad_T L|| ||d||).

Run on a GPU:  python tests/fd_check_droplet3d.py [--n 96 --steps 200 --dirs 16]
Prints one JSON line.  Not collected by pytest (minutes of GPU time).
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2209_09671_amd import inputs as I  # noqa: E402
from paper_2209_09671_amd import tcf  # noqa: E402
from test_gpu_adjoint import centroid_loss, dev, host  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--every", type=int, default=20)
    ap.add_argument("--dirs", type=int, default=16)
    ap.add_argument("--rtol", type=float, default=1e-13)
    args = ap.parse_args()
    c = I.config(3) if args.n == 96 else I.custom(I.config(3), nx=args.n, ny=args.n, nz=args.n)
    c["p_rtol"] = args.rtol
    st = I.initial_state(c)
    a0, u0, v0, w0 = dev(st["alpha"]), dev(st["u"]), dev(st["v"]), dev(st["w"])
    tgt = torch.tensor(np.array(c["drop_centre"]) + I.target_centroid(c), device="cuda")
    n, k = args.steps, args.every

    def L(sv, T):
        with torch.no_grad():
            o = tcf.TcfRollout.apply(torch.tensor(sv, dtype=torch.float64), T, c, a0, u0, v0, w0, n, k)
            return float(centroid_loss(c, o[0], o[2], o[3], o[4], tgt))

    s = torch.tensor(c["dsigma_dT"], dtype=torch.float64, requires_grad=True)
    T0 = dev(st["T"]).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = tcf.TcfRollout.apply(s, T0, c, a0, u0, v0, w0, n, k)
    loss = centroid_loss(c, out[0], out[2], out[3], out[4], tgt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gs, gT = float(s.grad), host(T0.grad)
    gnorm = float(np.linalg.norm(gT))
    print(f"[fd] loss {float(loss):.6e} dL/ds {gs:.6e} |dL/dT0| {gnorm:.3e} "
          f"forward {t1 - t0:.2f} s backward {t2 - t1:.2f} s", flush=True)

    s0 = c["dsigma_dT"]
    es = 1e-4 * abs(s0)
    fds = (L(s0 + es, T0.detach()) - L(s0 - es, T0.detach())) / (2 * es)
    rows = [dict(kind="dsigma_dT", adjoint=gs, fd=fds, err=abs(gs - fds), scale=abs(fds),
                 ok=abs(gs - fds) <= 1e-5 * abs(fds))]
    print(f"[fd] s: adjoint {gs:.10e} fd {fds:.10e} rel {abs(gs - fds) / abs(fds):.2e}", flush=True)

    def richardson(fun, eps):
        d1 = (fun(eps) - fun(-eps)) / (2 * eps)
        d2 = (fun(eps / 2) - fun(-eps / 2)) / eps
        return (4 * d2 - d1) / 3

    for q, dT in enumerate(I.t_directions(c, k=args.dirs)):
        dTd = dev(dT)
        fd = richardson(lambda e: L(s0, T0.detach() + e * dTd), 4e-2)
        ad = float(np.vdot(gT, dT))
        scale = max(abs(fd), 1e-3 * gnorm * float(np.linalg.norm(dT)))
        rows.append(dict(kind=f"T0 direction {q}", adjoint=ad, fd=fd, err=abs(ad - fd), scale=scale,
                         ok=abs(ad - fd) <= 1e-5 * scale))
        print(f"[fd] T{q}: adjoint {ad:.10e} fd {fd:.10e} rel {abs(ad - fd) / scale:.2e}", flush=True)
    worst = max(r["err"] / r["scale"] for r in rows)
    print(json.dumps({"workload": c["name"], "grid": [c["nx"], c["ny"], c["nz"]], "steps": n,
                      "checkpoint_every": k, "loss": float(loss), "dL_dsigmaT": gs, "grad_T0_norm": gnorm,
                      "checks": len(rows), "passed": sum(r["ok"] for r in rows), "worst_rel": worst,
                      "forward_s_per_step": (t1 - t0) / n,
                      "adjoint_s_per_step": (t2 - t1) / n}), flush=True)
    sys.exit(0 if all(r["ok"] for r in rows) else 1)


if __name__ == "__main__":
    main()
