"""Solutal Marangoni (species field c, sigma(T, c)) on the HIP path, through
the C ABI, against the FP64 oracle on the same seeded inputs.

Bars as for the thermal step: FP64 per-field relative L2 <= 1e-10 after one
step and <= 1e-8 after many; the species itself (c) is held to the same bar.
The FP32 + FP64-refinement path keeps its divergence residual <= 1e-8 with
alpha, T and c within 1e-6 of the FP64 oracle.  The GPU also reproduces the
oracle's reductions: c = alpha stays alpha, and c := T with the slopes
swapped gives the thermal step.
"""
import numpy as np
import pytest
import torch

from oracle import pyoracle as O
from paper_2209_09671_amd import inputs as I
from paper_2209_09671_amd import tcf

pytestmark = pytest.mark.gpu

KEYS = ("alpha", "T", "c", "u", "v", "w", "p")


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def errors(g, o, keys=KEYS):
    e = {}
    for k in keys:
        if g.get(k) is None or o.get(k) is None:
            continue
        x, y = g[k], o[k]
        if k == "p":
            x, y = x - x.mean(), y - y.mean()
        e[k] = rel(x, y)
    return e


def gpu_run(c, st, dt, nsteps, precision=0):
    print(f"[gpu] species {c.get('name')} {c['nx']}x{c['ny']}x{c['nz']} prec={precision} steps={nsteps}",
          flush=True)
    g = tcf.Grid(c, precision=precision)
    g.set_state(st)
    info = g.step(dt, nsteps, check=False)
    out = g.get_fields()
    out["c"] = g.get_species()
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in out.items()}
    g.close()
    return out, info


def species_state(cs):
    st = I.initial_state(cs)
    st["c"] = I.species_field(cs)
    return st


@pytest.mark.parametrize("nsteps,tol", [(1, 1e-10), (30, 1e-8)])
def test_species_step_2d_matches_oracle(nsteps, tol):
    cs = I.with_species(I.config(0), -0.3, "blob")
    st = species_state(cs)
    g, info = gpu_run(cs, st, cs["dt"], nsteps)
    o, _, _ = O.step(cs, st, 0.0, cs["dt"], nsteps)
    assert info["status"] == 0, info
    e = errors(g, o)
    assert max(e.values()) <= tol, e
    assert abs(g["c"].sum() - st["c"].sum()) <= 1e-13 * nsteps * st["c"].sum()


def test_species_step_3d_matches_oracle():
    cs = I.with_species(I.custom(I.config(3), nx=40, ny=40, nz=40), -0.3, "linear_x")
    st = species_state(cs)
    g, info = gpu_run(cs, st, cs["dt"], 2)
    o, _, _ = O.step(cs, st, 0.0, cs["dt"], 2)
    e = errors(g, o)
    assert max(e.values()) <= 1e-10, e


def test_species_fp32_refined_meltpool():
    c = I.custom(I.config(2), nx=64, ny=32, nz=32)
    c["p_rtol"] = 1e-8
    cs = I.with_species(c, -2e-3, "blob")
    st = species_state(cs)
    g, info = gpu_run(cs, st, 1e-8, 2, precision=1)
    o, _, _ = O.step(cs, st, 0.0, 1e-8, 2, rtol=1e-12)
    assert info["status"] == 0, info
    assert info["div_rel"] <= 1e-8
    e = errors(g, o, ("alpha", "T", "c"))
    assert max(e.values()) <= 1e-6, e


def test_species_copy_of_alpha_stays_alpha():
    cs = I.with_species(I.custom(I.config(3), nx=32, ny=32, nz=32), -0.2, "alpha")
    st = species_state(cs)
    g, _ = gpu_run(cs, st, cs["dt"], 5)
    assert np.array_equal(g["c"], g["alpha"])


def test_species_equal_to_temperature_gives_thermal_step():
    c = I.custom(I.config(0), nx=48, ny=48)
    c["T_bc"] = [0] * 6
    c["lambda1"] = c["lambda2"] = 0.0
    st = I.initial_state(c)
    g0 = tcf.Grid(c, precision=0)
    g0.set_state(st)
    g0.step(c["dt"], 6)
    ref = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in g0.get_fields().items()}
    g0.close()
    cs = I.with_species(c, c["dsigma_dT"], c0=c["T0"])
    cs["dsigma_dT"] = 0.0
    g, _ = gpu_run(cs, dict(st, c=st["T"].copy()), c["dt"], 6)
    for k in ("alpha", "T", "u", "v", "p"):
        assert np.array_equal(g[k], ref[k]), k
    assert np.array_equal(g["c"], g["T"])


def test_species_state_errors():
    cs = I.with_species(I.config(0), -0.3)
    g = tcf.Grid(cs, precision=0)
    g.set_state(I.initial_state(cs))  # no species field yet
    with pytest.raises(tcf.TcfError) as ei:
        g.step(cs["dt"], 1)
    assert ei.value.status == tcf.TCF_E_STATE
    g.close()
    g = tcf.Grid(I.config(0), precision=0)
    with pytest.raises(tcf.TcfError) as ei:
        g.set_species(torch.zeros((1, 64, 64), dtype=torch.float64, device="cuda"))
    assert ei.value.status == tcf.TCF_E_STATE
    g.close()
