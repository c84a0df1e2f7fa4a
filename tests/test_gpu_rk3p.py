"""The time-accurate integrator (integrator 1: SSP-RK3 over the whole state
with a projection in every stage) on the HIP path, through the C ABI, against
the FP64 oracle on the same seeded inputs.

Bars as for the default step: FP64 per-field relative L2 <= 1e-10 after one
step and <= 1e-8 after many (p mean-free); FP32 + FP64 refinement keeps the
divergence residual <= 1e-8 with alpha and T within 1e-6 of the FP64 oracle.
Without momentum and heat source the GPU's two integrators agree bitwise,
and the GPU path itself converges at third order in time.
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


def gpu_run(c, st, dt, nsteps, precision=0, flags=None):
    print(f"[gpu] rk3p {c.get('name')} {c['nx']}x{c['ny']}x{c['nz']} prec={precision} steps={nsteps}",
          flush=True)
    g = tcf.Grid(c, precision=precision, flags=flags)
    g.set_state(st)
    info = g.step(dt, nsteps, check=False)
    out = g.get_fields()
    if c.get("species"):
        out["c"] = g.get_species()
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in out.items()}
    g.close()
    return out, info


@pytest.mark.parametrize("nsteps,tol", [(1, 1e-10), (20, 1e-8)])
def test_rk3p_2d_droplet_matches_oracle(nsteps, tol):
    c = dict(I.config(0), integrator=1)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], nsteps)
    o, oinfo, _ = O.step(c, st, 0.0, c["dt"], nsteps)
    assert info["status"] == 0, info
    e = errors(g, o)
    assert max(e.values()) <= tol, e
    assert info["div_rel"] <= 1e-9, info


def test_rk3p_3d_with_species_matches_oracle():
    c = I.with_species(dict(I.custom(I.config(3), nx=40, ny=40, nz=40), integrator=1), -0.3, "linear_x")
    st = I.initial_state(c)
    st["c"] = I.species_field(c)
    g, info = gpu_run(c, st, c["dt"], 2)
    o, _, _ = O.step(c, st, 0.0, c["dt"], 2)
    e = errors(g, o)
    assert max(e.values()) <= 1e-10, e


def test_rk3p_moving_heat_source_matches_oracle():
    """The stage times of the heat source (t, t + dt, t + dt/2)."""
    c = dict(I.custom(I.config(0), nx=48, ny=40), integrator=1)
    c.update(q_power=5.0, q_radius=0.1, q_x0=0.3, q_y0=0.5, q_vx=5.0, q_vy=0.0)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, 1e-3, 4)
    o, _, _ = O.step(c, st, 0.0, 1e-3, 4)
    e = errors(g, o)
    assert max(e.values()) <= 1e-10, e


def test_rk3p_fp32_refined_meltpool():
    c = dict(I.custom(I.config(2), nx=64, ny=32, nz=32), integrator=1)
    c["p_rtol"] = 1e-8
    st = I.initial_state(c)
    g, info = gpu_run(c, st, 1e-8, 2, precision=1)
    o, _, _ = O.step(c, st, 0.0, 1e-8, 2, rtol=1e-12)
    assert info["status"] == 0, info
    assert info["div_rel"] <= 1e-8
    e = errors(g, o, ("alpha", "T"))
    assert max(e.values()) <= 1e-6, e


def test_rk3p_transport_only_equals_default_transport():
    """Frozen velocity and no heat source: the GPU's two integrators run the
    same three transport stages, bitwise."""
    c = I.with_species(I.custom(I.config(0), nx=48, ny=48), -0.3, "blob")
    st = I.initial_state(c)
    st["c"] = I.species_field(c)
    st["u"], st["v"] = I.stream_velocity(c, 1.0)[:2]
    f = tcf.TCF_TRANSPORT_ONLY
    g0, _ = gpu_run(dict(c, integrator=0), st, 2e-3, 5, flags=f)
    g1, _ = gpu_run(dict(c, integrator=1), st, 2e-3, 5, flags=f)
    for k in ("alpha", "T", "c"):
        assert np.array_equal(g0[k], g1[k]), k


def test_rk3p_third_order_on_the_gpu():
    """The 32^2 thermocapillary droplet in FP64: the GPU path's time error at
    t = 0.008 falls by about 8 per halving of dt."""
    c = dict(I.custom(I.config(0), nx=32, ny=32), integrator=1, p_rtol=1e-13)
    st = I.initial_state(c)
    runs = {}
    for dt in (0.001, 0.0005, 0.00025, 0.00025 / 8):
        runs[dt], _ = gpu_run(c, st, dt, int(round(0.008 / dt)))
    ref = runs[0.00025 / 8]
    for k in ("u", "alpha", "T"):
        es = [rel(runs[dt][k], ref[k]) for dt in (0.001, 0.0005, 0.00025)]
        orders = [np.log2(es[i] / es[i + 1]) for i in range(2)]
        assert min(orders) >= 2.8, (k, es, orders)


def test_rk3p_rejected_with_adjoint_and_bad_value():
    with pytest.raises(tcf.TcfError) as ei:
        tcf.Grid(dict(I.config(0), integrator=1), precision=0, flags=tcf.TCF_WITH_ADJOINT)
    assert ei.value.status == tcf.TCF_E_INVALID
    with pytest.raises(tcf.TcfError) as ei:
        tcf.Grid(dict(I.config(0), integrator=3), precision=0)
    assert ei.value.status == tcf.TCF_E_INVALID


def test_rk3p_full_size_meltpool_256_properties():
    """256^3 melt pool in the benchmark's launch configuration for the
    time-accurate integrator (FP32 + refinement): two steps, finite fields,
    every stage's solve converged (status 0), FP64 divergence residual of
    the last projection <= 1e-8, alpha conserved."""
    c = dict(I.config(4), integrator=1, p_rtol=1e-8)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], 2, precision=1)
    assert info["status"] == 0 and info["nonfinite"] == 0, info
    assert info["div_rel"] <= 1e-8, info
    s0 = st["alpha"].sum()
    assert abs(float(g["alpha"].sum()) - s0) <= 1e-6 * s0
