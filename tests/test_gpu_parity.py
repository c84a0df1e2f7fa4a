"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Same seeded inputs on both sides; per-field relative L2 errors
||x_gpu - x_oracle|| / ||x_oracle|| (pressure compared mean-free).
Bars: FP64 step <= 1e-10 after one step and <= 1e-8 after 100 steps;
transport-only and single operators, which involve no iterative solve,
<= 1e-12; the FP32 + FP64-refinement step is held to a looser per-field bar
(reported) with its FP64 divergence residual <= 1e-8.
"""
import numpy as np
import pytest
import torch

from oracle import pyoracle as O
from paper_2209_09671_amd import inputs as I
from paper_2209_09671_amd import tcf

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def host(d):
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in d.items()}


def gpu_run(c, st, dt, nsteps, precision=0, flags=0, t=0.0):
    print(f"[gpu] {c.get('name')} {c['nx']}x{c['ny']}x{c['nz']} prec={precision} flags={flags} "
          f"steps={nsteps}", flush=True)
    g = tcf.Grid(c, precision=precision, flags=flags)
    g.set_state(st, t)
    info = g.step(dt, nsteps, check=False)
    out = host(g.get_fields())
    g.close()
    return out, info


FIELDS = ("alpha", "T", "u", "v", "w", "p")


def field_errors(a, b, keys=FIELDS):
    e = {}
    for k in keys:
        if a.get(k) is None or b.get(k) is None:
            continue
        x, y = a[k], b[k]
        if k == "p":
            x, y = x - x.mean(), y - y.mean()
        e[k] = rel(x, y)
    return e


# ---------------------------------------------------------------------------
def _with_flow(c, amp):
    st = I.initial_state(c)
    st["u"], st["v"], st["w"] = I.stream_velocity(c, amp)
    return st


@pytest.mark.parametrize("nsteps", [1, 100])
def test_transport_only_2d_droplet(nsteps):
    c = I.config(0)
    st = _with_flow(c, 0.5)
    dt = 1e-3
    g, _ = gpu_run(c, st, dt, nsteps, flags=tcf.TCF_TRANSPORT_ONLY)
    o, _, _ = O.step(c, st, 0.0, dt, nsteps, flags=O.F_TRANSPORT_ONLY)
    e = field_errors(g, o, ("alpha", "T"))
    assert max(e.values()) <= 1e-12, e


def test_transport_only_2d_ragged_tiles():
    c = I.custom(I.config(0), nx=100, ny=70)
    c["h"] = 1.0 / 100
    st = _with_flow(c, 0.5)
    g, _ = gpu_run(c, st, 1e-3, 5, flags=tcf.TCF_TRANSPORT_ONLY)
    o, _, _ = O.step(c, st, 0.0, 1e-3, 5, flags=O.F_TRANSPORT_ONLY)
    e = field_errors(g, o, ("alpha", "T"))
    assert max(e.values()) <= 1e-12, e


def test_transport_only_3d_meltpool_ragged_with_heat_source():
    c = I.custom(I.config(2), nx=70, ny=29, nz=21)
    c["q_x0"], c["q_y0"] = 35 * c["h"], 14 * c["h"]
    st = _with_flow(c, 5.0)
    g, _ = gpu_run(c, st, 1e-8, 3, precision=0, flags=tcf.TCF_TRANSPORT_ONLY)
    o, _, _ = O.step(c, st, 0.0, 1e-8, 3, flags=O.F_TRANSPORT_ONLY)
    e = field_errors(g, o, ("alpha", "T"))
    assert max(e.values()) <= 1e-12, e
    assert np.abs(g["T"] - st["T"]).max() > 1.0     # the beam heated the surface


def test_predictor_parity_2d_and_3d():
    for c in (I.config(0), I.custom(I.config(3), nx=36, ny=28, nz=20)):
        st = _with_flow(c, 0.2)
        print(f"[gpu] predictor {c['nx']}x{c['ny']}x{c['nz']}", flush=True)
        g = tcf.Grid(c)
        g.set_state(st)
        us, vs, ws = g.predictor(c["dt"])
        got = host(dict(u=us, v=vs, w=ws))
        g.close()
        ref = O.predictor(c, c["dt"], st["alpha"], st["T"], st["u"], st["v"], st["w"])
        for k, r in zip(("u", "v", "w"), ref):
            if r is not None:
                assert rel(got[k], r) <= 1e-12, (k, rel(got[k], r))


def test_apply_A_and_solve_pressure_parity():
    c = I.config(0)
    st = I.initial_state(c)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(st["p"].shape)
    g = tcf.Grid(c)
    g.set_state(st)
    Ax = host(dict(y=g.apply_A(torch.from_numpy(x))))["y"]
    assert rel(Ax, O.apply_A(c, st["alpha"], x)) <= 1e-13
    b = rng.standard_normal(st["p"].shape)
    p, status, info = g.solve_pressure(torch.from_numpy(b))
    p = host(dict(p=p))["p"]
    g.close()
    po, sto, _ = O.solve_pressure(c, st["alpha"], b, rtol=1e-13)
    assert status == 0 and sto == 0
    assert info["p_relres"] <= 1e-13
    assert rel(p, po) <= 1e-10, rel(p, po)


@pytest.mark.parametrize("nsteps,tol", [(1, 1e-10), (100, 1e-8)])
def test_full_step_2d_droplet(nsteps, tol):
    c = I.config(0)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], nsteps)
    o, oinf, _ = O.step(c, st, 0.0, c["dt"], nsteps)
    assert info["status"] == 0, info
    e = field_errors(g, o)
    assert max(e.values()) <= tol, e
    assert info["div_rel"] <= 1e-12
    assert abs(info["sum_alpha"] - st["alpha"].sum()) <= 1e-13 * nsteps * st["alpha"].sum()


def test_full_step_2d_ragged_perturbed():
    c = I.custom(I.config(1), nx=100, ny=72)
    c["h"] = 1.0 / 100
    c["normal_eps"] = 1e-6 / c["h"]
    st = I.initial_state(c)
    g, info = gpu_run(c, st, 2e-5, 3)
    o, _, _ = O.step(c, st, 0.0, 2e-5, 3)
    e = field_errors(g, o)
    assert max(e.values()) <= 1e-10, e


def test_full_step_3d_droplet_reduced():
    c = I.custom(I.config(3), nx=48, ny=48, nz=48)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], 3)
    o, _, _ = O.step(c, st, 0.0, c["dt"], 3)
    e = field_errors(g, o)
    assert max(e.values()) <= 1e-10, e


def test_full_step_3d_droplet_96():
    c = I.config(3)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], 1)
    o, _, _ = O.step(c, st, 0.0, c["dt"], 1)
    e = field_errors(g, o)
    assert max(e.values()) <= 1e-10, e


def test_full_step_meltpool_fp64():
    c = I.config(2)
    c["p_rtol"] = 1e-13
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], 2, precision=0)
    o, _, _ = O.step(c, st, 0.0, c["dt"], 2, rtol=1e-13)
    assert info["status"] == 0, info
    e = field_errors(g, o)
    assert max(e.values()) <= 1e-9, e


def test_full_step_meltpool_fp32_refined():
    """FP32 stencils and inner solve, FP64 refinement residual: divergence
    residual <= 1e-8, per-field error against the FP64 oracle reported."""
    c = I.config(2)
    c["p_rtol"] = 1e-10
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], 1, precision=1)
    o, _, _ = O.step(c, st, 0.0, c["dt"], 1, rtol=1e-13)
    assert info["status"] == 0, info
    assert info["p_relres"] <= 1e-10 and info["div_rel"] <= 1e-8, info
    e = field_errors(g, o)
    print("fp32-refined per-field rel. L2 vs FP64 oracle:", e, flush=True)
    assert e["alpha"] <= 1e-6 and e["T"] <= 1e-6, e
    assert max(e.values()) <= 1e-4, e


def test_full_step_fp32_refined_single_level():
    """FP32 refinement on grids whose hierarchy has one level (an odd
    extent): the inner right-hand side is then scaled in a pass of its own
    instead of by the first multigrid sweep.  One step of each against the
    FP64 oracle, to the bar of the multigrid case."""
    for c in (I.custom(I.config(2), nx=18, ny=13, nz=10), I.custom(I.config(0), nx=33, ny=20)):
        c["p_rtol"] = 1e-10
        c["p_maxit"] = 1000
        st = I.initial_state(c)
        g, info = gpu_run(c, st, c["dt"], 1, precision=1)
        o, _, _ = O.step(c, st, 0.0, c["dt"], 1, rtol=1e-13)
        assert info["status"] == 0, info
        assert info["p_relres"] <= 1e-10 and info["div_rel"] <= 1e-8, info
        e = field_errors(g, o)
        print("fp32-refined single-level rel. L2 vs FP64 oracle:", e, flush=True)
        assert e["alpha"] <= 1e-6 and e["T"] <= 1e-6, e
        assert max(e.values()) <= 1e-4, e


def test_deterministic_and_restart_bitwise():
    c = I.config(0)
    st = I.initial_state(c)
    a, _ = gpu_run(c, st, c["dt"], 4)
    b, _ = gpu_run(c, st, c["dt"], 4)
    for k in ("alpha", "T", "u", "v", "p"):
        assert np.array_equal(a[k], b[k]), k
    h1, _ = gpu_run(c, st, c["dt"], 2)
    h2, _ = gpu_run(c, h1, c["dt"], 2, t=2 * c["dt"])
    for k in ("alpha", "T", "u", "v", "p"):
        assert np.array_equal(a[k], h2[k]), k


def test_degenerate_cases():
    c = I.custom(I.config(0), nx=4, ny=4)
    st = I.initial_state(c)
    st["alpha"][:] = 0.25
    st["T"][:] = 0.0
    c["T_bc"] = [0] * 6
    g, info = gpu_run(c, st, 1e-4, 2)
    assert info["status"] == 0
    assert np.all(g["u"] == 0) and np.all(g["v"] == 0) and np.all(g["p"] == 0)
    assert np.all(g["alpha"] == 0.25)
    # nsteps = 0 leaves everything untouched
    c0 = I.config(0)
    s0 = I.initial_state(c0)
    g0, _ = gpu_run(c0, s0, 1e-4, 0)
    assert np.array_equal(g0["alpha"], s0["alpha"]) and g0["t"] == 0.0


def test_error_paths_on_device():
    c = I.config(0)
    st = I.initial_state(c)
    st["alpha"][0, 10, 10] = np.nan
    g = tcf.Grid(c)
    g.set_state(st)
    r = g.step(c["dt"], 1, check=False)
    assert r["status"] == tcf.TCF_E_NONFINITE
    g.close()
    c2 = dict(I.config(0), p_maxit=1)
    g2 = tcf.Grid(c2)
    g2.set_state(I.initial_state(c2))
    r2 = g2.step(c2["dt"], 1, check=False)
    assert r2["status"] == tcf.TCF_E_NOT_CONVERGED
    g2.close()
    # the step adjoint refuses a transport-only grid and NULL stage pointers
    c3 = I.config(0)
    g3 = tcf.Grid(c3, precision=0, flags=tcf.TCF_WITH_ADJOINT | tcf.TCF_TRANSPORT_ONLY)
    st3 = I.initial_state(c3)
    g3.set_state(st3)
    sbar = torch.zeros((), dtype=torch.float64, device="cuda")
    dev3 = {k: (None if v is None else torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda"))
            for k, v in st3.items() if k in ("alpha", "T", "u", "v", "w", "p")}
    lam = {k: (None if v is None else torch.zeros_like(v)) for k, v in dev3.items() if k != "p"}
    with pytest.raises(tcf.TcfError) as ei:
        g3.step_backward(0.0, c3["dt"], dev3, lam, sbar)
    assert ei.value.status == tcf.TCF_E_INVALID
    assert tcf.load().tcf_step_keep(g3.h, c3["dt"], None, None) == tcf.TCF_E_INVALID
    g3.close()


def test_full_size_meltpool_256_properties():
    """256^3 (the benchmark workload): one FP32-refined step; properties that
    hold at any size (finite fields, FP64 divergence residual, alpha sum)."""
    c = I.config(4)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], 1, precision=1)
    assert info["status"] == 0 and info["nonfinite"] == 0, info
    assert info["p_relres"] <= c["p_rtol"] and info["div_rel"] <= 1e-8, info
    s0 = st["alpha"].sum()
    assert abs(info["sum_alpha"] - s0) <= 1e-6 * s0


def test_full_size_meltpool_256_matches_oracle():
    """256^3 in the benchmark's configuration (FP32 stencils and inner solve,
    FP64 refinement to rtol 1e-8): one step against the FP64 oracle solved to
    1e-12, every field of the whole grid.  alpha and T are held to 1e-6.  The
    velocity is the small remainder of a balanced surface-tension force and
    moves by ~1e-5 when alpha moves by FP32 rounding alone (measured on the
    oracle by test_velocity_sensitivity_to_alpha_rounding), so u, v, w are
    held to 1e-4 and p to 2e-5 (one step here: u, v, w ~1-2e-5, p ~3e-6)."""
    c = dict(I.config(4), p_rtol=1e-8)
    st = I.initial_state(c)
    g, info = gpu_run(c, st, c["dt"], 1, precision=1)
    assert info["status"] == 0, info
    print("[oracle] 256^3 one step", flush=True)
    o, _, status = O.step(c, st, 0.0, c["dt"], 1, rtol=1e-12)
    assert status == 0
    e = field_errors(g, o)
    print("[errors]", e, flush=True)
    for k in ("alpha", "T"):
        assert e[k] <= 1e-6, e
    for k in ("u", "v", "w"):
        assert e[k] <= 1e-4, e
    assert e["p"] <= 2e-5, e
    assert info["div_rel"] <= 1e-8, info


def test_extrapolated_pressure_guess_agrees_and_saves_iterations():
    """The extrapolated initial guess (order 1: 2 p^n - p^(n-1); order 2:
    3 p^n - 3 p^(n-1) + p^(n-2)) changes only the iteration count: over 10
    FP64 steps of the 2D droplet and of a 64 x 32 x 32 melt pool the fields
    agree with the last-pressure guess to the solve tolerance, and the CG
    iterations do not increase."""
    for c0, dt in ((I.config(0), None), (I.custom(I.config(2), nx=64, ny=32, nz=32), 1e-8)):
        c0 = dict(c0, p_rtol=1e-11)
        dt = dt or c0["dt"]
        st = I.initial_state(c0)
        res = {}
        for ex in (0, 1, 2):
            c = dict(c0, p_extrapolate=ex)
            print(f"[gpu] extrapolate={ex} {c['nx']}x{c['ny']}x{c['nz']}", flush=True)
            g = tcf.Grid(c, precision=0)
            g.set_state(st)
            iters = 0
            for _ in range(10):
                iters += g.step(dt, 1)["cg_iters"]
            res[ex] = (host(g.get_fields()), iters)
            g.close()
        print("[iters]", {k: v[1] for k, v in res.items()}, flush=True)
        for ex in (1, 2):
            e = field_errors(res[ex][0], res[0][0])
            assert max(e.values()) <= 1e-8, (ex, e)
            assert res[ex][1] <= res[0][1], (ex, res[0][1], res[ex][1])


def test_restart_with_second_order_history_bitwise():
    """A run restarted from get_fields (with the two previous pressures of
    the order-2 guess) repeats the uninterrupted run bitwise."""
    c = dict(I.config(0), p_extrapolate=2)
    st = I.initial_state(c)
    a, _ = gpu_run(c, st, c["dt"], 5)
    h1, _ = gpu_run(c, st, c["dt"], 3)
    assert h1["p_held"] == 2
    h2, _ = gpu_run(c, h1, c["dt"], 2, t=3 * c["dt"])
    for k in ("alpha", "T", "u", "v", "p"):
        assert np.array_equal(a[k], h2[k]), k


def test_pressure_history_entry_points():
    """The history of the extrapolated guess round-trips through the C ABI,
    tcf_set_fields clears it, and held outside 0..p_extrapolate or a missing
    pointer is refused."""
    import ctypes as C
    c = dict(I.config(0), p_extrapolate=2)
    st = I.initial_state(c)
    g = tcf.Grid(c, precision=0)
    g.set_state(st)
    assert g.get_fields()["p_held"] == 0
    g.step(c["dt"], 3)
    f = g.get_fields()
    assert f["p_held"] == 2
    lib = tcf.load()
    p1 = torch.rand(g.shapes["cell"], dtype=torch.float64, device="cuda")
    p2 = torch.rand(g.shapes["cell"], dtype=torch.float64, device="cuda")
    assert lib.tcf_set_pressure_history(g.h, C.c_void_p(p1.data_ptr()), C.c_void_p(p2.data_ptr()), 2) == tcf.TCF_OK
    h = g.get_fields()
    torch.cuda.synchronize()
    assert h["p_held"] == 2 and torch.equal(h["p_prev"], p1) and torch.equal(h["p_prev2"], p2)
    assert lib.tcf_set_pressure_history(g.h, C.c_void_p(p1.data_ptr()), None, 2) == tcf.TCF_E_INVALID
    assert lib.tcf_set_pressure_history(g.h, None, None, 3) == tcf.TCF_E_INVALID
    assert lib.tcf_set_pressure_history(g.h, None, None, 0) == tcf.TCF_OK
    assert g.get_fields()["p_held"] == 0
    g.step(c["dt"], 1)
    assert g.get_fields()["p_held"] == 1
    g.set_state(st)
    assert g.get_fields()["p_held"] == 0
    g.close()
    g = tcf.Grid(dict(c, p_extrapolate=0), precision=0)
    held = C.c_int(-1)
    assert lib.tcf_get_pressure_history(g.h, None, None, C.byref(held)) == tcf.TCF_E_STATE
    g.close()
