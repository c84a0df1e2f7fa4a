"""Pins of the oracle's time-accurate integrator (integrator 1: SSP-RK3 over
the whole state with a projection in every stage).

The paper leaves its time integrator unstated (Section "Implementation"
builds on an OpenFOAM solver without describing the coupling); the default
step splits the transport from one forward-Euler momentum predictor and one
projection.  The pins tie the variant to facts outside its own code:
  - without momentum and heat source it is the default transport, bitwise;
  - it converges at third order in time (the order of the Shu-Osher scheme)
    on a smooth single-phase flow, on the thermocapillary droplet (variable
    density, CSF and Marangoni forces) and on a moving heat source, where
    the default step converges at first order;
  - every stage is projected (divergence ratio at the solver tolerance);
  - the balanced-force null case still gives u = 0 and p = C alpha.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2209_09671_amd import inputs as I


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def run(c, integ, dt, t_end, st):
    n = int(round(t_end / dt))
    s, info, status = O.step(dict(c, integrator=integ), st, 0.0, dt, n, rtol=1e-13)
    assert status == 0, status
    return s


def orders(c, st, t_end, dts, integ, keys):
    """Observed orders of the time error at t_end for the steps dts (halving),
    against a run at dts[-1] / 8 of the same integrator."""
    ref = run(c, integ, dts[-1] / 8, t_end, st)
    errs = [{k: rel(run(c, integ, dt, t_end, st)[k], ref[k]) for k in keys} for dt in dts]
    return {k: [float(np.log2(errs[i][k] / errs[i + 1][k])) for i in range(len(dts) - 1)] for k in keys}


def test_without_momentum_and_heat_source_it_is_the_default_transport():
    """Frozen velocity (transport only), no heat source, with a species: the
    three stages are the default SSP-RK3 transport, so alpha, T and c agree
    bitwise."""
    c = I.with_species(I.custom(I.config(0), nx=48, ny=48), -0.3, "blob")
    assert c["q_power"] == 0.0
    st = I.initial_state(c)
    st["c"] = I.species_field(c)
    st["u"], st["v"] = I.stream_velocity(c, 1.0)[:2]
    r0, _, _ = O.step(dict(c, integrator=0), st, 0.0, 2e-3, 5, flags=O.F_TRANSPORT_ONLY)
    r1, _, _ = O.step(dict(c, integrator=1), st, 0.0, 2e-3, 5, flags=O.F_TRANSPORT_ONLY)
    for k in ("alpha", "T", "c", "u", "v"):
        assert np.array_equal(r0[k], r1[k]), k
    assert not np.array_equal(r1["alpha"], st["alpha"])


def test_third_order_single_phase_smooth_flow():
    """Uniform density and viscosity, no surface tension, a smooth
    divergence-free start that vanishes at the walls: third order in u."""
    c = I.custom(I.config(0), nx=32, ny=32)
    c.update(rho1=1.0, rho2=1.0, mu1=0.01, mu2=0.01, sigma0=0.0, dsigma_dT=0.0)
    st = I.initial_state(c)
    st["u"], st["v"] = I.stream_velocity(c, 1.0)[:2]
    o1 = orders(c, st, 0.04, [0.004, 0.002, 0.001], 1, ("u", "alpha", "T"))
    o0 = orders(c, st, 0.04, [0.004, 0.002, 0.001], 0, ("u",))
    for k, v in o1.items():
        assert min(v) >= 2.8, (k, v)
    assert all(0.8 <= x <= 1.3 for x in o0["u"]), o0


def test_third_order_thermocapillary_droplet():
    """The 2D droplet (density ratio 2, CSF and thermal Marangoni force from
    rest): third order in u, alpha and T; the default split step is first
    order on the same case (its O(dt) splitting error)."""
    c = I.custom(I.config(0), nx=32, ny=32)
    st = I.initial_state(c)
    dts = [0.001, 0.0005, 0.00025]
    o1 = orders(c, st, 0.008, dts, 1, ("u", "alpha", "T"))
    o0 = orders(c, st, 0.008, dts, 0, ("u", "alpha", "T"))
    for k, v in o1.items():
        assert min(v) >= 2.8, (k, v)
    for k, v in o0.items():
        assert all(0.8 <= x <= 1.3 for x in v), (k, v)


def test_third_order_moving_heat_source():
    """A Gaussian flux moving along x heats a flat interface: T converges at
    third order only if every stage takes the source at its own stage time
    (t, t + dt, t + dt/2)."""
    c = I.custom(I.config(0), nx=32, ny=32)
    c.update(q_power=5.0, q_radius=0.1, q_x0=0.3, q_y0=0.5, q_vx=5.0, q_vy=0.0, sigma0=0.0, dsigma_dT=0.0)
    st = I.initial_state(c)
    o1 = orders(c, st, 0.02, [0.002, 0.001, 0.0005], 1, ("T",))
    assert min(o1["T"]) >= 2.8, o1


def test_every_stage_is_projected():
    """After a step the divergence ratio of the last stage is at the solver
    tolerance, and the new velocity is discretely divergence-free relative to
    the forcing it received."""
    c = I.config(0)
    st = I.initial_state(c)
    s, info, status = O.step(dict(c, integrator=1), st, 0.0, c["dt"], 3, rtol=1e-12)
    assert status == 0
    assert info["div_rel"] <= 1e-11
    D = O.divergence(c, s["u"], s["v"])
    assert np.linalg.norm(D) * c["h"] <= 1e-9 * np.abs(s["u"]).max()


def test_balanced_force_null_case():
    """sigma*kappa forced to a constant C, no Marangoni term: each stage's
    face force C grad(alpha) is balanced by its projection with the same
    density, so u stays 0 and p = C alpha + const."""
    c = I.config(0)
    c["dsigma_dT"] = 0.0
    st = I.initial_state(c)
    C = 3.7
    s, info, stt = O.step(dict(c, integrator=1), st, 0.0, c["dt"], 2, flags=O.F_CONST_SIGKAP,
                          sigkap_const=C, rtol=1e-14)
    ref = C * st["alpha"]
    assert rel(s["p"], ref - ref.mean()) < 1e-11
    assert np.abs(np.concatenate([s["u"].ravel(), s["v"].ravel()])).max() < 1e-11
    assert rel(s["alpha"], st["alpha"]) < 1e-12  # carried by a velocity at the solver tolerance
