"""Pins of the oracle's solutal-Marangoni extension (species field c with
sigma = sigma0 + dsigma_dT (T - T0) + dsigma_dc (c - c0); eq. 5 writes the
surface-tension gradient as the chain rule over temperature and
concentration, Section "Theory"; in-situ alloying is the motivating case).

Every pin ties the new arithmetic to something fixed outside it: reductions
to the already pinned thermal path (c taking the role of T, or of alpha),
a conservation invariant, and the closed-form total tangential force on a
flat interface.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2209_09671_amd import inputs as I


def neumann_droplet(n=48):
    """2D droplet with adiabatic walls and no conduction: T is then carried
    exactly like a passive scalar with even wall ghosts."""
    c = I.custom(I.config(0), nx=n, ny=n)
    c["T_bc"] = [0] * 6
    c["lambda1"] = c["lambda2"] = 0.0
    return c


def test_zero_slope_species_leaves_the_step_unchanged():
    """dsigma_dc = 0: carrying a species changes nothing else, bitwise."""
    c = I.config(0)
    st = I.initial_state(c)
    ref, _, _ = O.step(c, st, 0.0, c["dt"], 5)
    cs = I.with_species(c, 0.0, "blob")
    st2 = dict(st, c=I.species_field(cs))
    out, _, _ = O.step(cs, st2, 0.0, c["dt"], 5)
    for k in ("alpha", "T", "u", "v", "p"):
        assert np.array_equal(out[k], ref[k]), k


def test_species_equal_to_temperature_reproduces_thermal_marangoni():
    """With c := T, dsigma_dc := dsigma_dT and dsigma_dT := 0 (c0 = T0) the
    surface-tension field is the same function of space, so the step is the
    thermal one bitwise, and c stays equal to T (both are carried by the same
    WENO5 flux with even ghosts when there is no conduction)."""
    c = neumann_droplet()
    st = I.initial_state(c)
    ref, _, _ = O.step(c, st, 0.0, c["dt"], 6)
    cs = I.with_species(c, c["dsigma_dT"], c0=c["T0"])
    cs["dsigma_dT"] = 0.0
    out, _, _ = O.step(cs, dict(st, c=st["T"].copy()), 0.0, c["dt"], 6)
    for k in ("alpha", "T", "u", "v", "p"):
        assert np.array_equal(out[k], ref[k]), k
    assert np.array_equal(out["c"], out["T"])
    assert np.abs(ref["u"]).max() > 0  # the pin is not vacuous


def test_species_equal_to_alpha_stays_equal_to_alpha():
    """A species field that starts as a copy of alpha is transported by the
    same operator (eq. 1) and stays bitwise equal to alpha; 3D case."""
    c = I.custom(I.config(3), nx=24, ny=24, nz=24)
    cs = I.with_species(c, -0.2, "alpha")
    st = I.initial_state(cs)
    out, _, _ = O.step(cs, dict(st, c=I.species_field(cs)), 0.0, c["dt"], 4)
    assert np.array_equal(out["c"], out["alpha"])
    assert not np.array_equal(out["alpha"], st["alpha"])


def test_species_is_conserved():
    """Telescoping fluxes and zero wall flux: sum(c) is constant to round-off."""
    cs = I.with_species(I.config(0), -0.3, "blob")
    st = I.initial_state(cs)
    cf = I.species_field(cs)
    out, _, _ = O.step(cs, dict(st, c=cf), 0.0, cs["dt"], 20)
    assert abs(out["c"].sum() - cf.sum()) <= 1e-13 * cf.sum()
    assert not np.array_equal(out["c"], cf)


def test_total_solutal_force_on_flat_interface():
    """Flat interface x = const with c = y and uniform T: the summed
    tangential (y) face force equals dsigma_dc * (the c range seen by the
    faces) * (h sum_x delta_s), in closed form for the discrete gradient with
    even wall ghosts; a concentration gradient along the normal gives no
    tangential force."""
    n = 64
    c = I.custom(I.config(0), nx=n, ny=n)
    c["T_bc"] = [0] * 6
    cs = I.with_species(c, -0.7)
    cs["dsigma_dT"] = 0.0
    h = c["h"]
    x = (np.arange(n) + 0.5) * h
    al = 0.5 * (1 - np.tanh((x - 0.503) / (1.5 * h)))
    alpha = np.ascontiguousarray(np.broadcast_to(al[None, :], (n, n)).reshape(1, n, n))
    T = np.full((1, n, n), 0.3)
    cy = np.ascontiguousarray(np.broadcast_to(x[:, None], (n, n)).reshape(1, n, n))  # c = y
    g = O.geometry(cs, alpha, T, cfield=cy)
    row = h * g["delta_s"][0, 0, :].sum()
    assert row == pytest.approx(1.0, abs=1e-4)
    us, vs, _ = O.predictor(cs, 1.0, alpha, T, np.zeros((1, n, n + 1)), np.zeros((1, n + 1, n)), cfield=cy)
    rho = c["rho1"] + np.clip(alpha, 0, 1) * (c["rho2"] - c["rho1"])
    fy = vs[0, 1:-1, :] * 0.5 * (rho[0, 1:, :] + rho[0, :-1, :])   # face force (dt = 1, u = 0)
    total = fy.sum() * h * h
    # the central gradient of c is 1 in every row but the two wall rows, where
    # the even ghost (no flux of c through the wall) halves it; the face force
    # averages two rows, so the n-1 interior faces sum to (n - 1.5) rows
    assert total == pytest.approx(cs["dsigma_dc"] * (n - 1.5) * h * row, rel=1e-10)
    # c along the interface normal (x): no tangential (y) Marangoni component
    cx = np.ascontiguousarray(np.broadcast_to(x[None, :], (n, n)).reshape(1, n, n))
    g2 = O.geometry(cs, alpha, T, cfield=cx)
    assert np.abs(g2["M"][:, 1]).max() == 0.0
    assert np.abs(g2["M"][:, 0]).max() <= 0.5 * abs(cs["dsigma_dc"]) * cs["normal_eps"]


def test_solutal_migration_direction():
    """A drop in a concentration gradient with dsigma_dc < 0 migrates toward
    higher c (low surface tension pulls), and reverses with the sign."""
    c = I.config(0)
    c["dsigma_dT"] = 0.0
    cs = I.with_species(c, -0.3, "linear_x")
    st = I.initial_state(cs)
    cf = I.species_field(cs)
    s, _, _ = O.step(cs, dict(st, c=cf), 0.0, c["dt"], 30)
    uc = 0.5 * (s["u"][:, :, 1:] + s["u"][:, :, :-1])
    assert (s["alpha"] * uc).sum() > 0
    cs2 = dict(cs, dsigma_dc=0.3)
    s2, _, _ = O.step(cs2, dict(st, c=cf), 0.0, c["dt"], 30)
    uc2 = 0.5 * (s2["u"][:, :, 1:] + s2["u"][:, :, :-1])
    assert (s2["alpha"] * uc2).sum() < 0
