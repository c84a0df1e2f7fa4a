"""Pins of the oracle's N-phase extension (eq. 1 for every phase j of several
in one domain; the paper names arbitrarily many phases and the solid /
liquid / gas case of the powder-bed experiment, without giving mixture laws
or pairwise surface tension).

Reading under test: phase 1 is the background with alpha_1 = 1 - sum of
the others; material laws are linear in each clamped fraction relative to
phase 1; each pair of phases i < j has its own surface tension sigma_ij(T)
acting through the pair gradient g_ij = alpha_i grad alpha_j - alpha_j grad
alpha_i with eqs. 4-7; the face force sums the pairs.

The pins tie it to the already pinned two-phase model and to closed forms:
  - a third phase of zero fraction changes nothing;
  - a relabelled two-phase problem (the drop carried as phase 3) is the
    two-phase step;
  - two well-separated drops of two phases with identical properties and
    tensions are the two-phase step of their union;
  - flat layers with uniform T stay at rest;
  - the summed Marangoni force of layered interfaces equals, interface by
    interface, the pair's slope times the closed-form sum of the discrete
    gradient (pair slopes land on the right interfaces);
  - every phase's volume is conserved.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2209_09671_amd import inputs as I

FIELDS = ("alpha", "T", "u", "v", "p")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_absent_third_phase_changes_nothing():
    c = I.config(0)
    st = I.initial_state(c)
    ref, _, s0 = O.step(c, st, 0.0, c["dt"], 5)
    cn = I.droplet_phases(c, "absent")
    out, _, s1 = O.step(cn, I.phase_state(cn), 0.0, c["dt"], 5)
    assert s0 == s1 == 0
    for k in FIELDS:
        assert rel(out[k], ref[k]) <= 1e-12, k
    assert np.array_equal(out["alpha3"], np.zeros_like(out["alpha3"]))


def test_relabelled_two_phase_problem():
    """Phase 2 absent and the drop carried as phase 3 with phase 2's
    materials and tension as pair (1,3): the two-phase step (pins the pair
    table slots and the phase-3 material values)."""
    c = I.config(0)
    st = I.initial_state(c)
    ref, _, _ = O.step(c, st, 0.0, c["dt"], 5)
    ph3 = dict(rho=c["rho2"], mu=c["mu2"], rhocp=c["rhocp2"], **{"lambda": c["lambda2"]})
    cn = I.with_phases(c, "absent", [ph3], {(1, 2): 0.3, (1, 3): c["sigma0"], (2, 3): 0.2},
                       {(1, 2): 0.05, (1, 3): c["dsigma_dT"]})
    s = dict(st, alpha=np.zeros_like(st["alpha"]), alpha3=st["alpha"].copy())
    out, _, status = O.step(cn, s, 0.0, c["dt"], 5)
    assert status == 0
    for k in ("T", "u", "v", "p"):
        assert rel(out[k], ref[k]) <= 1e-12, k
    assert rel(out["alpha3"], ref["alpha"]) <= 1e-12
    assert np.array_equal(out["alpha"], np.zeros_like(out["alpha"]))


def test_separated_drops_of_identical_phases_are_their_union():
    """Drops of phases 2 and 3 whose edges are 38 cells apart, identical
    materials and (1,2), (1,3) tensions: the same step as the two-phase model
    with alpha = alpha_2 + alpha_3 (the (2,3) tension never acts)."""
    c = I.custom(I.config(0), nx=128, ny=128)
    same = dict(rho=c["rho2"], mu=c["mu2"], rhocp=c["rhocp2"], **{"lambda": c["lambda2"]})
    cn = I.with_phases(c, "two_drops", [same], {(1, 2): 1.0, (1, 3): 1.0, (2, 3): 0.7},
                       {(1, 2): -0.1, (1, 3): -0.1})
    st = I.phase_state(cn)
    out, _, s1 = O.step(cn, st, 0.0, 5e-5, 10)
    union = dict(st, alpha=st["alpha"] + st["alpha3"])
    union.pop("alpha3")
    ref, _, s0 = O.step(c, union, 0.0, 5e-5, 10)
    assert s0 == s1 == 0
    for k in ("T", "u", "v", "p"):
        assert rel(out[k], ref[k]) <= 1e-11, k
    assert rel(out["alpha"] + out["alpha3"], ref["alpha"]) <= 1e-12
    assert np.abs(ref["u"]).max() > 0


def test_flat_layers_at_uniform_temperature_stay_at_rest():
    """Three flat layers (3 | 2 | 1 upward), uniform T: every pair force is a
    function of the vertical coordinate along it, balanced by the pressure;
    u stays 0 to the solver tolerance and the layers do not move."""
    c = I.custom(I.config(0), nx=48, ny=48)
    c["T_bc"] = [0] * 6
    cn = I.droplet_phases(c, "layers")
    st = I.phase_state(cn)
    st["T"] = np.full_like(st["T"], 0.3)
    us, vs, _ = O.predictor(cn, c["dt"], st["alpha"], st["T"], st["u"], st["v"], alpha3=st["alpha3"])
    out, info, status = O.step(cn, st, 0.0, c["dt"], 1, rtol=1e-12)
    assert status == 0
    assert np.abs(vs).max() > 0
    assert np.abs(out["u"]).max() <= 1e-10 * np.abs(vs).max()
    assert np.abs(out["v"]).max() <= 1e-10 * np.abs(vs).max()
    assert rel(out["alpha"], st["alpha"]) <= 1e-14 and rel(out["alpha3"], st["alpha3"]) <= 1e-14


def test_marangoni_force_per_interface():
    """Layers with T = x: the tangential force of pair (i, j) is its slope
    s_ij times the summed discrete gradient of T ((n - 1.5) rows, the wall
    rows' even ghosts halving it) times the pair's integrated delta; the two
    real interfaces integrate to one, the absent (1,3) pair to nothing."""
    n = 64
    c = I.custom(I.config(0), nx=n, ny=n)
    c["T_bc"] = [0] * 6
    cn = I.droplet_phases(c, "layers")
    st = I.phase_state(cn)
    h = c["h"]
    x = (np.arange(n) + 0.5) * h
    T = np.ascontiguousarray(np.broadcast_to(x[None, :], (n, n)).reshape(1, n, n))
    g = O.geometry_n(cn, st["alpha"], st["alpha3"], T)
    rows = {p: h * g["delta"][p][0, :, 0].sum() for p in g["delta"]}
    assert rows[(1, 2)] == pytest.approx(1.0, abs=1e-4)
    assert rows[(2, 3)] == pytest.approx(1.0, abs=1e-4)
    assert abs(rows[(1, 3)]) <= 1e-12
    us, _, _ = O.predictor(cn, 1.0, st["alpha"], T, np.zeros((1, n, n + 1)), np.zeros((1, n + 1, n)),
                           alpha3=st["alpha3"])
    rho = (cn["rho1"] + np.clip(st["alpha"], 0, 1) * (cn["rho2"] - cn["rho1"])
           + np.clip(st["alpha3"], 0, 1) * (cn["phases"][0]["rho"] - cn["rho1"]))
    fx = us[0, :, 1:-1] * 0.5 * (rho[0, :, 1:] + rho[0, :, :-1])  # face force (dt = 1, u = 0)
    slope = dict(zip(I.PAIRS, cn["pair_dsigma_dT"]))
    expect = sum(slope[p] * (n - 1.5) * h * rows[p] for p in rows)
    assert fx.sum() * h * h == pytest.approx(expect, rel=1e-10)
    assert slope[(1, 2)] != slope[(2, 3)]


def test_every_phase_is_conserved():
    """The lens (a phase-3 drop on a phase-2 layer, with triple junctions)
    over 20 steps: the volume of each phase is constant to round-off."""
    c = I.config(0)
    cn = I.droplet_phases(c, "lens")
    st = I.phase_state(cn)
    out, info, status = O.step(cn, st, 0.0, c["dt"], 20)
    assert status == 0
    for k in ("alpha", "alpha3"):
        assert abs(out[k].sum() - st[k].sum()) <= 1e-12 * st[k].sum(), k
    assert not np.array_equal(out["alpha3"], st["alpha3"])


def test_absent_fourth_phase_changes_nothing():
    """Four phases with phase 4 of zero fraction: the three-phase step."""
    c = I.config(0)
    c3 = I.droplet_phases(c, "lens")
    c4 = I.droplet_phases4(c, "absent4")
    for q in ((1, 2), (1, 3), (2, 3)):  # same tensions for the three pairs that act
        k = I.PAIRS.index(q)
        c4["pair_sigma0"][k], c4["pair_dsigma_dT"][k] = c3["pair_sigma0"][k], c3["pair_dsigma_dT"][k]
    s3 = I.phase_state(c3)
    s4 = I.phase_state(c4)
    ref, _, st3 = O.step(c3, s3, 0.0, c["dt"], 5)
    out, _, st4 = O.step(c4, s4, 0.0, c["dt"], 5)
    assert st3 == st4 == 0
    for k in FIELDS + ("alpha3",):
        assert rel(out[k], ref[k]) <= 1e-12, k
    assert np.array_equal(out["alpha4"], np.zeros_like(out["alpha4"]))


def test_four_flat_layers_at_uniform_temperature_stay_at_rest():
    c = I.custom(I.config(0), nx=48, ny=48)
    c["T_bc"] = [0] * 6
    cn = I.droplet_phases4(c, "layers4")
    st = I.phase_state(cn)
    st["T"] = np.full_like(st["T"], 0.3)
    _, vs, _ = O.predictor(cn, c["dt"], st["alpha"], st["T"], st["u"], st["v"], alpha3=st["alpha3"],
                           alpha4=st["alpha4"])
    out, info, status = O.step(cn, st, 0.0, c["dt"], 1, rtol=1e-12)
    assert status == 0
    assert np.abs(vs).max() > 0
    assert np.abs(out["u"]).max() <= 1e-10 * np.abs(vs).max()
    assert np.abs(out["v"]).max() <= 1e-10 * np.abs(vs).max()


def test_undefined_combinations_are_refused():
    c = I.droplet_phases(I.config(0), "lens")
    st = I.phase_state(c)
    for bad in (dict(c, integrator=1), dict(c, species=1)):
        _, _, status = O.step(bad, st, 0.0, c["dt"], 1)
        assert status == 5
    s2 = dict(st)
    s2.pop("alpha3")
    _, _, status = O.step(c, s2, 0.0, c["dt"], 1)
    assert status == 5
