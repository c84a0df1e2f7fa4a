"""Seeded synthetic inputs: parameter sheets and initial fields.

This module is shared by the GPU path, its tests, the benchmark and the
oracle's tests.  It holds no arithmetic of the method itself: it only builds
parameter dictionaries and initial states (smoothed indicator profiles, a
temperature ramp, a prescribed divergence-free velocity for transport-only
checks).

The workloads stand in for the paper's two experiments (Section "Numerical
experiments"): the thermocapillary droplet of Ma and Bothe (Table I) and the
laser powder-bed single track (Table II).  The case files of those experiments
are not available, so every field here is synthetic and seeded.

Array layout (both solvers): C order with shape (nz, ny, nx) for cell fields
(x fastest), (nz, ny, nx+1) for x-face velocity, (nz, ny+1, nx) for y-face,
(nz+1, ny, nx) for z-face.  In 2D nz == 1 and there is no z-face array.
Phase 1 (alpha = 0) is the ambient fluid, phase 2 (alpha = 1) the drop/metal.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Wall order for the temperature boundary arrays: -x, +x, -y, +y, -z, +z.
NEUMANN, DIRICHLET = 0, 1

_DEFAULTS = dict(
    precision=0,          # 0 = FP64, 1 = FP32 stencils + FP64 refinement
    flags=0,
    weno_eps=1e-6,
    p_rtol=1e-13,
    p_maxit=200,
    inner_rtol=1e-5,
    refine_maxit=30,
    mg_levels=0,          # 0 = as many as the grid allows
    mg_nu=2,
    p_extrapolate=2,      # pressure guess 3 p^n - 3 p^(n-1) + p^(n-2) (lower orders until held)
    q_power=0.0, q_radius=1.0, q_x0=0.0, q_y0=0.0, q_vx=0.0, q_vy=0.0,
)


def _droplet_2d(n, steps, dt, name):
    h = 1.0 / n
    c = dict(_DEFAULTS)
    c.update(name=name, dim=2, nx=n, ny=n, nz=1, h=h,
             rho1=1.0, rho2=2.0, mu1=0.01, mu2=0.02,
             rhocp1=1.0, rhocp2=4.0, lambda1=1e-3, lambda2=2e-3,
             sigma0=1.0, dsigma_dT=-0.1, T0=0.0,
             T_bc=[NEUMANN, NEUMANN, DIRICHLET, DIRICHLET, NEUMANN, NEUMANN],
             T_wall=[0.0, 0.0, 0.0, 1.0, 0.0, 0.0],
             normal_eps=1e-6 / h, dt=dt, steps=steps)
    return c


def _meltpool_3d(nx, ny, nz, h, steps, dt, name, seed):
    c = dict(_DEFAULTS)
    lx, ly = nx * h, ny * h
    c.update(name=name, dim=3, nx=nx, ny=ny, nz=nz, h=h,
             rho1=1.0, rho2=7500.0, mu1=2e-5, mu2=5e-3,
             rhocp1=1900.0, rhocp2=7500.0 * 790.0, lambda1=0.02, lambda2=6.6,
             sigma0=1.908, dsigma_dT=-4e-4, T0=1700.0,
             T_bc=[NEUMANN] * 6, T_wall=[0.0] * 6,
             q_power=200.0, q_radius=40e-6, q_x0=lx / 4.0, q_y0=ly / 2.0,
             q_vx=0.5, q_vy=0.0,
             normal_eps=1e-6 / h, dt=dt, steps=steps, precision=1,
             p_rtol=1e-10, inner_rtol=1e-6, seed=seed)
    return c


def config(idx: int) -> dict:
    """Parameter sheet of workload ``idx`` (0..4); a fresh dict each call."""
    if idx == 0:
        c = _droplet_2d(64, 100, 1e-4, "droplet2d-64")
        c.update(drop_centre=[0.5, 0.4], drop_radius=0.2)
    elif idx == 1:
        c = _droplet_2d(512, 1000, 2e-5, "droplet2d-512-perturbed")
        c.update(drop_centre=[0.5, 0.4], drop_radius=0.2, perturb_seed=1,
                 perturb_amp=0.01)
    elif idx == 2:
        c = _meltpool_3d(128, 64, 64, 5e-6, 2000, 1e-8, "meltpool-128x64x64", 2)
    elif idx == 3:
        n = 96
        h = 1.0 / n
        c = dict(_DEFAULTS)
        c.update(name="droplet3d-96", dim=3, nx=n, ny=n, nz=n, h=h,
                 rho1=1.0, rho2=2.0, mu1=0.01, mu2=0.02,
                 rhocp1=1.0, rhocp2=4.0, lambda1=1e-3, lambda2=2e-3,
                 sigma0=1.0, dsigma_dT=-0.2, T0=0.0,
                 T_bc=[NEUMANN, NEUMANN, NEUMANN, NEUMANN, DIRICHLET, DIRICHLET],
                 T_wall=[0.0, 0.0, 0.0, 0.0, 0.0, 1.0],
                 normal_eps=1e-6 / h, dt=1e-4, steps=200,
                 drop_centre=[0.5, 0.5, 0.4], drop_radius=0.25,
                 checkpoint_every=20, target_seed=3)
    elif idx == 4:
        c = _meltpool_3d(256, 256, 256, 2.5e-6, 5000, 1e-8, "meltpool-256^3", 4)
        c.update(adjoint_steps=200, checkpoint_every=25)
    else:
        raise ValueError(f"no workload {idx}")
    c["index"] = idx
    return c


def custom(base: dict, **over) -> dict:
    """Copy of ``base`` with fields replaced (grid changes keep h = 1/nx
    for unit-box droplets unless h is given)."""
    c = copy.deepcopy(base)
    c.update(over)
    if ("nx" in over or "ny" in over or "nz" in over) and "h" not in over \
            and base.get("dim") and base.get("rho2", 0) < 100:
        c["h"] = 1.0 / c["nx"]
        c["normal_eps"] = 1e-6 / c["h"]
    return c


# ----------------------------------------------------------------------------
# geometry helpers
def cell_centres(c):
    h = c["h"]
    x = (np.arange(c["nx"]) + 0.5) * h
    y = (np.arange(c["ny"]) + 0.5) * h
    z = (np.arange(c["nz"]) + 0.5) * h
    return x, y, z


def shapes(c):
    nx, ny, nz = c["nx"], c["ny"], c["nz"]
    s = dict(cell=(nz, ny, nx), u=(nz, ny, nx + 1), v=(nz, ny + 1, nx))
    s["w"] = (nz + 1, ny, nx) if c["dim"] == 3 else None
    return s


def _smooth_step(signed_dist, width):
    """Indicator 1 on the positive side with a tanh edge of length scale width."""
    return 0.5 * (1.0 + np.tanh(signed_dist / width))


def _radius_perturbation(seed, amp, modes=range(2, 9)):
    """Fourier series in the polar angle, modes 2..8, scaled so that its
    maximum modulus over the angle is ``amp``; returns a callable."""
    rng = np.random.default_rng(seed)
    ms = np.array(list(modes))
    a = rng.standard_normal(len(ms))
    b = rng.standard_normal(len(ms))
    th = np.linspace(0.0, 2 * np.pi, 20001)
    raw = (a[:, None] * np.cos(ms[:, None] * th) + b[:, None] * np.sin(ms[:, None] * th)).sum(0)
    scale = amp / np.abs(raw).max()

    def f(theta):
        return scale * (a[:, None, None] * np.cos(ms[:, None, None] * theta)
                        + b[:, None, None] * np.sin(ms[:, None, None] * theta)).sum(0)
    return f


def _surface_roughness(seed, nx, ny, h, modes=range(2, 9)):
    """Seeded Fourier sum in x and y (modes 2..8 along each axis) sampled at
    cell centres, scaled to maximum modulus 1."""
    rng = np.random.default_rng(seed)
    lx, ly = nx * h, ny * h
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    r = np.zeros((ny, nx))
    for m in modes:
        a, b, cc, d = rng.standard_normal(4)
        r += (a * np.cos(2 * np.pi * m * x / lx) + b * np.sin(2 * np.pi * m * x / lx))[None, :]
        r += (cc * np.cos(2 * np.pi * m * y / ly) + d * np.sin(2 * np.pi * m * y / ly))[:, None]
    return r / np.abs(r).max()


def initial_state(c) -> dict:
    """Initial (alpha, T, u, v, w, p) of a workload as float64 numpy arrays."""
    s = shapes(c)
    h = c["h"]
    x, y, z = cell_centres(c)
    width = 1.5 * h
    if c["dim"] == 2:
        Y, X = np.meshgrid(y, x, indexing="ij")
        X, Y = X[None], Y[None]
    else:
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    if "drop_radius" in c:
        ctr = c["drop_centre"]
        dx, dy = X - ctr[0], Y - ctr[1]
        if c["dim"] == 2:
            r = np.hypot(dx, dy)
            R = c["drop_radius"] * np.ones_like(r)
            if c.get("perturb_seed") is not None:
                f = _radius_perturbation(c["perturb_seed"], c["perturb_amp"])
                R = c["drop_radius"] * (1.0 + f(np.arctan2(dy, dx)))
        else:
            r = np.sqrt(dx * dx + dy * dy + (Z - ctr[2]) ** 2)
            R = c["drop_radius"]
        alpha = _smooth_step(R - r, width)
        vert = Y if c["dim"] == 2 else Z
        T = np.array(vert, dtype=np.float64)       # T equals the vertical coordinate
    else:
        lz = c["nz"] * h
        zs = lz / 2.0 + h * _surface_roughness(c["seed"], c["nx"], c["ny"], h)
        alpha = _smooth_step(zs[None, :, :] - Z, width)
        T = np.full(s["cell"], c["T0"])
    st = dict(alpha=np.ascontiguousarray(alpha.reshape(s["cell"]), dtype=np.float64),
              T=np.ascontiguousarray(T.reshape(s["cell"]), dtype=np.float64),
              u=np.zeros(s["u"]), v=np.zeros(s["v"]),
              w=np.zeros(s["w"]) if s["w"] else None,
              p=np.zeros(s["cell"]))
    return st


def with_species(c, dsigma_dc, kind="linear_x", c0=0.0, seed=5) -> dict:
    """Config with a species field c (solutal Marangoni): sigma gains
    dsigma_dc (c - c0).  The field itself comes from species_field(c)."""
    out = dict(c)
    out.update(species=1, dsigma_dc=float(dsigma_dc), c0=float(c0), species_kind=kind, species_seed=seed)
    return out


def species_field(c) -> np.ndarray:
    """Initial species field of a config made by with_species, float64, cell
    layout.  linear_x: c = x / L_x.  blob: a smooth seeded Gaussian bump of
    amplitude 1 (centre and width from the seed).  alpha: a copy of the
    initial volume fraction."""
    s = shapes(c)
    x, y, z = cell_centres(c)
    kind = c.get("species_kind", "linear_x")
    if kind == "alpha":
        return initial_state(c)["alpha"].copy()
    if c["dim"] == 2:
        Y, X = np.meshgrid(y, x, indexing="ij")
        X, Y, Z = X[None], Y[None], np.zeros_like(X[None])
    else:
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    lx = c["nx"] * c["h"]
    if kind == "linear_x":
        f = X / lx
    elif kind == "blob":
        rng = np.random.default_rng(c.get("species_seed", 5))
        ly, lz = c["ny"] * c["h"], c["nz"] * c["h"]
        ctr = rng.uniform(0.3, 0.7, 3) * np.array([lx, ly, lz])
        wid = rng.uniform(0.15, 0.25) * lx
        r2 = (X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + ((Z - ctr[2]) ** 2 if c["dim"] == 3 else 0.0)
        f = np.exp(-r2 / (wid * wid))
    else:
        raise ValueError(f"unknown species kind {kind}")
    return np.ascontiguousarray(np.broadcast_to(f, s["cell"]).reshape(s["cell"]), dtype=np.float64)


# ----------------------------------------------------------------------------
# N-phase VOF (eq. 1 for every phase; phase 1 is the background with
# alpha_1 = 1 - sum of the others)
PAIRS = ((1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (3, 4))


def with_phases(c, layout, phases, pair_sigma0, pair_dsigma_dT) -> dict:
    """N-phase config: ``phases`` lists the material values of phases 3 (and
    4) as dicts with rho, mu, rhocp, lambda; ``pair_sigma0`` and
    ``pair_dsigma_dT`` map a pair (i, j) of phases to sigma_ij = sigma0 +
    dsigma_dT (T - T0) (missing pairs carry no tension).  ``layout`` names
    the initial fractions built by phase_fields."""
    out = dict(c)
    out.update(nphases=2 + len(phases), phases=[dict(p) for p in phases], phase_layout=layout,
               pair_sigma0=[float(pair_sigma0.get(p, 0.0)) for p in PAIRS],
               pair_dsigma_dT=[float(pair_dsigma_dT.get(p, 0.0)) for p in PAIRS])
    return out


def droplet_phases(c, layout):
    """The 2D droplet sheet with a third phase (denser, more viscous) and
    distinct surface tensions for the three pairs."""
    ph3 = dict(rho=3.0, mu=0.03, rhocp=2.0, **{"lambda": 1.5e-3})
    return with_phases(c, layout, [ph3], {(1, 2): 1.0, (1, 3): 0.8, (2, 3): 0.5},
                       {(1, 2): -0.1, (1, 3): -0.05, (2, 3): -0.02})


def droplet_phases4(c, layout):
    """droplet_phases with a fourth phase (lighter, less viscous) and tensions
    for all six pairs."""
    ph3 = dict(rho=3.0, mu=0.03, rhocp=2.0, **{"lambda": 1.5e-3})
    ph4 = dict(rho=1.5, mu=0.005, rhocp=3.0, **{"lambda": 0.8e-3})
    return with_phases(c, layout, [ph3, ph4],
                       {(1, 2): 1.0, (1, 3): 0.8, (1, 4): 0.6, (2, 3): 0.5, (2, 4): 0.4, (3, 4): 0.3},
                       {(1, 2): -0.1, (1, 3): -0.05, (1, 4): -0.08, (2, 3): -0.02, (2, 4): -0.03, (3, 4): -0.01})


def meltpool_phases(c):
    """The melt-pool sheet with three phases: gas (1), liquid metal (2) in a
    pool under the beam's start, and solid metal (3) around and below it.
    Without a phase-change model the solid is a more viscous fluid with a
    higher conductivity; gas-liquid keeps the thermal
    Marangoni law, gas-solid a constant tension, liquid-solid none.  The
    solid's viscosity (50 times the melt's) keeps the explicit viscous number
    dt mu / (rho h^2) at 0.05 on the 2.5 um grid with dt = 1e-8 s."""
    ph3 = dict(rho=c["rho2"], mu=50.0 * c["mu2"], rhocp=c["rhocp2"], **{"lambda": 20.0})
    out = with_phases(c, "meltpool3", [ph3], {(1, 2): c["sigma0"], (1, 3): c["sigma0"]},
                      {(1, 2): c["dsigma_dT"]})
    # the beam starts at (L_x / 4, L_y / 2) of this box, above the pool
    out.update(q_x0=c["nx"] * c["h"] / 4.0, q_y0=c["ny"] * c["h"] / 2.0)
    return out


def phase_fields(c) -> dict:
    """Initial fractions of an N-phase config: dict(alpha=alpha_2,
    alpha3=..., [alpha4=...]) as float64 cell arrays (tanh edges of length
    1.5 h).  Layouts: absent (phase 2 as in initial_state, phase 3 zero),
    two_drops (2D: drops of phases 2 and 3 of radius 0.1 L at 0.25 L and
    0.75 L), layers4 (phases 4 | 3 | 2 | 1 upward, edges at 0.25, 0.45,
    0.65 L), absent4 (the lens with a fourth phase of zero fraction), layers
    (phase 3 below
    0.3 L, phase 2 up to 0.6 L, background above, along the vertical), lens
    (2D: a phase-3 drop on a phase-2 layer), meltpool3 (the melt-pool surface
    with a liquid half-ellipsoid under the beam's start, solid elsewhere)."""
    s = shapes(c)
    h = c["h"]
    w = 1.5 * h
    x, y, z = cell_centres(c)
    if c["dim"] == 2:
        Y, X = np.meshgrid(y, x, indexing="ij")
        X, Y, Z = X[None], Y[None], None
    else:
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    vert = Y if c["dim"] == 2 else Z
    lv = (c["ny"] if c["dim"] == 2 else c["nz"]) * h
    lay = c["phase_layout"]
    if lay == "absent":
        a2 = initial_state(c)["alpha"]
        a3 = np.zeros_like(a2)
    elif lay == "two_drops":
        lx, ly = c["nx"] * h, c["ny"] * h
        r2 = np.hypot(X - 0.25 * lx, Y - 0.5 * ly)
        r3 = np.hypot(X - 0.75 * lx, Y - 0.5 * ly)
        a2 = _smooth_step(0.1 * lx - r2, w)
        a3 = _smooth_step(0.1 * lx - r3, w)
    elif lay == "layers":
        a3 = _smooth_step(0.3 * lv - vert, w)
        a2 = _smooth_step(0.6 * lv - vert, w) - a3
    elif lay == "layers4":
        a4 = _smooth_step(0.25 * lv - vert, w)
        a3 = _smooth_step(0.45 * lv - vert, w) - a4
        a2 = _smooth_step(0.65 * lv - vert, w) - a3 - a4
    elif lay == "absent4":
        a2, a3 = None, None
    elif lay == "lens":
        a3 = _smooth_step(0.15 - np.hypot(X - 0.5, Y - 0.45), w)
        a2 = _smooth_step(0.45 - Y, w) * (1.0 - a3)
    elif lay == "meltpool3":
        ac = initial_state(c)["alpha"]
        lx, ly, lz = c["nx"] * h, c["ny"] * h, c["nz"] * h
        e = np.sqrt(((X - 0.25 * lx) / (0.25 * lx)) ** 2 + ((Y - 0.5 * ly) / (0.25 * ly)) ** 2
                    + ((Z - 0.5 * lz) / (0.2 * lz)) ** 2)
        pool = _smooth_step(0.25 * lx * (1.0 - e), w)
        a2 = ac * pool
        a3 = ac * (1.0 - pool)
    else:
        raise ValueError(f"unknown phase layout {lay}")
    f = lambda q: np.ascontiguousarray(np.broadcast_to(q, s["cell"]).reshape(s["cell"]), dtype=np.float64)
    if lay == "absent4":  # the lens of three phases with a fourth of zero fraction
        out = phase_fields(dict(c, phase_layout="lens"))
        out["alpha4"] = np.zeros_like(out["alpha"])
        return out
    out = dict(alpha=f(a2), alpha3=f(a3))
    if lay == "layers4":
        out["alpha4"] = f(a4)
    return out


def phase_state(c) -> dict:
    """initial_state(c) with the fractions of phase_fields(c)."""
    st = initial_state(c)
    st.update(phase_fields(c))
    return st


def stream_velocity(c, amp=1.0):
    """Discretely divergence-free MAC velocity from face differences of the
    corner stream function psi = L sin^2(pi x/Lx) sin^2(pi y/Ly)/pi (L = Ly,
    so the speed is of order amp on any box; times a z profile in 3D), zero
    on every wall face.  Used to drive transport-only checks."""
    nx, ny, nz, h = c["nx"], c["ny"], c["nz"], c["h"]
    lx, ly, lz = nx * h, ny * h, nz * h
    xn = np.arange(nx + 1) * h
    yn = np.arange(ny + 1) * h
    psi = ly * (np.sin(np.pi * xn / lx)[None, :] ** 2 * np.sin(np.pi * yn / ly)[:, None] ** 2) / np.pi
    if c["dim"] == 3:
        zc = (np.arange(nz) + 0.5) * h
        g = (0.5 + 0.5 * np.cos(np.pi * zc / lz))[:, None, None]
    else:
        g = np.ones((1, 1, 1))
    u = amp * g * (psi[1:, :] - psi[:-1, :])[None] / h          # (nz, ny, nx+1)
    v = -amp * g * (psi[:, 1:] - psi[:, :-1])[None] / h         # (nz, ny+1, nx)
    w = np.zeros((nz + 1, ny, nx)) if c["dim"] == 3 else None
    return (np.ascontiguousarray(u), np.ascontiguousarray(v), w)


def stream_velocity_3d(c, amp=1.0):
    """A 3-D discretely divergence-free MAC velocity with all three
    components nonzero: the x-y flow of stream_velocity (modulated along z)
    plus an x-z flow from the edge stream function
    L sin^2(pi x/Lx) sin^2(pi z/Lz)/pi, modulated along y by
    1/2 + cos(pi y/Ly)/3.  Each part is a face difference of an edge
    potential times a factor constant on the faces it differences, so the
    discrete divergence vanishes; normal velocities vanish on the walls."""
    assert c["dim"] == 3
    nx, ny, nz, h = c["nx"], c["ny"], c["nz"], c["h"]
    lx, ly, lz = nx * h, ny * h, nz * h
    u, v, w = stream_velocity(c, amp)
    xn = np.arange(nx + 1) * h
    zn = np.arange(nz + 1) * h
    yc = (np.arange(ny) + 0.5) * h
    psi = lz * (np.sin(np.pi * xn / lx)[None, :] ** 2 * np.sin(np.pi * zn / lz)[:, None] ** 2) / np.pi
    f = (0.5 + np.cos(np.pi * yc / ly) / 3.0)[None, :, None]
    u = u + amp * f * ((psi[1:, :] - psi[:-1, :]) / h)[:, None, :]            # (nz, ny, nx+1)
    w = -amp * f * ((psi[:, 1:] - psi[:, :-1]) / h)[:, None, :]               # (nz+1, ny, nx)
    u[:, :, 0] = u[:, :, -1] = 0.0
    w[0] = w[-1] = 0.0
    return (np.ascontiguousarray(u), v, np.ascontiguousarray(w))


def random_fields(c, seed, scale=1.0):
    """Smooth-ish random fields for operator checks (not physical)."""
    rng = np.random.default_rng(seed)
    s = shapes(c)
    out = {k: scale * rng.standard_normal(v) if v else None for k, v in s.items()}
    return out


def target_centroid(c):
    """Seeded target for the droplet centroid loss: initial centroid of the
    indicator plus a uniform offset in [-0.02, 0.02]^3."""
    rng = np.random.default_rng(c.get("target_seed", 3))
    return rng.uniform(-0.02, 0.02, 3)


def t_directions(c, k=16, seed=3, modes=4):
    """Seeded smooth unit directions in the space of initial temperature
    fields: random combinations of the cosine modes 0..modes-1 along each
    axis (white noise would probe mostly grid-scale components to which a
    loss of the droplet centroid is nearly blind)."""
    rng = np.random.default_rng(seed + 1000)
    nz, ny, nx = shapes(c)["cell"]
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    out = np.zeros((k, nz, ny, nx))
    mz = modes if c["dim"] == 3 else 1
    for q in range(k):
        for l in range(mz):
            for m in range(modes):
                for n in range(modes):
                    out[q] += rng.standard_normal() * (np.cos(l * np.pi * z)[:, None, None] *
                                                       np.cos(m * np.pi * y)[None, :, None] *
                                                       np.cos(n * np.pi * x)[None, None, :])
        out[q] /= np.linalg.norm(out[q])
    return out


def describe(c) -> str:
    return f"{c['name']} ({c['nx']}x{c['ny']}x{c['nz']}, h={c['h']:.3g})"


__all__ = ["config", "custom", "initial_state", "stream_velocity", "shapes",
           "random_fields", "cell_centres", "target_centroid", "t_directions",
           "describe", "NEUMANN", "DIRICHLET"]

if __name__ == "__main__":  # pragma: no cover
    for i in range(4):
        c = config(i)
        st = initial_state(c)
        print(describe(c), {k: (None if v is None else v.shape) for k, v in st.items()},
              float(st["alpha"].sum()), math.isfinite(float(st["T"].sum())))
