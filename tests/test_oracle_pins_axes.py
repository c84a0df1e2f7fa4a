"""Pins of the oracle's operators along y and z, and of the variable
coefficients, against what the mathematics fixes.

The x-direction pins of the WENO5 transport, the conduction and the
momentum operators sit in test_oracle_pins.py.  The oracle writes every
direction through the same face loops with a direction index, so a swapped
j/k index, a wrong upwind branch along y or z, or a z-edge term taken from
the wrong face would leave the x-direction pins green.  The tests below
repeat the pins along y and z, diagonally, and for the u, v and w components
in 3D, each against a closed form, a convergence order or an exact
invariant:
  - WENO5-JS with SSP-RK3 (eq. 1, the advection of the volume fraction) is
    fifth order on smooth periodic advection along any axis and diagonally;
  - the conduction term of the energy equation is exact for a quadratic
    temperature when the conductivity is linear in space (arithmetic face
    mean), and its Neumann cosine modes decay at the RK3 amplification;
  - the convective and viscous momentum terms (Navier-Stokes, Section
    "Theory") converge at second order to div(u u) and
    div(mu (grad u + grad u^T)) for every component.
"""
import math

import numpy as np
import pytest
import sympy as sp

from oracle import pyoracle as O
from paper_2209_09671_amd import inputs as I


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _grid(dim, nx, ny, nz=1, **over):
    base = I.config(0) if dim == 2 else I.config(3)
    c = I.custom(base, nx=nx, ny=ny, nz=nz) if dim == 3 else I.custom(base, nx=nx, ny=ny)
    c["h"] = 1.0 / max(nx, ny, nz)
    c["normal_eps"] = 1e-6 / c["h"]
    c["T_bc"] = [0] * 6
    c.update(over)
    return c


def _zero_state(c):
    nx, ny = c["nx"], c["ny"]
    nz = c["nz"] if c["dim"] == 3 else 1
    z = np.zeros((nz, ny, nx))
    return dict(alpha=z.copy(), T=z.copy(), u=np.zeros((nz, ny, nx + 1)), v=np.zeros((nz, ny + 1, nx)),
                w=np.zeros((nz + 1, ny, nx)) if c["dim"] == 3 else None, p=z.copy())


# ---------------------------------------------------------------------------
# WENO5 + SSP-RK3 along y, along z and diagonally (eq. 1).
def _cell_avg_sin(n):
    """Exact cell averages of sin(2 pi x) on n unit-interval cells."""
    h = 1.0 / n
    x = np.arange(n + 1) * h
    return (np.cos(2 * np.pi * x[:-1]) - np.cos(2 * np.pi * x[1:])) / (2 * np.pi * h)


def _advect_along_axis(n, axis):
    """One period of periodic advection at unit speed along `axis` of a
    one-cell-thick grid (2D for x and y, 3D for z); returns (L1 error, field)."""
    dim = 3 if axis == 2 else 2
    ext = [1, 1, 1]
    ext[axis] = n
    c = _grid(dim, ext[0], ext[1], ext[2], lambda1=0.0, lambda2=0.0)
    st = _zero_state(c)
    shape = st["alpha"].shape
    prof = [1, 1, 1]
    prof[2 - axis] = n
    exact = np.broadcast_to(_cell_avg_sin(n).reshape(prof), shape).copy()
    st["alpha"] = exact.copy()
    (st["u"], st["v"], st["w"])[axis][:] = 1.0
    h = c["h"]
    nsteps = int(math.ceil(1.0 / (0.4 * h ** (5.0 / 3.0))))
    s, _, _ = O.step(c, st, 0.0, 1.0 / nsteps, nsteps, flags=O.F_TRANSPORT_ONLY | O.F_PERIODIC)
    return h * np.abs(s["alpha"] - exact).sum(), s["alpha"].ravel()


@pytest.mark.parametrize("axis", [1, 2])
def test_weno_rk3_fifth_order_along_y_and_z(axis):
    """Fifth-order convergence along y (2D) and z (3D).  A face loop along
    y or z that took its stencil from the wrong index (j for k), or the
    downwind branch, would lose the order or go unstable.  The same 1-D
    problem along x gives the same numbers to rounding: the result may not
    depend on the axis it is laid along."""
    ns = [32, 64, 128, 256]
    err, fields = zip(*[_advect_along_axis(n, axis) for n in ns])
    orders = [math.log2(err[i] / err[i + 1]) for i in range(len(ns) - 1)]
    assert min(orders) >= 4.8, (err, orders)
    ex, fx = _advect_along_axis(64, 0)
    assert np.abs(fields[1] - fx).max() <= 1e-14
    assert abs(err[1] - ex) <= 1e-12 * ex


def _advect_diagonal(n, dims):
    """One period of advection of sin(2 pi (sum of the coordinates in
    `dims`)) at unit speed along every axis in `dims` (periodic); returns the
    L1 error against the exact cell averages."""
    dim = 3 if 2 in dims else 2
    ext = [n if d in dims else 1 for d in range(3)]
    c = _grid(dim, ext[0], ext[1], ext[2], lambda1=0.0, lambda2=0.0)
    st = _zero_state(c)
    h = c["h"]
    xc = (np.arange(n) + 0.5) * h
    nz, ny, nx = st["alpha"].shape
    coords = np.meshgrid(*[xc if e > 1 else np.zeros(1) for e in (nz, ny, nx)], indexing="ij")
    phase = sum(coords[2 - d] for d in dims)
    damp = (math.sin(math.pi * h) / (math.pi * h)) ** len(dims)   # cell average of a plane wave
    exact = damp * np.sin(2 * np.pi * phase)
    st["alpha"] = exact.copy()
    for d in dims:
        (st["u"], st["v"], st["w"])[d][:] = 1.0
    nsteps = int(math.ceil(1.0 / (0.4 * h ** (5.0 / 3.0))))
    s, _, _ = O.step(c, st, 0.0, 1.0 / nsteps, nsteps, flags=O.F_TRANSPORT_ONLY | O.F_PERIODIC)
    return h ** len(dims) * np.abs(s["alpha"] - exact).sum()


@pytest.mark.parametrize("dims", [(0, 1), (1, 2)])
def test_weno_rk3_fifth_order_diagonal(dims):
    """Fifth order for a wave travelling diagonally in the x-y plane (2D)
    and in the y-z plane (3D grid): every face direction carries flux at
    once, so a mix-up between the y and z face loops shows here."""
    ns = [16, 32, 64]
    err = [_advect_diagonal(n, dims) for n in ns]
    orders = [math.log2(err[i] / err[i + 1]) for i in range(len(ns) - 1)]
    assert min(orders) >= 4.8, (err, orders)


def test_weno_rk3_diagonal_3d():
    """The full 3-D diagonal (x + y + z).  At 16^3 -> 32^3 the scheme is
    not quite asymptotic (measured order 4.77; 3.9 from 8^3), so the bar is
    4.6: still far above what a stencil error in one direction leaves
    (third order or worse)."""
    err = [_advect_diagonal(n, (0, 1, 2)) for n in (16, 32)]
    order = math.log2(err[0] / err[1])
    assert order >= 4.6, (err, order)


@pytest.mark.parametrize("axis", [1, 2])
def test_upwind_mirror_symmetry_along_y_and_z(axis):
    """Advecting a random profile toward +y (+z) equals advecting its mirror
    image toward -y (-z), mirrored back, bitwise: catches index errors in
    the right-biased (negative velocity) branch along y and z."""
    n = 32
    dim = 3 if axis == 2 else 2
    ext = [1, 1, 1]
    ext[axis] = n
    c = _grid(dim, ext[0], ext[1], ext[2], lambda1=0.0, lambda2=0.0)
    rng = np.random.default_rng(7 + axis)
    a0 = rng.random(_zero_state(c)["alpha"].shape)
    ax = 2 - axis   # numpy axis of the grid axis

    def run(a, vel):
        st = _zero_state(c)
        st["alpha"] = a
        (st["u"], st["v"], st["w"])[axis][:] = vel
        s, _, _ = O.step(c, st, 0.0, 0.2 * c["h"], 5, flags=O.F_TRANSPORT_ONLY | O.F_PERIODIC)
        return s["alpha"]

    s1 = run(a0, 1.0)
    s2 = run(np.flip(a0, ax).copy(), -1.0)
    assert np.array_equal(s1, np.flip(s2, ax))


# ---------------------------------------------------------------------------
# Conduction (energy equation) along y and z, and with variable conductivity.
@pytest.mark.parametrize("axis", [1, 2])
def test_conduction_cosine_mode_along_y_and_z(axis):
    """cos(pi y) (cos(pi z)) at cell centres is a discrete Neumann
    eigenvector of the conduction operator with eigenvalue
    -(4/h^2) sin^2(pi/(2n)); with u = 0 one RK3 step multiplies it by
    1 + z + z^2/2 + z^3/6, z = dt lambda/(rho c_p) times that eigenvalue.
    A wall ghost taken from the wrong axis or a missing z-face term breaks
    the amplification."""
    n = 24
    dim = 3 if axis == 2 else 2
    c = _grid(dim, n, n, n if dim == 3 else 1, lambda1=2e-3, lambda2=2e-3, rhocp1=3.0, rhocp2=3.0)
    st = _zero_state(c)
    h = c["h"]
    x = (np.arange(n) + 0.5) * h
    prof = [1, 1, 1]
    prof[2 - axis] = n
    T0 = np.broadcast_to(np.cos(np.pi * x).reshape(prof), st["T"].shape).copy()
    st["T"] = T0
    dt = 0.05
    s, _, _ = O.step(c, st, 0.0, dt, 1, flags=O.F_TRANSPORT_ONLY)
    lam = -(4.0 / h ** 2) * np.sin(np.pi / (2 * n)) ** 2
    z = dt * 2e-3 / 3.0 * lam
    assert rel(s["T"], T0 * (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-13


def test_conduction_exact_for_linear_conductivity_and_quadratic_T():
    """With alpha linear in space, lambda = lambda1 + alpha (lambda2 -
    lambda1) is linear, so its arithmetic face mean is its exact face value;
    for a quadratic T the face difference is the exact face derivative, and
    lambda dT/dx_d is quadratic along x_d, so the discrete conduction term
    equals div(lambda grad T) at the cell centre exactly (to rounding), in
    every direction.  Divided by rho c_p(alpha) (linear mix) this is the T
    right-hand side with u = 0.  A harmonic or geometric face mean (here
    ~1e-3 off), a direction's term taken with another direction's
    neighbours, or rho c_p taken at another cell fails it."""
    n = 12
    c = _grid(3, n, n, n, lambda1=1e-3, lambda2=1e-2, rhocp1=1.0, rhocp2=3.0, q_power=0.0)
    h = c["h"]
    X, Y, Z = sp.symbols("x y z")
    alpha_s = 0.1 + 0.4 * X + 0.25 * Y + 0.15 * Z
    T_s = X ** 2 + 0.5 * Y ** 2 - 0.7 * Z ** 2 + 0.3 * X * Y - 0.2 * Y * Z + 0.4 * X * Z + X
    lam_s = 1e-3 + alpha_s * (1e-2 - 1e-3)
    div_s = sum(sp.diff(lam_s * sp.diff(T_s, v), v) for v in (X, Y, Z))
    rhs_s = div_s / (1.0 + alpha_s * 2.0)
    xc = (np.arange(n) + 0.5) * h
    Zc, Yc, Xc = np.meshgrid(xc, xc, xc, indexing="ij")
    f = lambda e: sp.lambdify((X, Y, Z), e, "numpy")(Xc, Yc, Zc) * np.ones_like(Xc)
    st = _zero_state(c)
    alpha, T = f(alpha_s), f(T_s)
    La, LT = O.transport_rhs(c, 0.0, alpha, T, st["u"], st["v"], st["w"])
    inner = (slice(1, -1),) * 3
    ref = f(rhs_s)[inner]
    assert np.abs(La).max() == 0.0
    assert np.abs(LT[inner] - ref).max() <= 1e-10 * np.abs(ref).max(), np.abs(LT[inner] - ref).max()


# ---------------------------------------------------------------------------
# Momentum operators for every component (Navier-Stokes, Section "Theory").
def _flow_2d():
    """Stream-function flow psi = sin^2(pi x) sin^2(pi y)/pi: u = psi_y,
    v = -psi_x (divergence free, normal velocity zero on the walls)."""
    X, Y = sp.symbols("x y")
    psi = sp.sin(sp.pi * X) ** 2 * sp.sin(sp.pi * Y) ** 2 / sp.pi
    return (X, Y), [sp.diff(psi, Y), -sp.diff(psi, X)]


def _flow_3d():
    """A genuinely 3-D divergence-free flow: an x-y stream-function flow
    modulated along z plus an x-z stream-function flow modulated along y,
    u = g(z) psi1_y + f(y) psi2_z, v = -g(z) psi1_x, w = -f(y) psi2_x, so
    every component depends on all three coordinates and w is nonzero."""
    X, Y, Z = sp.symbols("x y z")
    psi1 = sp.sin(sp.pi * X) ** 2 * sp.sin(sp.pi * Y) ** 2 / sp.pi
    psi2 = sp.sin(sp.pi * X) ** 2 * sp.sin(sp.pi * Z) ** 2 / sp.pi
    g = sp.Rational(1, 2) + sp.cos(sp.pi * Z) / 2
    f = sp.Rational(1, 2) + sp.cos(sp.pi * Y) / 3
    return (X, Y, Z), [g * sp.diff(psi1, Y) + f * sp.diff(psi2, Z), -g * sp.diff(psi1, X), -f * sp.diff(psi2, X)]


def _face_coords(c, d):
    """Coordinates of the d-faces (x, y, z arrays broadcast to the face
    array's shape)."""
    n = [c["nx"], c["ny"], c["nz"] if c["dim"] == 3 else 1]
    h = c["h"]
    ax = []
    for e in range(3):
        if e == d:
            ax.append(np.arange(n[e] + 1) * h)
        else:
            ax.append((np.arange(n[e]) + 0.5) * h)
    Zc, Yc, Xc = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return Xc, Yc, Zc


def _momentum_errors(dim, n, mu_var):
    """Max interior errors of the oracle's convective and viscous terms of
    each component against div(u u_d) and div(mu (grad u + grad u^T))_d.
    The predictor at amplitudes A and 2A (rho = 1, no surface tension)
    gives (u* - u)/dt = -A^2 C + A V with linear WENO weights (A tiny), so
    C and V separate exactly."""
    syms, vel = (_flow_2d() if dim == 2 else _flow_3d())
    c = _grid(dim, n, n, n if dim == 3 else 1, rho1=1.0, rho2=1.0, mu1=0.01, mu2=0.05 if mu_var else 0.01,
              sigma0=0.0, dsigma_dT=0.0)
    if dim == 2:
        alpha_s = 0.2 + 0.35 * syms[0] + 0.3 * syms[1]
    else:
        alpha_s = 0.1 + 0.4 * syms[0] + 0.25 * syms[1] + 0.15 * syms[2]
    mu_s = c["mu1"] + alpha_s * (c["mu2"] - c["mu1"])
    conv_s, visc_s = [], []
    for d in range(dim):
        conv_s.append(sum(vel[e] * sp.diff(vel[d], syms[e]) for e in range(dim)))
        visc_s.append(sum(sp.diff(mu_s * (sp.diff(vel[d], syms[e]) + sp.diff(vel[e], syms[d])), syms[e])
                          for e in range(dim)))

    def ev(expr, X, Y, Z):
        args = (X, Y) if dim == 2 else (X, Y, Z)
        return sp.lambdify(syms, expr, "numpy")(*args) * np.ones_like(X)

    st = _zero_state(c)
    h = c["h"]
    xc = (np.arange(n) + 0.5) * h
    if dim == 2:
        Yc, Xc = np.meshgrid(xc, xc, indexing="ij")
        alpha = ev(alpha_s, Xc, Yc, None)[None]
    else:
        Zc, Yc, Xc = np.meshgrid(xc, xc, xc, indexing="ij")
        alpha = ev(alpha_s, Xc, Yc, Zc)
    base = [ev(vel[d], *_face_coords(c, d)) for d in range(dim)]
    A1 = 1e-5
    du = []
    for A in (A1, 2 * A1):
        fl = [A * b for b in base]
        out = O.predictor(c, 1.0, alpha, np.zeros_like(alpha), *fl, *([None] if dim == 2 else []))
        du.append([out[d] - fl[d] for d in range(dim)])
    econv, evisc = [], []
    for d in range(dim):
        C1 = -(du[1][d] - 2 * du[0][d]) / (2 * A1 * A1)
        V1 = (4 * du[0][d] - du[1][d]) / (2 * A1)
        X, Y, Z = _face_coords(c, d)
        inner = (slice(4, -4),) * 3 if dim == 3 else (slice(None), slice(4, -4), slice(4, -4))
        cref = ev(conv_s[d], X, Y, Z)
        vref = ev(visc_s[d], X, Y, Z)
        econv.append(np.abs(C1[inner] - cref[inner]).max())
        evisc.append(np.abs(V1[inner] - vref[inner]).max())
    return econv, evisc


def _orders(errs, ns):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("mu_var", [False, True])
def test_momentum_v_component_2d_converges_to_closed_forms(mu_var):
    """The v component in 2D (the x-direction pin covers u only): its
    convection along x uses the edge-averaged u and the WENO5 value of v
    along x, along y the cell-averaged v; its viscous term uses the cell
    viscosity for tau_yy and the four-cell edge mean for tau_xy.  With a
    linear viscosity field (mu_var) the variable-viscosity stress
    div(mu (grad u + grad u^T)) is pinned too.  Orders >= 1.8."""
    ns = (32, 64, 128)
    errs = [_momentum_errors(2, n, mu_var) for n in ns]
    for d in range(2):
        oc = _orders([e[0][d] for e in errs], ns)
        ov = _orders([e[1][d] for e in errs], ns)
        assert min(oc) >= 1.8, ("conv", d, [e[0][d] for e in errs], oc)
        assert min(ov) >= 1.8, ("visc", d, [e[1][d] for e in errs], ov)


@pytest.mark.parametrize("mu_var", [False, True])
def test_momentum_3d_every_component_converges_to_closed_forms(mu_var):
    """u, v and w in 3D on a flow where every component depends on x, y
    and z: pins the z-direction convective fluxes (w-averaged edges, WENO5
    along z), the z-edge shear stresses tau_xz, tau_yz and the w component's
    own terms, which no 2-D pin reaches.  Orders >= 1.8 from 24^3 to 96^3
    (measured 1.86-2.0; at 16^3 the convection is not yet asymptotic)."""
    ns = (24, 48, 96)
    errs = [_momentum_errors(3, n, mu_var) for n in ns]
    for d in range(3):
        oc = _orders([e[0][d] for e in errs], ns)
        ov = _orders([e[1][d] for e in errs], ns)
        assert min(oc) >= 1.8, ("conv", d, [e[0][d] for e in errs], oc)
        assert min(ov) >= 1.8, ("visc", d, [e[1][d] for e in errs], ov)
