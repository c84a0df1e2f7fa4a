"""ctypes wrapper of the FP64 CPU oracle (oracle/tcf_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tcf_oracle.cpp")
_LIB = os.path.join(_HERE, "libtcf_oracle.so")

F_TRANSPORT_ONLY, F_PERIODIC, F_CONST_SIGKAP = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class OrcConfig(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("h", C.c_double), ("flags", C.c_int),
                ("rho1", C.c_double), ("rho2", C.c_double), ("mu1", C.c_double), ("mu2", C.c_double),
                ("rhocp1", C.c_double), ("rhocp2", C.c_double), ("lam1", C.c_double), ("lam2", C.c_double),
                ("sigma0", C.c_double), ("dsigma_dT", C.c_double), ("T0", C.c_double),
                ("T_bc", C.c_int * 6), ("T_wall", C.c_double * 6),
                ("q_power", C.c_double), ("q_radius", C.c_double), ("q_x0", C.c_double),
                ("q_y0", C.c_double), ("q_vx", C.c_double), ("q_vy", C.c_double),
                ("weno_eps", C.c_double), ("normal_eps", C.c_double),
                ("p_rtol", C.c_double), ("p_maxit", C.c_int), ("mg_nu", C.c_int),
                ("mg_omega_c", C.c_double), ("mg_coarse_sweeps", C.c_int),
                ("sigkap_const", C.c_double),
                ("species", C.c_int), ("dsigma_dc", C.c_double), ("c0", C.c_double),
                ("integrator", C.c_int),
                ("nphases", C.c_int), ("rho34", C.c_double * 2), ("mu34", C.c_double * 2),
                ("rhocp34", C.c_double * 2), ("lam34", C.c_double * 2),
                ("sig0_pair", C.c_double * 6), ("dsig_pair", C.c_double * 6)]


class OrcInfo(C.Structure):
    _fields_ = [("cg_iters", C.c_int), ("status", C.c_int), ("p_relres", C.c_double),
                ("div_rel", C.c_double), ("sum_alpha", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("cfl_max", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d = C.c_double
        _lib.orc_weno5.restype = d
        _lib.orc_weno5.argtypes = [d] * 6
        _lib.orc_heat_flux.restype = d
        _lib.orc_heat_flux.argtypes = [C.POINTER(OrcConfig), d, d, d]
        _lib.orc_solve_pressure.restype = C.c_int
        _lib.orc_step.restype = C.c_int
        _lib.orc_mg_levels.restype = C.c_int
        _lib.orc_num_threads.restype = C.c_int
    return _lib


def make_config(c: dict, flags: int = 0, sigkap_const: float = 0.0) -> OrcConfig:
    o = OrcConfig()
    o.dim, o.nx, o.ny = c["dim"], c["nx"], c["ny"]
    o.nz = c["nz"] if c["dim"] == 3 else 1
    o.h = c["h"]
    o.flags = flags | (c.get("flags", 0) & 0)
    o.rho1, o.rho2, o.mu1, o.mu2 = c["rho1"], c["rho2"], c["mu1"], c["mu2"]
    o.rhocp1, o.rhocp2, o.lam1, o.lam2 = c["rhocp1"], c["rhocp2"], c["lambda1"], c["lambda2"]
    o.sigma0, o.dsigma_dT, o.T0 = c["sigma0"], c["dsigma_dT"], c["T0"]
    for i in range(6):
        o.T_bc[i] = int(c["T_bc"][i])
        o.T_wall[i] = float(c["T_wall"][i])
    o.q_power, o.q_radius, o.q_x0 = c["q_power"], c["q_radius"], c["q_x0"]
    o.q_y0, o.q_vx, o.q_vy = c["q_y0"], c["q_vx"], c["q_vy"]
    o.weno_eps, o.normal_eps = c["weno_eps"], c["normal_eps"]
    o.p_rtol, o.p_maxit = c.get("oracle_rtol", c["p_rtol"]), c.get("oracle_maxit", 400)
    o.mg_nu = c.get("mg_nu", 2)
    o.mg_omega_c = 1.9
    o.mg_coarse_sweeps = 30
    o.sigkap_const = sigkap_const
    o.species = int(c.get("species", 0))
    o.dsigma_dc, o.c0 = float(c.get("dsigma_dc", 0.0)), float(c.get("c0", 0.0))
    o.integrator = int(c.get("integrator", 0))
    o.nphases = int(c.get("nphases", 0))
    for q, ph in enumerate(c.get("phases", [])[:2]):  # phases 3 and 4
        o.rho34[q], o.mu34[q] = ph["rho"], ph["mu"]
        o.rhocp34[q], o.lam34[q] = ph["rhocp"], ph["lambda"]
    for q in range(6):  # pairs (1,2), (1,3), (1,4), (2,3), (2,4), (3,4)
        o.sig0_pair[q] = float(c.get("pair_sigma0", [0.0] * 6)[q])
        o.dsig_pair[q] = float(c.get("pair_dsigma_dT", [0.0] * 6)[q])
    return o


def _p(x):
    if x is None:
        return None
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data_as(C.POINTER(C.c_double))


def _f64(x):
    return None if x is None else np.ascontiguousarray(x, dtype=np.float64)


def weno5(a, b, c, d, e, eps=1e-6):
    return lib().orc_weno5(a, b, c, d, e, eps)


def heat_flux(c, x, y, t):
    o = make_config(c)
    return lib().orc_heat_flux(C.byref(o), x, y, t)


def num_threads():
    return lib().orc_num_threads()


def transport_rhs(c, t, alpha, T, u, v, w=None, flags=0):
    o = make_config(c, flags)
    alpha, T, u, v, w = map(_f64, (alpha, T, u, v, w))
    La = np.empty_like(alpha)
    LT = np.empty_like(alpha)
    lib().orc_transport_rhs(C.byref(o), C.c_double(t), _p(alpha), _p(T), _p(u), _p(v), _p(w), _p(La), _p(LT))
    return La, LT


def transport_step(c, t, dt, alpha, T, u, v, w=None, flags=0, cfield=None, alpha3=None, alpha4=None):
    """One SSP-RK3 transport step; returns (alpha, T), with a species field
    (alpha, T, c), and for N phases (alpha, T, alpha3[, alpha4])."""
    o = make_config(c, flags)
    a = _f64(alpha).copy()
    TT = _f64(T).copy()
    cc = None if cfield is None else _f64(cfield).copy()
    a3 = None if alpha3 is None else _f64(alpha3).copy()
    a4 = None if alpha4 is None else _f64(alpha4).copy()
    u, v, w = map(_f64, (u, v, w))
    lib().orc_transport_step(C.byref(o), C.c_double(t), C.c_double(dt), _p(a), _p(TT), _p(u), _p(v), _p(w),
                             _p(cc), _p(a3), _p(a4))
    if a3 is not None:
        return (a, TT, a3) if a4 is None else (a, TT, a3, a4)
    return (a, TT) if cc is None else (a, TT, cc)


def geometry(c, alpha, T, flags=0, sigkap_const=0.0, cfield=None):
    o = make_config(c, flags, sigkap_const)
    alpha, T, cf = _f64(alpha), _f64(T), _f64(cfield)
    N = alpha.size
    n = np.empty((N, 3))
    kap, ds, sk = (np.empty_like(alpha) for _ in range(3))
    M = np.empty((N, 3))
    lib().orc_geometry(C.byref(o), _p(alpha), _p(T), _p(n), _p(kap), _p(ds), _p(sk), _p(M), _p(cf))
    return dict(n=n, kappa=kap, delta_s=ds, sigkap=sk, M=M)


def predictor(c, dt, alpha, T, u, v, w=None, flags=0, sigkap_const=0.0, cfield=None, alpha3=None, alpha4=None):
    o = make_config(c, flags, sigkap_const)
    alpha, T, u, v, w, cf, a3, a4 = map(_f64, (alpha, T, u, v, w, cfield, alpha3, alpha4))
    us, vs = np.empty_like(u), np.empty_like(v)
    ws = np.empty_like(w) if w is not None else None
    lib().orc_predictor(C.byref(o), C.c_double(dt), _p(alpha), _p(T), _p(u), _p(v), _p(w),
                        _p(us), _p(vs), _p(ws), _p(cf), _p(a3), _p(a4))
    return us, vs, ws


def phase_pairs(nph):
    """Pairs (i, j), i < j, of an N-phase config in the order of the pair tables."""
    return [p for p in ((1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (3, 4)) if p[1] <= nph]


def geometry_n(c, alpha, alpha3, T, alpha4=None):
    """N-phase geometry: dict of per-pair sigma_ij kappa_ij and delta_ij
    (keys (i, j)) and the summed Marangoni vector M (N x 3)."""
    o = make_config(c)
    alpha, a3, a4, T = map(_f64, (alpha, alpha3, alpha4, T))
    pairs = phase_pairs(o.nphases)
    N = alpha.size
    skp = np.zeros((len(pairs), N))
    dsp = np.zeros((len(pairs), N))
    M = np.empty((N, 3))
    lib().orc_geometry_n(C.byref(o), _p(alpha), _p(a3), _p(a4), _p(T), _p(skp), _p(dsp), _p(M))
    sh = alpha.shape
    return dict(sigkap={p: skp[q].reshape(sh) for q, p in enumerate(pairs)},
                delta={p: dsp[q].reshape(sh) for q, p in enumerate(pairs)}, M=M)


def divergence(c, u, v, w=None):
    o = make_config(c)
    u, v, w = map(_f64, (u, v, w))
    out = np.empty((o.nz, o.ny, o.nx))
    lib().orc_divergence(C.byref(o), _p(u), _p(v), _p(w), _p(out))
    return out


def apply_A(c, alpha, p):
    o = make_config(c)
    alpha, p = _f64(alpha), _f64(p)
    out = np.empty_like(p)
    lib().orc_apply_A(C.byref(o), _p(alpha), _p(p), _p(out))
    return out


def apply_mg(c, alpha, r):
    o = make_config(c)
    alpha, r = _f64(alpha), _f64(r)
    z = np.empty_like(r)
    lib().orc_apply_mg(C.byref(o), _p(alpha), _p(r), _p(z))
    return z


def mg_levels(c):
    o = make_config(c)
    return lib().orc_mg_levels(C.byref(o))


def solve_pressure(c, alpha, b, p0=None, rtol=None, alpha3=None, alpha4=None):
    cc = dict(c)
    if rtol is not None:
        cc["oracle_rtol"] = rtol
    o = make_config(cc)
    alpha, b, a3, a4 = map(_f64, (alpha, b, alpha3, alpha4))
    p = np.zeros_like(b) if p0 is None else _f64(p0).copy()
    info = OrcInfo()
    st = lib().orc_solve_pressure(C.byref(o), _p(alpha), _p(b), _p(p), C.byref(info), _p(a3), _p(a4))
    return p, st, info.as_dict()


def project(c, dt, alpha, p, us, vs, ws=None, alpha3=None, alpha4=None):
    o = make_config(c)
    alpha, p, us, vs, ws, a3, a4 = map(_f64, (alpha, p, us, vs, ws, alpha3, alpha4))
    u, v = np.empty_like(us), np.empty_like(vs)
    w = np.empty_like(ws) if ws is not None else None
    lib().orc_project(C.byref(o), C.c_double(dt), _p(alpha), _p(p), _p(us), _p(vs), _p(ws), _p(u), _p(v), _p(w),
                      _p(a3), _p(a4))
    return u, v, w


def step(c, state, t, dt, nsteps=1, flags=0, sigkap_const=0.0, rtol=None):
    """Run nsteps full steps; returns (new_state, info dict, status).  A
    species field travels as state["c"] (used when the config has species),
    the fractions of phases 3 and 4 of an N-phase config as state["alpha3"]
    and state["alpha4"]."""
    cc = dict(c)
    if rtol is not None:
        cc["oracle_rtol"] = rtol
    o = make_config(cc, flags, sigkap_const)
    s = {k: (None if v is None else _f64(v).copy()) for k, v in state.items()}
    info = OrcInfo()
    st = lib().orc_step(C.byref(o), C.c_double(t), C.c_double(dt), C.c_int(nsteps),
                        _p(s["alpha"]), _p(s["T"]), _p(s["u"]), _p(s["v"]), _p(s["w"]), _p(s["p"]),
                        C.byref(info), _p(s.get("c")), _p(s.get("alpha3")), _p(s.get("alpha4")))
    return s, info.as_dict(), st
