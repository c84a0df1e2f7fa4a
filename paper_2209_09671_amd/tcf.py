"""Python binding of libtcf.so (the C ABI in include/tcf.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  PyTorch provides device memory (the workspace and the field
tensors) and the stream.  Loading fails loudly when the library is missing:
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcf.so")

TCF_OK, TCF_E_INVALID, TCF_E_DEVICE, TCF_E_NOT_CONVERGED, TCF_E_NONFINITE, TCF_E_STATE, TCF_E_WORKSPACE = range(7)
TCF_FP64, TCF_FP32_REFINE = 0, 1
TCF_TRANSPORT_ONLY = 1
TCF_WITH_ADJOINT = 2
STATUS_NAMES = {0: "TCF_OK", 1: "TCF_E_INVALID", 2: "TCF_E_DEVICE", 3: "TCF_E_NOT_CONVERGED",
                4: "TCF_E_NONFINITE", 5: "TCF_E_STATE", 6: "TCF_E_WORKSPACE"}


class TcfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class TcfConfig(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double),
                ("precision", C.c_int), ("flags", C.c_int),
                ("rho1", C.c_double), ("rho2", C.c_double), ("mu1", C.c_double), ("mu2", C.c_double),
                ("rhocp1", C.c_double), ("rhocp2", C.c_double), ("lambda1", C.c_double), ("lambda2", C.c_double),
                ("sigma0", C.c_double), ("dsigma_dT", C.c_double), ("T0", C.c_double),
                ("T_bc", C.c_int * 6), ("T_wall", C.c_double * 6),
                ("q_power", C.c_double), ("q_radius", C.c_double), ("q_x0", C.c_double), ("q_y0", C.c_double),
                ("q_vx", C.c_double), ("q_vy", C.c_double),
                ("weno_eps", C.c_double), ("normal_eps", C.c_double),
                ("p_rtol", C.c_double), ("p_maxit", C.c_int), ("inner_rtol", C.c_double),
                ("refine_maxit", C.c_int), ("mg_levels", C.c_int), ("mg_nu", C.c_int), ("p_extrapolate", C.c_int),
                ("species", C.c_int), ("dsigma_dc", C.c_double), ("c0", C.c_double),
                ("integrator", C.c_int),
                ("nphases", C.c_int), ("rho34", C.c_double * 2), ("mu34", C.c_double * 2),
                ("rhocp34", C.c_double * 2), ("lambda34", C.c_double * 2),
                ("pair_sigma0", C.c_double * 6), ("pair_dsigma_dT", C.c_double * 6)]


class TcfStepInfo(C.Structure):
    _fields_ = [("cg_iters", C.c_int), ("refine_iters", C.c_int), ("p_relres", C.c_double),
                ("div_rel", C.c_double), ("sum_alpha", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("cfl_max", C.c_double), ("nonfinite", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["tcf_workspace_bytes", "tcf_init_grid", "tcf_init_grid_static", "tcf_set_fields", "tcf_get_fields",
           "tcf_get_pressure_history", "tcf_set_pressure_history", "tcf_set_species",
           "tcf_get_species", "tcf_set_phases", "tcf_get_phases", "tcf_step",
           "tcf_solve_pressure", "tcf_predictor", "tcf_apply_A", "tcf_step_backward", "tcf_step_keep",
           "tcf_step_backward_kept", "tcf_adjoint_transport",
           "tcf_adjoint_predictor", "tcf_profile", "tcf_profile_read", "tcf_destroy", "tcf_last_error"]

_lib = None


def load():
    """Load libtcf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the HIP library is required; there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, cfgp, st = C.c_void_p, C.POINTER(TcfConfig), C.c_int
    lib.tcf_workspace_bytes.restype = C.c_size_t
    lib.tcf_workspace_bytes.argtypes = [cfgp]
    lib.tcf_init_grid.restype = st
    lib.tcf_init_grid.argtypes = [cfgp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.tcf_init_grid_static.restype = st
    lib.tcf_init_grid_static.argtypes = [cfgp, vp, C.POINTER(vp)]
    lib.tcf_set_fields.restype = st
    lib.tcf_set_fields.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, vp]
    lib.tcf_get_fields.restype = st
    lib.tcf_get_fields.argtypes = [vp, C.POINTER(C.c_double), vp, vp, vp, vp, vp, vp]
    lib.tcf_get_pressure_history.restype = st
    lib.tcf_get_pressure_history.argtypes = [vp, vp, vp, C.POINTER(C.c_int)]
    lib.tcf_set_pressure_history.restype = st
    lib.tcf_set_pressure_history.argtypes = [vp, vp, vp, C.c_int]
    lib.tcf_set_species.restype = st
    lib.tcf_set_species.argtypes = [vp, vp]
    lib.tcf_get_species.restype = st
    lib.tcf_get_species.argtypes = [vp, vp]
    lib.tcf_set_phases.restype = C.c_int
    lib.tcf_set_phases.argtypes = [vp, vp, vp]
    lib.tcf_get_phases.restype = C.c_int
    lib.tcf_get_phases.argtypes = [vp, vp, vp]
    lib.tcf_step.restype = st
    lib.tcf_step.argtypes = [vp, C.c_double, C.c_int, C.POINTER(TcfStepInfo)]
    lib.tcf_solve_pressure.restype = st
    lib.tcf_solve_pressure.argtypes = [vp, vp, vp, C.POINTER(TcfStepInfo)]
    lib.tcf_predictor.restype = st
    lib.tcf_predictor.argtypes = [vp, C.c_double, vp, vp, vp]
    lib.tcf_apply_A.restype = st
    lib.tcf_apply_A.argtypes = [vp, vp, vp]
    pp = C.POINTER(vp)
    lib.tcf_step_backward.restype = st
    lib.tcf_step_backward.argtypes = [vp, C.c_double, C.c_double, pp, pp, pp, vp]
    lib.tcf_step_keep.restype = st
    lib.tcf_step_keep.argtypes = [vp, C.c_double, pp, vp]
    lib.tcf_step_backward_kept.restype = st
    lib.tcf_step_backward_kept.argtypes = [vp, C.c_double, C.c_double, pp, pp, pp, pp, pp, vp]
    lib.tcf_adjoint_transport.restype = st
    lib.tcf_adjoint_transport.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, vp, vp]
    lib.tcf_adjoint_predictor.restype = st
    lib.tcf_adjoint_predictor.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.tcf_profile.restype = st
    lib.tcf_profile.argtypes = [vp, C.c_char_p]
    lib.tcf_profile_read.restype = st
    lib.tcf_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_long)]
    lib.tcf_destroy.restype = None
    lib.tcf_destroy.argtypes = [vp]
    lib.tcf_last_error.restype = C.c_char_p
    lib.tcf_last_error.argtypes = []
    _lib = lib
    return lib


def make_config(c: dict, precision=None, flags=None) -> TcfConfig:
    o = TcfConfig()
    o.dim, o.nx, o.ny = c["dim"], c["nx"], c["ny"]
    o.nz = c["nz"] if c["dim"] == 3 else 1
    o.h = c["h"]
    o.precision = c.get("precision", 0) if precision is None else precision
    o.flags = c.get("flags", 0) if flags is None else flags
    o.rho1, o.rho2, o.mu1, o.mu2 = c["rho1"], c["rho2"], c["mu1"], c["mu2"]
    o.rhocp1, o.rhocp2, o.lambda1, o.lambda2 = c["rhocp1"], c["rhocp2"], c["lambda1"], c["lambda2"]
    o.sigma0, o.dsigma_dT, o.T0 = c["sigma0"], c["dsigma_dT"], c["T0"]
    for i in range(6):
        o.T_bc[i] = int(c["T_bc"][i])
        o.T_wall[i] = float(c["T_wall"][i])
    o.q_power, o.q_radius, o.q_x0 = c["q_power"], c["q_radius"], c["q_x0"]
    o.q_y0, o.q_vx, o.q_vy = c["q_y0"], c["q_vx"], c["q_vy"]
    o.weno_eps, o.normal_eps = c["weno_eps"], c["normal_eps"]
    o.p_rtol, o.p_maxit = c["p_rtol"], c["p_maxit"]
    o.inner_rtol, o.refine_maxit = c["inner_rtol"], c["refine_maxit"]
    o.mg_levels, o.mg_nu = c["mg_levels"], c["mg_nu"]
    o.p_extrapolate = int(c.get("p_extrapolate", 2))
    o.species = int(c.get("species", 0))
    o.dsigma_dc, o.c0 = float(c.get("dsigma_dc", 0.0)), float(c.get("c0", 0.0))
    o.integrator = int(c.get("integrator", 0))
    o.nphases = int(c.get("nphases", 0))
    for q, ph in enumerate(c.get("phases", [])[:2]):  # phases 3 and 4
        o.rho34[q], o.mu34[q] = ph["rho"], ph["mu"]
        o.rhocp34[q], o.lambda34[q] = ph["rhocp"], ph["lambda"]
    for q in range(6):  # pairs (1,2), (1,3), (1,4), (2,3), (2,4), (3,4)
        o.pair_sigma0[q] = float(c.get("pair_sigma0", [0.0] * 6)[q])
        o.pair_dsigma_dT[q] = float(c.get("pair_dsigma_dT", [0.0] * 6)[q])
    return o


def _ptr(x):
    if x is None:
        return None
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise TcfError(TCF_E_INVALID, "fields must be contiguous float64 CUDA tensors")
    return C.c_void_p(x.data_ptr())


def _check(st):
    if st != TCF_OK:
        raise TcfError(st, load().tcf_last_error().decode())


def workspace_bytes(c: dict, precision=None, flags=None) -> int:
    cfg = make_config(c, precision, flags)
    return load().tcf_workspace_bytes(C.byref(cfg))


class Grid:
    """One simulation state on one GPU (device memory owned by torch)."""

    def __init__(self, c: dict, precision=None, flags=None, device="cuda", static=False):
        """static=True: the workspace is the library's fixed per-GPU array
        (tcf_init_grid_static), nothing is allocated for it."""
        lib = load()
        self.c = dict(c)
        self.cfg = make_config(c, precision, flags)
        nbytes = lib.tcf_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise TcfError(TCF_E_INVALID, "invalid configuration")
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        if static:
            self._ws_raw, self.ws_ptr, self.ws_bytes = None, None, nbytes
            with torch.cuda.device(self.device):
                _check(lib.tcf_init_grid_static(C.byref(self.cfg), C.c_void_p(self.stream.cuda_stream),
                                                C.byref(h)))
        else:
            raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-raw.data_ptr()) % 256
            self._ws_raw = raw
            self.ws_ptr = raw.data_ptr() + off
            self.ws_bytes = nbytes
            _check(lib.tcf_init_grid(C.byref(self.cfg), C.c_void_p(self.ws_ptr), C.c_size_t(nbytes),
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        nx, ny, nz = self.cfg.nx, self.cfg.ny, self.cfg.nz
        self.shapes = dict(cell=(nz, ny, nx), u=(nz, ny, nx + 1), v=(nz, ny + 1, nx),
                           w=(nz + 1, ny, nx) if self.cfg.dim == 3 else None)

    def _t(self, x):
        if x is None:
            return None
        if not torch.is_tensor(x):
            x = torch.as_tensor(x)
        return x.to(device=self.device, dtype=torch.float64).contiguous()

    def set_fields(self, t, alpha, T, u, v, w=None, p=None):
        ts = [self._t(x) for x in (alpha, T, u, v, w, p)]
        self._keep = ts
        _check(load().tcf_set_fields(self.h, C.c_double(t), *[_ptr(x) for x in ts]))

    def set_state(self, st: dict, t=0.0):
        """Fields (and, when given, the species, the phases and the previous
        pressure of the extrapolated guess, as get_fields returns them)."""
        self.set_fields(t, st["alpha"], st["T"], st["u"], st["v"], st.get("w"), st.get("p"))
        if st.get("p_held"):
            p1, p2 = self._t(st.get("p_prev")), self._t(st.get("p_prev2"))
            self._keep_pp = (p1, p2)
            _check(load().tcf_set_pressure_history(self.h, _ptr(p1), _ptr(p2), C.c_int(st["p_held"])))
        if st.get("c") is not None:
            self.set_species(st["c"])
        if st.get("alpha3") is not None:
            self.set_phases(st["alpha3"], st.get("alpha4"))

    def set_phases(self, a3, a4=None):
        """Fractions of phases 3 (and 4) of an N-phase grid."""
        t3 = self._t(a3)
        t4 = None if a4 is None else self._t(a4)
        self._keep_ph = (t3, t4)
        _check(load().tcf_set_phases(self.h, _ptr(t3), _ptr(t4)))

    def get_phases(self):
        """(alpha3, alpha4 or None) of an N-phase grid."""
        shp = self.shapes["cell"]
        a3 = torch.empty(shp, dtype=torch.float64, device=self.device)
        a4 = torch.empty(shp, dtype=torch.float64, device=self.device) if self.c.get("nphases", 0) == 4 else None
        _check(load().tcf_get_phases(self.h, _ptr(a3), _ptr(a4)))
        return a3, a4

    def set_species(self, c):
        ct = self._t(c)
        self._keep_c = ct
        _check(load().tcf_set_species(self.h, _ptr(ct)))

    def get_species(self):
        out = torch.empty(self.shapes["cell"], dtype=torch.float64, device=self.device)
        _check(load().tcf_get_species(self.h, _ptr(out)))
        return out

    def get_fields(self, history=True) -> dict:
        """Copies of the grid's fields (fresh tensors); with history, also the
        previous pressures the extrapolated initial guess holds."""
        s = self.shapes
        out = {k: torch.empty(s[k if k in ("u", "v", "w") else "cell"], dtype=torch.float64, device=self.device)
               for k in ("alpha", "T", "u", "v", "p")}
        out["w"] = torch.empty(s["w"], dtype=torch.float64, device=self.device) if s["w"] else None
        t = C.c_double()
        _check(load().tcf_get_fields(self.h, C.byref(t), _ptr(out["alpha"]), _ptr(out["T"]), _ptr(out["u"]),
                                     _ptr(out["v"]), _ptr(out["w"]), _ptr(out["p"])))
        out["t"] = t.value
        # the previous pressures of the extrapolated initial guess, if the
        # grid keeps them (one-solve integrator) and holds any
        n = 0
        p1 = p2 = None
        if history and self.cfg.p_extrapolate > 0 and self.cfg.integrator == 0:
            p1 = torch.empty(s["cell"], dtype=torch.float64, device=self.device)
            p2 = torch.empty(s["cell"], dtype=torch.float64, device=self.device)
            held = C.c_int(0)
            _check(load().tcf_get_pressure_history(self.h, _ptr(p1), _ptr(p2), C.byref(held)))
            n = held.value
        out["p_held"] = n
        out["p_prev"] = p1 if n >= 1 else None
        out["p_prev2"] = p2 if n >= 2 else None
        return out

    def step(self, dt, nsteps=1, info=True, check=True):
        inf = TcfStepInfo()
        st = load().tcf_step(self.h, C.c_double(dt), C.c_int(nsteps), C.byref(inf) if info else None)
        if check and st not in (TCF_OK,):
            raise TcfError(st, load().tcf_last_error().decode())
        d = inf.as_dict() if info else {}
        d["status"] = st
        return d

    def solve_pressure(self, rhs, p0=None):
        rhs = self._t(rhs)
        p = torch.zeros_like(rhs) if p0 is None else self._t(p0).clone()
        inf = TcfStepInfo()
        st = load().tcf_solve_pressure(self.h, _ptr(rhs), _ptr(p), C.byref(inf))
        if st not in (TCF_OK, TCF_E_NOT_CONVERGED):
            raise TcfError(st, load().tcf_last_error().decode())
        return p, st, inf.as_dict()

    def predictor(self, dt):
        s = self.shapes
        us = torch.empty(s["u"], dtype=torch.float64, device=self.device)
        vs = torch.empty(s["v"], dtype=torch.float64, device=self.device)
        ws = torch.empty(s["w"], dtype=torch.float64, device=self.device) if s["w"] else None
        _check(load().tcf_predictor(self.h, C.c_double(dt), _ptr(us), _ptr(vs), _ptr(ws)))
        return us, vs, ws

    def apply_A(self, x):
        x = self._t(x)
        y = torch.empty_like(x)
        _check(load().tcf_apply_A(self.h, _ptr(x), _ptr(y)))
        return y

    # ---- adjoint -------------------------------------------------------------
    def _empty(self, kind):
        shp = self.shapes[kind]
        return None if shp is None else torch.empty(shp, dtype=torch.float64, device=self.device)

    def step_backward(self, t_n, dt, state_n: dict, adj_np1: dict, sbar):
        """One adjoint step: returns dL/d(alpha, T, u, v, w) at step n and adds
        dL/d(dsigma_dT) of this step into the 0-d device tensor sbar."""
        keys = ("alpha", "T", "u", "v", "w")
        st = [self._t(state_n.get(k)) for k in keys] + [self._t(state_n.get("p"))]
        ad = [self._t(adj_np1.get(k)) if adj_np1.get(k) is not None else
              (torch.zeros(self.shapes[("cell" if k in ("alpha", "T") else k)], dtype=torch.float64,
                           device=self.device) if (k != "w" or self.shapes["w"]) else None) for k in keys]
        out = [self._empty("cell"), self._empty("cell"), self._empty("u"), self._empty("v"), self._empty("w")]
        arr6 = (C.c_void_p * 6)(*[None if x is None else x.data_ptr() for x in st])
        arr5a = (C.c_void_p * 5)(*[None if x is None else x.data_ptr() for x in ad])
        arr5o = (C.c_void_p * 5)(*[None if x is None else x.data_ptr() for x in out])
        assert sbar.dtype == torch.float64 and sbar.is_cuda and sbar.numel() == 1
        self._keep = (st, ad)
        _check(load().tcf_step_backward(self.h, C.c_double(t_n), C.c_double(dt), arr6, arr5a, arr5o,
                                        C.c_void_p(sbar.data_ptr())))
        return dict(zip(keys, out))

    def step_keep(self, dt, p_np1=None):
        """One forward step (as step(dt, 1)) that also returns the transport's
        stage values (alpha1, T1, alpha2, T2) for step_backward_kept; with
        p_np1 (the pressure an earlier run of this step returned) the step
        takes it instead of solving for it."""
        stages = [self._empty("cell") for _ in range(4)]
        arr = (C.c_void_p * 4)(*[x.data_ptr() for x in stages])
        pp = self._t(p_np1)
        self._keep = (pp,)
        _check(load().tcf_step_keep(self.h, C.c_double(dt), arr, _ptr(pp)))
        return stages

    def get_pressure(self):
        """A copy of the grid's pressure (FP64, cell layout)."""
        p = self._empty("cell")
        _check(load().tcf_get_fields(self.h, None, None, None, None, None, None, _ptr(p)))
        return p

    def step_backward_kept(self, t_n, dt, state_n: dict, stages, state_np1: dict, adj_np1: dict, sbar):
        """step_backward with the forward step's intermediates supplied: the
        stages from step_keep of this step and alpha, T, p of step n+1."""
        keys = ("alpha", "T", "u", "v", "w")
        st = [self._t(state_n.get(k)) for k in keys] + [self._t(state_n.get("p"))]
        stg = [self._t(x) for x in stages]
        nxt = [self._t(state_np1[k]) for k in ("alpha", "T", "p")]
        ad = [self._t(adj_np1.get(k)) if adj_np1.get(k) is not None else
              (torch.zeros(self.shapes[("cell" if k in ("alpha", "T") else k)], dtype=torch.float64,
                           device=self.device) if (k != "w" or self.shapes["w"]) else None) for k in keys]
        out = [self._empty("cell"), self._empty("cell"), self._empty("u"), self._empty("v"), self._empty("w")]
        arr6 = (C.c_void_p * 6)(*[None if x is None else x.data_ptr() for x in st])
        arr4 = (C.c_void_p * 4)(*[x.data_ptr() for x in stg])
        arr3 = (C.c_void_p * 3)(*[x.data_ptr() for x in nxt])
        arr5a = (C.c_void_p * 5)(*[None if x is None else x.data_ptr() for x in ad])
        arr5o = (C.c_void_p * 5)(*[None if x is None else x.data_ptr() for x in out])
        assert sbar.dtype == torch.float64 and sbar.is_cuda and sbar.numel() == 1
        self._keep = (st, stg, nxt, ad)
        _check(load().tcf_step_backward_kept(self.h, C.c_double(t_n), C.c_double(dt), arr6, arr4, arr3, arr5a,
                                             arr5o, C.c_void_p(sbar.data_ptr())))
        return dict(zip(keys, out))

    def adjoint_transport(self, dt, ab, Tb):
        ab, Tb = self._t(ab), self._t(Tb)
        ao, To = self._empty("cell"), self._empty("cell")
        ub, vb, wb = self._empty("u"), self._empty("v"), self._empty("w")
        _check(load().tcf_adjoint_transport(self.h, C.c_double(dt), _ptr(ab), _ptr(Tb), _ptr(ao), _ptr(To),
                                            _ptr(ub), _ptr(vb), _ptr(wb)))
        return dict(alpha=ao, T=To, u=ub, v=vb, w=wb)

    def adjoint_predictor(self, dt, usb, vsb, wsb=None):
        usb, vsb, wsb = self._t(usb), self._t(vsb), self._t(wsb)
        ab, Tb = self._empty("cell"), self._empty("cell")
        ub, vb, wb = self._empty("u"), self._empty("v"), self._empty("w")
        sb = torch.empty((), dtype=torch.float64, device=self.device)
        _check(load().tcf_adjoint_predictor(self.h, C.c_double(dt), _ptr(usb), _ptr(vsb), _ptr(wsb), _ptr(ab),
                                            _ptr(Tb), _ptr(ub), _ptr(vb), _ptr(wb), _ptr(sb)))
        return dict(alpha=ab, T=Tb, u=ub, v=vb, w=wb, dsigma_dT=sb)

    def profile(self, family):
        """Start timing the launches of one kernel family (None stops)."""
        _check(load().tcf_profile(self.h, None if family is None else family.encode()))

    def profile_read(self):
        ms, n = C.c_double(), C.c_long()
        _check(load().tcf_profile_read(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().tcf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
class TcfRollout(torch.autograd.Function):
    """n steps of the projection step as a differentiable function of the
    surface-tension slope s = dsigma/dT (0-d tensor) and the initial
    temperature field T0.  alpha0 and the initial velocity are fixed inputs.

    forward stores a checkpoint of the state every k steps and every step's
    pressure (nx*ny*nz FP64 values per step); backward replays each segment
    from its checkpoint with tcf_step_keep given those pressures (no solve;
    the replayed states are bitwise the forward's), keeping the segment's
    states and each step's transport stages, and runs tcf_step_backward_kept
    through it in reverse.  Outputs: final (alpha, T, u, v, w) (w is an empty
    tensor in 2D)."""

    @staticmethod
    def forward(ctx, s, T0, cfg, alpha0, u0, v0, w0, nsteps, k, *start):
        """start: optional (t0, p0), the time of the initial state (the
        moving heat source's position) and its pressure (the first solve's
        initial guess); default (0, zero pressure)."""
        c = dict(cfg)
        c["dsigma_dT"] = float(s)
        g = Grid(c, precision=TCF_FP64, flags=TCF_WITH_ADJOINT, device=T0.device)
        dt = c["dt"]
        t0 = float(start[0]) if len(start) > 0 else 0.0
        p0 = start[1] if len(start) > 1 else None
        ctx.n_start = len(start)
        g.set_fields(t0, alpha0, T0, u0, v0, w0, p0)
        ckpt = []
        pres = [None] * (nsteps + 1)  # every step's pressure: the replay takes it instead of solving
        for n in range(nsteps):
            if n % k == 0:
                ckpt.append((n, g.get_fields()))
            g.step(dt, 1, info=False)
            pres[n + 1] = g.get_pressure()
        out = g.get_fields()
        ctx.grid, ctx.ckpt, ctx.nsteps, ctx.dt, ctx.pres = g, ckpt, nsteps, dt, pres
        ctx.has_w = out["w"] is not None
        w = out["w"] if ctx.has_w else torch.empty(0, dtype=torch.float64, device=T0.device)
        return out["alpha"], out["T"], out["u"], out["v"], w

    @staticmethod
    def backward(ctx, ga, gT, gu, gv, gw):
        g, dt = ctx.grid, ctx.dt
        dev = g.device
        lam = dict(alpha=ga, T=gT, u=gu, v=gv, w=gw if ctx.has_w else None)
        for key, shp in (("alpha", "cell"), ("T", "cell"), ("u", "u"), ("v", "v"), ("w", "w")):
            if lam[key] is None and g.shapes[shp] is not None:
                lam[key] = torch.zeros(g.shapes[shp], dtype=torch.float64, device=dev)
            elif lam[key] is not None:
                lam[key] = lam[key].contiguous()
        sbar = torch.zeros((), dtype=torch.float64, device=dev)
        bounds = [n for n, _ in ctx.ckpt] + [ctx.nsteps]
        for seg in reversed(range(len(ctx.ckpt))):
            n0, st0 = ctx.ckpt[seg]
            n1 = bounds[seg + 1]
            # replay the segment, keeping every state and every step's stages
            g.set_state(st0, st0["t"])  # with the pressure history, so the replay repeats the forward
            states, stages = [], []
            for n in range(n0, n1):
                states.append(g.get_fields(history=False))
                stages.append(g.step_keep(dt, ctx.pres[n + 1]))
            states.append(g.get_fields(history=False))  # the state after the segment's last step
            for n in reversed(range(n0, n1)):
                st, nxt = states[n - n0], states[n - n0 + 1]
                lam = g.step_backward_kept(st["t"], dt, st, stages[n - n0], nxt, lam, sbar)
                stages[n - n0] = None
                ctx.pres[n + 1] = None
        return (sbar, lam["T"], None, None, None, None, None, None, None) + (None,) * ctx.n_start
