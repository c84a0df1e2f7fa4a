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
                ("refine_maxit", C.c_int), ("mg_levels", C.c_int), ("mg_nu", C.c_int)]


class TcfStepInfo(C.Structure):
    _fields_ = [("cg_iters", C.c_int), ("refine_iters", C.c_int), ("p_relres", C.c_double),
                ("div_rel", C.c_double), ("sum_alpha", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("cfl_max", C.c_double), ("nonfinite", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["tcf_workspace_bytes", "tcf_init_grid", "tcf_set_fields", "tcf_get_fields", "tcf_step",
           "tcf_solve_pressure", "tcf_predictor", "tcf_apply_A", "tcf_profile", "tcf_profile_read",
           "tcf_destroy", "tcf_last_error"]

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
    lib.tcf_set_fields.restype = st
    lib.tcf_set_fields.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, vp]
    lib.tcf_get_fields.restype = st
    lib.tcf_get_fields.argtypes = [vp, C.POINTER(C.c_double), vp, vp, vp, vp, vp, vp]
    lib.tcf_step.restype = st
    lib.tcf_step.argtypes = [vp, C.c_double, C.c_int, C.POINTER(TcfStepInfo)]
    lib.tcf_solve_pressure.restype = st
    lib.tcf_solve_pressure.argtypes = [vp, vp, vp, C.POINTER(TcfStepInfo)]
    lib.tcf_predictor.restype = st
    lib.tcf_predictor.argtypes = [vp, C.c_double, vp, vp, vp]
    lib.tcf_apply_A.restype = st
    lib.tcf_apply_A.argtypes = [vp, vp, vp]
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

    def __init__(self, c: dict, precision=None, flags=None, device="cuda"):
        lib = load()
        self.c = dict(c)
        self.cfg = make_config(c, precision, flags)
        nbytes = lib.tcf_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise TcfError(TCF_E_INVALID, "invalid configuration")
        self.device = torch.device(device)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws_ptr = raw.data_ptr() + off
        self.ws_bytes = nbytes
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
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
        self.set_fields(t, st["alpha"], st["T"], st["u"], st["v"], st.get("w"), st.get("p"))

    def get_fields(self) -> dict:
        s = self.shapes
        out = {k: torch.empty(s[k if k in ("u", "v", "w") else "cell"], dtype=torch.float64, device=self.device)
               for k in ("alpha", "T", "u", "v", "p")}
        out["w"] = torch.empty(s["w"], dtype=torch.float64, device=self.device) if s["w"] else None
        t = C.c_double()
        _check(load().tcf_get_fields(self.h, C.byref(t), _ptr(out["alpha"]), _ptr(out["T"]), _ptr(out["u"]),
                                     _ptr(out["v"]), _ptr(out["w"]), _ptr(out["p"])))
        out["t"] = t.value
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
