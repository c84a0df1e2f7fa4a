"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/tcf.h, sizes workspaces, and rejects bad
arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2209_09671_amd import inputs as I
from paper_2209_09671_amd import tcf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tcf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tcf_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_lists_the_binding_exports():
    assert set(declared_symbols()) == set(tcf.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = tcf.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("idx", [0, 1, 2, 3, 4])
def test_workspace_sizes(idx):
    c = I.config(idx)
    n64 = tcf.workspace_bytes(c, precision=0)
    n32 = tcf.workspace_bytes(c, precision=1)
    N = c["nx"] * c["ny"] * c["nz"]
    assert n64 > 20 * 8 * N and n32 > 20 * 4 * N
    # the 256^3 box fits comfortably in one GPU's 288 GB
    assert n64 < 60 * 8 * N + (1 << 20)


@pytest.mark.parametrize("bad", [dict(dim=4), dict(nx=2), dict(nz=3), dict(h=-1.0), dict(precision=7),
                                 dict(rho1=0.0), dict(p_maxit=0), dict(mg_nu=0), dict(flags=8),
                                 dict(weno_eps=0.0)])
def test_invalid_configs_rejected(bad):
    c = dict(I.config(0))
    if bad.get("nz") == 3:
        c = dict(I.config(3))
    c.update(bad)
    assert tcf.workspace_bytes(c) == 0
    lib = tcf.load()
    cfg = tcf.make_config(c)
    h = C.c_void_p()
    st = lib.tcf_init_grid(C.byref(cfg), C.c_void_p(256), C.c_size_t(1 << 30), None, C.byref(h))
    assert st == tcf.TCF_E_INVALID and h.value is None
    assert lib.tcf_last_error().decode()


def test_workspace_errors_before_device_use():
    lib = tcf.load()
    cfg = tcf.make_config(I.config(0))
    h = C.c_void_p()
    assert lib.tcf_init_grid(C.byref(cfg), None, C.c_size_t(1 << 30), None, C.byref(h)) == tcf.TCF_E_WORKSPACE
    assert lib.tcf_init_grid(C.byref(cfg), C.c_void_p(256 + 8), C.c_size_t(1 << 30), None,
                             C.byref(h)) == tcf.TCF_E_WORKSPACE
    assert lib.tcf_init_grid(C.byref(cfg), C.c_void_p(256), C.c_size_t(16), None, C.byref(h)) == tcf.TCF_E_WORKSPACE
    assert b"too small" in lib.tcf_last_error()


def test_null_handles_rejected():
    lib = tcf.load()
    assert lib.tcf_step(None, C.c_double(1e-3), 1, None) == tcf.TCF_E_INVALID
    assert lib.tcf_set_fields(None, C.c_double(0.0), None, None, None, None, None, None) == tcf.TCF_E_INVALID
    assert lib.tcf_solve_pressure(None, None, None, None) == tcf.TCF_E_INVALID
    lib.tcf_destroy(None)


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(tcf, "_lib", None)
    monkeypatch.setattr(tcf, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        tcf.load()


def test_species_workspace_and_validation():
    """A species adds its field and two RK3 stage arrays to the workspace;
    species must be 0/1 and is not combined with the adjoint."""
    c = I.config(3)
    N = c["nx"] * c["ny"] * c["nz"]
    cs = I.with_species(c, -0.2)
    assert tcf.workspace_bytes(cs, precision=0) - tcf.workspace_bytes(c, precision=0) >= 3 * 8 * N
    assert tcf.workspace_bytes(cs, precision=1) - tcf.workspace_bytes(c, precision=1) >= 3 * 4 * N
    assert tcf.workspace_bytes(dict(cs, species=2)) == 0
    assert tcf.workspace_bytes(dict(cs, dsigma_dc=float("nan"))) == 0
    assert tcf.workspace_bytes(cs, precision=0, flags=tcf.TCF_WITH_ADJOINT) == 0
    assert tcf.workspace_bytes(c, precision=0, flags=tcf.TCF_WITH_ADJOINT) > 0


def test_time_accurate_integrator_workspace_and_validation():
    """Integrator 1 keeps the step's base velocity (three FP64 face arrays);
    the integrator must be 0/1 and 1 is not combined with the adjoint."""
    c = dict(I.config(3), p_extrapolate=0)
    nf = 3 * (c["nx"] + 1) * c["ny"] * c["nz"]
    for prec in (0, 1):
        extra = tcf.workspace_bytes(dict(c, integrator=1), precision=prec) - tcf.workspace_bytes(c, precision=prec)
        assert nf * 8 <= extra < nf * 8 + 4096
    assert tcf.workspace_bytes(dict(c, integrator=2)) == 0
    assert tcf.workspace_bytes(dict(c, integrator=1), precision=0, flags=tcf.TCF_WITH_ADJOINT) == 0
    assert tcf.workspace_bytes(dict(c, integrator=0), precision=0, flags=tcf.TCF_WITH_ADJOINT) > 0


def test_nphase_workspace_and_validation():
    """N phases add the extra fractions with their RK3 stages, the mixture,
    per-pair sigma*kappa and the face force; nphases must be 0, 2, 3 or 4,
    phase materials physical, and N phases exclude species, integrator 1 and
    the adjoint."""
    c = I.config(3)
    N = c["nx"] * c["ny"] * c["nz"]
    c3 = I.droplet_phases(c, "lens")
    c4 = I.droplet_phases4(c, "layers4")
    b2 = tcf.workspace_bytes(c, precision=0)
    b3 = tcf.workspace_bytes(c3, precision=0)
    b4 = tcf.workspace_bytes(c4, precision=0)
    assert b3 - b2 >= (3 + 6 + 3 + 3) * 8 * N
    assert b4 - b3 >= (3 + 3) * 8 * N
    assert tcf.workspace_bytes(c3, precision=1) - tcf.workspace_bytes(c, precision=1) >= (3 + 6 + 3 + 3) * 4 * N
    assert tcf.workspace_bytes(dict(c3, nphases=5)) == 0
    assert tcf.workspace_bytes(dict(c3, nphases=1)) == 0
    bad = dict(c3, phases=[dict(c3["phases"][0], rho=-1.0)])
    assert tcf.workspace_bytes(bad) == 0
    nan_pair = dict(c3, pair_sigma0=[float("nan")] + c3["pair_sigma0"][1:])
    assert tcf.workspace_bytes(nan_pair) == 0
    assert tcf.workspace_bytes(dict(c3, integrator=1)) == 0
    assert tcf.workspace_bytes(I.with_species(c3, -0.1)) == 0
    assert tcf.workspace_bytes(c3, precision=0, flags=tcf.TCF_WITH_ADJOINT) == 0
    assert tcf.workspace_bytes(dict(c, nphases=2)) == b2


def test_phase_entry_points_reject_null():
    lib = tcf.load()
    assert lib.tcf_set_phases(None, None, None) == tcf.TCF_E_INVALID
    assert lib.tcf_get_phases(None, None, None) == tcf.TCF_E_INVALID


def test_species_entry_points_reject_null():
    lib = tcf.load()
    assert lib.tcf_set_species(None, None) == tcf.TCF_E_INVALID
    assert lib.tcf_get_species(None, None) == tcf.TCF_E_INVALID


def test_pressure_extrapolation_workspace_and_validation():
    """p_extrapolate = K keeps the K previous pressures (FP64 cell arrays) on
    grids whose integrator solves once per step (also grids made for the
    adjoint), and K + 1 pressures per stage with integrator 1; it must be 0,
    1 or 2."""
    c = I.config(3)
    N = c["nx"] * c["ny"] * c["nz"]
    off = dict(c, p_extrapolate=0)
    for K in (1, 2):
        on = dict(c, p_extrapolate=K)
        for prec in (0, 1):
            d = tcf.workspace_bytes(on, precision=prec) - tcf.workspace_bytes(off, precision=prec)
            assert 8 * K * N <= d < 8 * K * N + 4096
        d1 = tcf.workspace_bytes(dict(on, integrator=1)) - tcf.workspace_bytes(dict(off, integrator=1))
        assert 8 * 3 * (K + 1) * N <= d1 < 8 * 3 * (K + 1) * N + 8192  # per stage K + 1 pressures
        da = (tcf.workspace_bytes(on, precision=0, flags=tcf.TCF_WITH_ADJOINT)
              - tcf.workspace_bytes(off, precision=0, flags=tcf.TCF_WITH_ADJOINT))
        assert 8 * K * N <= da < 8 * K * N + 4096
    assert tcf.workspace_bytes(dict(c, p_extrapolate=3)) == 0
    assert tcf.workspace_bytes(dict(c, p_extrapolate=-1)) == 0


def test_pressure_history_entry_points_reject_null():
    lib = tcf.load()
    assert lib.tcf_get_pressure_history(None, None, None, None) == tcf.TCF_E_INVALID
    assert lib.tcf_set_pressure_history(None, None, None, 0) == tcf.TCF_E_INVALID
