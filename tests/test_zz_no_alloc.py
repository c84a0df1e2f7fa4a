"""tcf_init_grid_static: the grid on the library's fixed per-GPU workspace
(for callers that cannot allocate) gives the results of the same grid on a
caller workspace, on two grids in a row (the second smaller, reusing the
array with the first one's contents in it); oversize configurations and a
second open grid on the same GPU are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2209_09671_amd import inputs as I
from paper_2209_09671_amd import tcf

pytestmark = pytest.mark.gpu


def run(c, st, precision, nsteps, static):
    print(f"[gpu] no-alloc {c['nx']}x{c['ny']}x{c['nz']} precision={precision} static={static} "
          f"workspace={tcf.workspace_bytes(c, precision)}", flush=True)
    g = tcf.Grid(c, precision=precision, static=static)
    g.set_state(st)
    info = g.step(c["dt"], nsteps)
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in g.get_fields().items()}
    torch.cuda.synchronize()
    g.close()
    return out, info


def compare(a, b, keys):
    worst = 0.0
    for k in keys:
        x, y = a[k], b[k]
        worst = max(worst, float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)))
    return worst


def test_static_workspace_matches_caller_workspace_two_calls():
    # first: a 3D melt pool in FP32 with FP64 refinement, ragged in every dimension
    c1 = dict(I.custom(I.config(2), nx=70, ny=40, nz=36), p_rtol=1e-10)
    assert tcf.workspace_bytes(c1, 1) <= (128 << 20)
    st1 = I.initial_state(c1)
    ref1, i1 = run(c1, st1, 1, 4, False)
    got1, j1 = run(c1, st1, 1, 4, True)
    keys3 = ("alpha", "T", "u", "v", "w", "p")
    e1 = compare(got1, ref1, keys3)
    print("[no-alloc] melt pool: max rel. difference", e1, "cg", i1["cg_iters"], j1["cg_iters"], flush=True)
    assert e1 <= 1e-12 and j1["status"] == 0
    # second, smaller: a 2D droplet in FP64 on the array the first grid left
    c2 = I.custom(I.config(0), nx=40, ny=32)
    st2 = I.initial_state(c2)
    ref2, _ = run(c2, st2, 0, 5, False)
    got2, _ = run(c2, st2, 0, 5, True)
    e2 = compare(got2, ref2, ("alpha", "T", "u", "v", "p"))
    print("[no-alloc] droplet: max rel. difference", e2, flush=True)
    assert e2 <= 1e-12


def test_static_workspace_refusals():
    lib = tcf.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = tcf.make_config(I.config(4), 1)
    h = C.c_void_p()
    assert lib.tcf_init_grid_static(C.byref(big), stream, C.byref(h)) == tcf.TCF_E_WORKSPACE
    assert not h.value
    small = tcf.make_config(I.config(0), 0)
    h1, h2 = C.c_void_p(), C.c_void_p()
    assert lib.tcf_init_grid_static(C.byref(small), stream, C.byref(h1)) == tcf.TCF_OK
    assert lib.tcf_init_grid_static(C.byref(small), stream, C.byref(h2)) == tcf.TCF_E_STATE
    lib.tcf_destroy(h1)
    assert lib.tcf_init_grid_static(C.byref(small), stream, C.byref(h2)) == tcf.TCF_OK
    lib.tcf_destroy(h2)
    assert lib.tcf_init_grid_static(None, stream, C.byref(h2)) == tcf.TCF_E_INVALID
