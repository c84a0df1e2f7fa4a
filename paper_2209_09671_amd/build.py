"""Build libtcf.so (HIP kernels + host library + C ABI) for gfx950 in-tree."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtcf.so")
SOURCES = ["tcf_kernels.hip", "tcf_transport.hip", "tcf_predictor.hip", "tcf_fine.hip", "tcf_adjoint.hip",
           "tcf_nphase.hip", "tcf_host.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # keep the compiler from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, defines=(), out: str | None = None) -> str:
    """Compile every source and link libtcf.so (or `out`); `defines` are
    extra -D options (tuning variants)."""
    lib = out or LIB
    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(os.path.dirname(lib), os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        try:
            subprocess.run(cmd, check=True, stderr=subprocess.PIPE if not verbose else None, text=True)
        except subprocess.CalledProcessError as e:
            if e.stderr:
                sys.stderr.write(e.stderr)
            raise
        return obj

    # the sources compile independently: one hipcc per source, side by side
    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", "-o", tmp] + objs, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
