"""Build libgt4mi.so: hipcc for gfx950, one object per source, in parallel.

Run as ``python -m paper_2311_08322_amd.build_lib`` or through
``__graft_entry__.build()``.  Objects go to ``paper_2311_08322_amd/_build``;
the shared library lands next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgt4mi.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
]
UNROLL = ["-mllvm", "-pragma-unroll-threshold=1000000", "-mllvm", "-unroll-max-upperbound=1000"]


def _units():
    """(source, object name, extra flags) of every compilation, slowest first."""
    u = []
    for t, cols in (("double", (1, 2)), ("float", (1,))):
        for ti in (64, 32, 16):
            for col in cols:
                u.append(("k_step_inst.hip", f"step_{t}_{ti}_c{col}",
                          [f"-DGT4MI_T={t}", f"-DGT4MI_TI={ti}", f"-DGT4MI_COL={col}", *UNROLL]))
        for adj in ("false", "true"):
            u.append(("k_step_inst.hip", f"colsplit_{t}_{adj}",
                      [f"-DGT4MI_T={t}", "-DGT4MI_COLSPLIT", f"-DGT4MI_ADJ={adj}", *UNROLL]))
        for ti in (64, 32, 16):
            u.append(("k_step_inst.hip", f"split_{t}_{ti}",
                      [f"-DGT4MI_T={t}", f"-DGT4MI_TI={ti}", "-DGT4MI_SPLIT",
                       *(["-DGT4MI_SPLIT_LONG"] if t == "double" else []), *UNROLL]))
            u.append(("k_step_inst.hip", f"splitvar_{t}_{ti}",
                      [f"-DGT4MI_T={t}", f"-DGT4MI_TI={ti}", "-DGT4MI_SPLIT", "-DGT4MI_VAR", *UNROLL]))
            # 128-column tiles (256-lane workgroups) of the two-ended step
            for var in ([], ["-DGT4MI_VAR"]):
                u.append(("k_step_inst.hip", f"split{'var' if var else ''}128_{t}_{ti}",
                          [f"-DGT4MI_T={t}", f"-DGT4MI_TI={ti}", "-DGT4MI_SPLIT", "-DGT4MI_SPLIT_NT=128", *var,
                           *UNROLL]))
        for col in cols:
            u.append(("k_step_inst.hip", f"vadv_{t}_c{col}",
                      [f"-DGT4MI_T={t}", "-DGT4MI_VADV", f"-DGT4MI_COL={col}", *UNROLL]))
            u.append(("k_vadj_inst.hip", f"vadj_{t}_c{col}", [f"-DGT4MI_T={t}", f"-DGT4MI_COL={col}", *UNROLL]))
        u.append(("k_batched.hip", f"batched_{t}",
                  [f"-DGT4MI_T={t}", *(["-DGT4MI_UPLOAD"] if t == "float" else ["-DGT4MI_BATCHED_LONG"]),
                   *UNROLL]))
    for src in ("k_adjoint.hip", "k_halo.hip", "k_hdiff.hip", "k_param.hip", "k_plain.hip", "k_step.hip", "noalloc.hip",
                "api.cpp", "tune.cpp",
                "graph.cpp", "batched.cpp", "param.cpp"):
        u.append((src, os.path.splitext(src)[0], []))
    return u


def _compile(unit, build_dir=BUILD, defines=()) -> str:
    src, name, extra = unit
    obj = os.path.join(build_dir, name + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *defines, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stderr[-6000:]}")
    return f"{name}: {time.time() - t:.1f}s"


def build(verbose: bool = True, jobs: int | None = None, out: str = LIB, build_dir: str = BUILD,
          defines=()) -> str:
    """Compile every unit and link `out`.  `defines` (e.g. -DGT4MI_PD=4)
    select compile-time variants of the kernels for tuning experiments."""
    os.makedirs(build_dir, exist_ok=True)
    units = _units()
    jobs = jobs or max(1, min(len(units), os.cpu_count() or 4))
    with cf.ThreadPoolExecutor(jobs) as ex:
        for msg in ex.map(lambda u: _compile(u, build_dir, tuple(defines)), units):
            if verbose:
                print("  built", msg, flush=True)
    objs = [os.path.join(build_dir, name + ".o") for _, name, _ in units]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    t0 = time.time()
    print(build(), f"{time.time() - t0:.1f}s")
    sys.exit(0)
