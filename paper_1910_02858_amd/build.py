"""Build libdgsem.so in-tree with hipcc for gfx950.

The kernel source is compiled once per polynomial degree (``-DDG_ONLY_N=k``) so the
template instantiations build in parallel, plus once for the degree-independent kernels.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdgsem.so")
BUILD = os.path.join(HERE, "_build")
NMAX = 8

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    # a*b+c is fused where one source expression says so, never across statements: every kernel
    # that instantiates the same per-element code then rounds alike, whatever the surrounding
    # code (the one-mesh, batched and gradient-keeping entry points agree bit for bit)
    "-ffp-contract=on",
]


HOST_SOURCES = ("dg_host.cpp", "dg_batch.cpp", "dg_meshio.cpp")


def _host_obj(src: str) -> str:
    return "host_" + src.split(".")[0] + ".o"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def kernel_units():
    units = [("dg_kernels.hip", [], "k_common.o")]
    for n in range(1, NMAX + 1):
        units.append(("dg_kernels.hip", [f"-DDG_ONLY_N={n}"], f"k_n{n}.o"))
    units.append(("dg_kernels.hip", ["-DDG_FUSED_BATCH"], "k_fused.o"))
    units.append(("dg_static.hip", [], "dg_static.o"))
    units.append(("dg_vjp.hip", [], "dg_vjp_common.o"))
    for n in range(1, NMAX + 1):
        units.append(("dg_vjp.hip", [f"-DDG_ONLY_N={n}"], f"dg_vjp_n{n}.o"))
    return units


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = kernel_units()
    cmds = []
    for src, defs, obj in units:
        cmds.append([HIPCC, *COMMON, *defs, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)])
    for src in HOST_SOURCES:
        cmds.append([HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, _host_obj(src))])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_run, c) for c in cmds]
        for f in futs:
            r = f.result()
            if verbose and (r.stderr.strip()):
                print(r.stderr)
    objs = [os.path.join(BUILD, o) for _, _, o in units] + [os.path.join(BUILD, _host_obj(s)) for s in HOST_SOURCES]
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
