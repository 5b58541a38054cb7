"""Build libdgsw.so in-tree for gfx950 with hipcc.

    python -m paper_2303_11767_amd.build

Objects go to _build/ at the repository root; the library lands next to
this file, where the binding loads it.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdgsw.so")
PROBE_SRC = ["probe_contraction.hip", "probe_floor.hip"]
PROBE_LIB = os.path.join(PKG, "libdgsw_probe.so")
SOURCES = ["dgsw_tables.cpp", "dgsw_kernels.hip", "dgsw_ens_kernels.hip", "dgsw_api.hip",
           "dgsw_ensemble.hip", "dgsw_mlp.hip", "dgsw_learned.hip", "dgsw_advection.hip"]
ARCH = os.environ.get("DGSW_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# device code: gfx950 only; packed FP32 instructions disabled
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-gpu-flush-denormals-to-zero", "-ffp-contract=fast"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, jobs=None):
    """Compile every source (in parallel, one hipcc per source) and link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        if src.endswith(".hip"):
            cmds.append([HIPCC] + COMMON + DEVICE + ["-c", path, "-o", obj])
        else:
            cmds.append([HIPCC] + COMMON + ["-c", path, "-o", obj])
        objs.append(obj)
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    # the measurement probes (contraction forms, launch and memory floor): not
    # part of the solver
    ptmp = PROBE_LIB + ".tmp"
    _run([HIPCC] + COMMON + DEVICE + ["-shared", "-o", ptmp] + [os.path.join(CSRC, f) for f in PROBE_SRC], verbose)
    os.replace(ptmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
