"""Build libras_pml.so (HIP for gfx950) in-tree.

    python -m paper_2602_00735_amd.build [-v]

Every HIP source is compiled with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); the host planner is
plain C++.  Objects go to paper_2602_00735_amd/_build/, the shared object
next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libras_pml.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["k_assemble.hip", "k_lu.hip", "k_lu_mfma.hip", "k_solve.hip", "k_krylov.hip",
               "k_warm.hip", "warm_net.hip", "abi.hip"]
CPP_SOURCES = ["plan.cpp", "devpool.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HIP_FLAGS = ["-x", "hip", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
# Per-source additions.  The factorisation keeps its accumulator tiles in
# ordinary vector registers (its vector code reads and writes them between
# the matrix-core updates): without this the compiler moves every tile into
# accumulation registers and back around each update.
HIP_EXTRA = {"k_lu_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


def _runtime_dir() -> str:
    """Directory of the HIP runtime the process will use.

    PyTorch ships its own libamdhip64; two HIP runtimes in one process do
    not share devices, so the library links against torch's copy when torch
    is installed, else against /opt/rocm/lib."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return "/opt/rocm/lib"


def build(verbose: bool = False, jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs_list = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        jobs_list.append([HIPCC, "-c", *COMMON, *HIP_FLAGS, *HIP_EXTRA.get(s, []),
                          os.path.join(CSRC, s), "-o", o])
    for s in CPP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        jobs_list.append([HIPCC, "-c", *COMMON, os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in jobs_list]:
            f.result()
    objs = [c[-1] for c in jobs_list]
    tmp = LIB + ".tmp%d" % os.getpid()
    rt = _runtime_dir()
    _run(["g++", "-shared", "-fPIC", *objs, "-o", tmp, "-L" + rt, "-l:libamdhip64.so",
          "-Wl,-rpath," + rt, "-Wl,--no-undefined"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
