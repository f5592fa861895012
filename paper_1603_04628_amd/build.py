"""Build libhmd.so for gfx950 from the sources in ``csrc/``.

Every HIP translation unit is compiled with hipcc for gfx950 with packed-FP32
instruction selection disabled; the host-only system builder is compiled
without floating-point contraction so its arithmetic rounds as written.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libhmd.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("HMD_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HIP_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", f"-I{INCLUDE}", f"-I{CSRC}"]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall", "-ffp-contract=off", "-fno-fast-math",
              f"-I{INCLUDE}", f"-I{CSRC}"]

# (source, compiler): host-only files use the system C++ compiler
SOURCES = [
    ("md_setup.cpp", "host"),
    ("md_kernels.hip", "hip"),
    ("md_engine.hip", "hip"),
    ("series.hip", "hip"),
    ("abi.cpp", "hip"),
    ("tune.cpp", "hip"),
    ("gp.hip", "hip"),
    ("ens.hip", "hip"),
    ("hybrid.cpp", "host"),
    ("startup.cpp", "host"),
    ("peaks.hip", "hip"),
]


def _compile(src_kind):
    src, kind = src_kind
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if kind == "hip":
        cmd = [HIPCC] + HIP_FLAGS + ["-c", path, "-o", obj]
    else:
        cmd = ["g++"] + HOST_FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = int(os.environ.get("MAX_JOBS", "8"))
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
