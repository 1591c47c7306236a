"""Build the HIP library libzinc.so in-tree for gfx950 (hipcc, no JIT)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libzinc.so")
SOURCES = ["capi.cpp", "host_math.cpp", "plan.cpp", "server.cpp", "tune.cpp", "kernels.hip", "kernels_split.hip",
           "kernels_plan_zinc.hip", "kernels_plan_vanilla.hip", "kernels_tiles_zinc.hip", "kernels_tiles_vanilla.hip",
           "kernels_elementwise.hip", "kernels_sp.hip", "kernels_sp_split.hip", "kernels_bfv.hip", "kernels_batch.hip", "kernels_rate.hip"]
ARCH = os.environ.get("ZINC_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [_hipcc(), *COMMON, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    warn = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if warn:
        sys.stderr.write("\n".join(warn) + "\n")
    return obj


def _stale(src: str) -> bool:
    """True if src's object is missing or older than src or any header."""
    obj = os.path.join(BUILD, src + ".o")
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(ROOT, "include", "zinc.h"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, only_stale: bool = False) -> str:
    """Compile every source (only_stale: only those whose object is out of
    date, a development shortcut) and link libzinc.so."""
    os.makedirs(BUILD, exist_ok=True)
    todo = [s for s in SOURCES if not only_stale or _stale(s)]
    with ThreadPoolExecutor(max_workers=max(1, len(todo))) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(BUILD, s + ".o") for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, only_stale="--stale" in sys.argv[1:])
