"""Build the C-ABI library libocean_bse.so for gfx950 with hipcc (in-tree).

build(asan=True) builds a second copy, _build_asan/libocean_bse_asan.so, whose host code
is compiled with AddressSanitizer (device code unchanged); it is for host-side checks on the
CPU only, loaded with the sanitizer runtime preloaded."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libocean_bse.so")
OBJ_ASAN = os.path.join(HERE, "_build_asan")
LIB_ASAN = os.path.join(OBJ_ASAN, "libocean_bse_asan.so")
# host code only: each sanitizer flag applies to the host compilation
ASAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
SOURCES = ["proj.hip", "proj_bf16.hip", "fftw.hip", "vec.hip", "runtime.hip", "mlp.hip", "ceilings.hip",
           "screening.hip", "multiplet.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core accumulators in ordinary VGPRs: with at most 256 threads per block the
         # compiler otherwise places them in AGPRs and copies them to VGPRs and back around
         # every group of MFMAs inside the loops
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wall", "-Wno-unused-function"]


def _compile(src: str, asan: bool = False) -> str:
    obj = os.path.join(OBJ_ASAN if asan else OBJ, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *FLAGS, *(ASAN_FLAGS if asan else []), *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, asan: bool = False) -> str:
    out = LIB_ASAN if asan else LIB
    os.makedirs(OBJ_ASAN if asan else OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda src: _compile(src, asan), SOURCES))
    tmp = out + ".tmp"
    san = ["-Xarch_host", "-fsanitize=address", "-shared-libsan"] if asan else []
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *san, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
