"""Build the HIP library ``libfzp.so`` for gfx950 in-tree.

    python -m paper_2609_01978_amd.build        # or paper_2609_01978_amd.build.build()
    python -m paper_2609_01978_amd.build --host-sanitize OUT.so   # host ASan + UBSan variant
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfzp.so")

SOURCES = ["fzp_plan.cpp", "fzp_fft.hip", "fzp_gemm.hip", "fzp_i8.hip", "fzp_cplx.hip", "fzp_metrics.hip", "fzp_mlp.hip",
           "fzp_static.hip", "fzp_sa.hip", "fzp_prior.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed-FP32 instructions in generated device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build (device code is
# built as usual): every -fsanitize applies to the host pass only.
HOST_SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                       "-g"]


def build(verbose: bool = False, out: str = LIB, host_sanitize: bool = False) -> str:
    """Compile every source into `out` (default paper_2609_01978_amd/libfzp.so;
    always rebuilds).  host_sanitize builds the host code with ASan and UBSan
    (load it with the sanitizer runtime preloaded and FZP_LIBRARY=<out>)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *(HOST_SANITIZE_FLAGS if host_sanitize else []), "-I", INCLUDE, "-I", CSRC,
           *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libfzp.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--host-sanitize":
        print(build(verbose=True, out=os.path.abspath(sys.argv[2]), host_sanitize=True))
    else:
        print(build(verbose=True))
