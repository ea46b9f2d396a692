"""Build libntt.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2008_01340_amd.build_lib   (or build() from __graft_entry__)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/ntt_kernels.hip", "csrc/ntt_bcd.hip", "csrc/ntt_api.hip"]
LIB = os.path.join(HERE, "libntt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-Wno-unused-command-line-argument",
    # rocSOLVER (symmetric eigenvalues for the rank rule) and the rocBLAS handle it runs on
    "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas",
]


def build(verbose: bool = True) -> str:
    """Compile every HIP source into paper_2008_01340_amd/libntt.so; returns its path."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libntt.so")
    if verbose and res.stderr.strip():
        # hipcc's host pass does not know the packed-fp32 feature; keep other warnings
        lines = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l]
        if any(l.strip() for l in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
