"""Build of the HIP library ``libsd.so`` for gfx950 (hipcc, in-tree)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsd.so")

SOURCES = ["sd_kernels.hip", "sd_operators.cpp"]
HEADERS = ["sd_internal.h", "sd_physics.h", "sd_ns_kernel.h", "sd_mlp.h", "sd_bloch_kernel.h", "sd_curv_kernel.h",
           "sd_dispatch.inc", "sd_closure.inc", "sd_bloch.inc", "sd_curv.inc", "sd_run1d.inc"]

# Packed FP32 instructions stay off: the compiler must not form them.
HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources_sha256(names):
    """SHA-256 of the compiler flags and the named sources under csrc/: the key
    of a committed measurement record (a record taken on other sources is not
    reported)."""
    import hashlib
    h = hashlib.sha256()
    h.update(" ".join(HIPCC_FLAGS).encode())
    for name in names:
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# the sources that define and launch the Navier-Stokes right-hand side, its
# operators and its launch configuration
NS_RHS_SOURCES = ["sd_ns_kernel.h", "sd_internal.h", "sd_physics.h", "sd_dispatch.inc", "sd_operators.cpp"]


def build_library(verbose=False):
    """Compile every HIP source into ``libsd.so`` (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
