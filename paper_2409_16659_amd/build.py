"""Build ``libmlfilm.so`` (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_2409_16659_amd.build [-v]``.  The library is always
rebuilt; callers that only need it loaded use :func:`lib_path`.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmlfilm.so")
SOURCES = [os.path.join(CSRC, "mlfilm.hip"), os.path.join(CSRC, "surrogate.hip"), os.path.join(CSRC, "stokes.hip")]
HEADERS = [os.path.join(CSRC, "step_kernel.hpp"), os.path.join(CSRC, "nop_kernels.hpp"),
           os.path.join(CSRC, "stream_probe.hpp"), os.path.join(CSRC, "d1q3_kernel.hpp"),
           os.path.join(CSRC, "d2q9_row_kernel.hpp"),
           os.path.join(ROOT, "include", "mlfilm.h"), os.path.join(ROOT, "include", "mlf_surrogate.h")]
ARCH = os.environ.get("MLF_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code; -O3 would
# otherwise form them from scalar float code.  Multiply-adds are fused only
# within one source expression (-ffp-contract=on), so that the same kernel
# body rounds identically in every kernel it is inlined into (single film,
# batch).
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


LIB_SAN = os.path.join(HERE, "libmlfilm_hostsan.so")
# AddressSanitizer + UBSan on the host code only (the device code is built
# as usual); load it with MLFILM_LIB pointing at it and clang's ASan runtime
# (libclang_rt.asan-x86_64.so) preloaded.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, extra=None, sanitize_host: bool = False) -> str:
    out = LIB_SAN if sanitize_host else LIB
    cmd = [hipcc(), *HIPCC_FLAGS, *(HOST_SANITIZE if sanitize_host else []), *(extra or []), "-o", out + ".tmp",
           *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def lib_path() -> str:
    """The library the binding loads: MLFILM_LIB (another build of the same
    sources, e.g. the host-sanitizer one) or the in-tree build."""
    return os.environ.get("MLFILM_LIB") or LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize_host="--sanitize-host" in sys.argv))
