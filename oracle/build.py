"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/liboracle.so``.

Plain C11, no fast-math and no floating-point contraction, so every product
and sum is rounded as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mlf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


LIB_SAN = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """sanitize: AddressSanitizer + UndefinedBehaviorSanitizer build into
    liboracle_san.so (load it with ORACLE_LIB pointing at it and the ASan
    runtime preloaded; every sanitizer report aborts)."""
    out = LIB_SAN if sanitize else LIB
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", *san,
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        "-o", out + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
