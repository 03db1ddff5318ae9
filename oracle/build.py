"""Compile the FP64 oracle (test infrastructure) into oracle/libtgo.so.

The float32 binning spec inside it must see every IEEE operation exactly as
written, so the build forbids floating-point contraction and fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tgo.cpp")
LIB = os.path.join(HERE, "libtgo.so")
FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
         "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only"]


# host-only sanitizer build (g++, no device code): AddressSanitizer and
# UndefinedBehaviorSanitizer, every finding fatal
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, out: str = LIB, plant: int = 0, sanitize: bool = False) -> str:
    """Compile the oracle to `out`.  `plant` > 0 builds a deliberately wrong
    variant (see the mutation hook in tgo.cpp), used only by the tests;
    `sanitize` builds it with the sanitizers (load it with the ASan runtime
    preloaded)."""
    cmd = ["g++", *FLAGS, *(SANITIZE if sanitize else []), f"-DTGO_PLANT={int(plant)}", SRC, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
