"""Build the FP64 CPU oracle (test infrastructure, not the product path).

Compiles ``qvm_oracle.c`` with gcc into ``liboracle.so`` next to this file.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qvm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


SAN_LIB = os.path.join(os.path.dirname(HERE), "_build", "sanitize", "liboracle.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """sanitize: a copy instrumented with AddressSanitizer and
    UndefinedBehaviorSanitizer, built with the same clang as the library's
    host code (one sanitizer runtime per process), at SAN_LIB."""
    out = SAN_LIB if sanitize else LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    if sanitize:
        cmd = [CLANG, "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-o", out + ".tmp", SRC, "-lm"]
    else:
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-D_DEFAULT_SOURCE", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
