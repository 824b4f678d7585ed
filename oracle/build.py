"""Build the C oracle (test infrastructure): gcc -O2 -fopenmp -ffp-contract=off, no hand SIMD.

--sanitize builds a second copy with AddressSanitizer and UndefinedBehaviorSanitizer (LLVM clang, so that one
sanitizer runtime serves it and the library's sanitizer build in one process) into SANITIZE_LIB."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qs_oracle.c")
LIB = os.path.join(HERE, "libqs_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


ROOT = os.path.dirname(HERE)
SANITIZE_LIB = os.path.join(ROOT, "_build", "sanitize", "libqs_oracle.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build_sanitized() -> str:
    os.makedirs(os.path.dirname(SANITIZE_LIB), exist_ok=True)
    cmd = [CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-shared-libsan", "-ffp-contract=off", "-shared", "-fPIC", "-Wall",
           "-Wextra", "-o", SANITIZE_LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(SANITIZE_LIB + ".tmp", SANITIZE_LIB)
    return SANITIZE_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized())
    else:
        print(build(force="--if-stale" not in sys.argv))
