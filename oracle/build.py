"""Compile the CPU oracle (test infrastructure only) with gcc.

Two shared libraries come out of the one source file:
  liborc_f64.so  -- REAL = double (reference arithmetic)
  liborc_f32.so  -- REAL = float  (the paper's 32-bit precision, for decisions)

Both are compiled with -ffp-contract=off so that every arithmetic operator is
one IEEE operation and fused multiply-adds appear only where written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "polar_oracle.c")
LIBS = {"f64": os.path.join(HERE, "liborc_f64.so"), "f32": os.path.join(HERE, "liborc_f32.so")}


def build(verbose: bool = False) -> None:
    for tag, out in LIBS.items():
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized"]
        if tag == "f32":
            cmd.append("-DORACLE_F32")
        cmd += [SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)


def ensure_built() -> None:
    src_mtime = os.path.getmtime(SRC)
    if any(not os.path.exists(p) or os.path.getmtime(p) < src_mtime for p in LIBS.values()):
        build()


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
