"""Build the CPU oracle shared library (plain C, gcc).

TEST INFRASTRUCTURE ONLY: the oracle is the checker for the GPU library and is
never part of its product path.

The single source is compiled twice, once with REAL = double and once with
REAL = long double, into one shared library ``liboracle_sigk.so`` placed next
to this file.  ``-ffp-contract=off`` keeps the rounding sequence fixed.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sigk_oracle.c")
LIB = os.path.join(HERE, "liboracle_sigk.so")

CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra",
          "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for real, sfx in (("double", "_f64"), ("long double", "_ld")):
            obj = os.path.join(tmp, f"oracle{sfx}.o")
            cmd = ["gcc", *CFLAGS, f"-DREAL={real}", f"-DSFX={sfx}", "-c", SRC, "-o", obj]
            if verbose:
                print(" ".join(cmd))
            subprocess.run(cmd, check=True)
            objs.append(obj)
        tmp_lib = LIB + ".tmp"
        cmd = ["gcc", "-shared", "-o", tmp_lib, *objs, "-lpthread", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
