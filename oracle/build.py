"""Builds the CPU reference libraries (plain C, gcc) next to this file.

liboracle_f64.so computes in double, liboracle_f80.so in x87 long double.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    src = os.path.join(HERE, "slbm_oracle.c")
    outs = []
    for name, extra in (("liboracle_f64.so", []), ("liboracle_f80.so", ["-DORACLE_EXTENDED"])):
        out = os.path.join(HERE, name)
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               "-Wno-unused-parameter", *extra, "-o", out + ".tmp", src, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
        outs.append(out)
    return outs


if __name__ == "__main__":
    for p in build(verbose=True):
        print(p)
    sys.exit(0)
