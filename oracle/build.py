"""Build the FP64 CPU oracle shared library (test infrastructure only).

``python oracle/build.py`` compiles ``abm_oracle.c`` (mechanics, cell
behaviour, statistics), ``sir_oracle.c`` (SIR epidemiology) and
``soma_oracle.c`` (diffusion, secretion, chemotaxis) with gcc into
``oracle/liboracle.so``.  The flags keep IEEE semantics: no fast-math and no
floating-point contraction, so every product and sum rounds as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("abm_oracle.c", "sir_oracle.c", "soma_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
        *SRCS, "-o", LIB + ".tmp", "-lquadmath", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
