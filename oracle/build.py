"""Build the C part of the oracle (test infrastructure only).

Compiles ``pic_oracle.c`` and ``fine_oracle.c`` with gcc into
``oracle/_build/liboracle.so``: FP64, ``-ffp-contract=off`` so every operation
rounds as written, OpenMP over particles in the push loop only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "pic_oracle.c"), os.path.join(HERE, "fine_oracle.c")]
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle library; returns its path."""
    if (not force and os.path.exists(LIB)
            and all(os.path.getmtime(LIB) >= os.path.getmtime(s) for s in SRCS)):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           *SRCS, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
