"""Build the HIP library ``libetdpic.so`` for gfx950 with hipcc.

Every ``csrc/*.hip`` file is compiled for ``--offload-arch=gfx950`` and linked
into one shared library next to this file.  Packed FP32 instructions are
disabled for the device code, and floating-point contraction is off: every
fused multiply-add is an explicit fma() in the source, so the same expression
rounds the same way in every kernel it is inlined into (the deposit of the
fused push kernel and of the sorted deposit must agree to the bit).
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libetdpic.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
CLI_SRC = os.path.join(HERE, "cli", "etdpic_run.c")
ROCM_LIB = "/opt/rocm/lib"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in ordinary VGPRs: the learned-inference kernel
         # feeds every layer's results straight into VALU activations, and
         # AGPR accumulators would cost one copy instruction per element
         "-mllvm", "-amdgpu-mfma-vgpr-form=1",
         "-Wall", "-Wno-unused-result", "-I" + INCLUDE]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile the library (always; a stale .so is never trusted).  Returns its path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + sources() + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if noise not in l]
    if res.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc failed building %s" % LIB)
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    build_cli()
    return LIB


def build_cli() -> str:
    """Compile the command-line driver ``etdpic_run`` (host C, gcc) against the library."""
    out = os.path.join(HERE, "etdpic_run")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu99", "-Wall", "-I" + INCLUDE, CLI_SRC, "-o", tmp,
           "-L" + HERE, "-letdpic", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath-link," + ROCM_LIB, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def is_built() -> bool:
    return os.path.exists(LIB)


if __name__ == "__main__":
    print(build(verbose=True))
