"""Build the FP64 CPU oracle (test infrastructure).

``build()`` writes ``oracle/liboracle.so``: gcc -O3 with generic x86-64 code
(it is built here and may run on a different host), OpenMP for the
per-neuron loops. ``build_native()`` writes ``oracle/liboracle_native.so``
with ``-O3 -march=native`` on the host that will run it; the benchmark's
CPU-baseline leg builds and times that copy.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bernnn_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")


def _gcc(out, arch_flags, verbose):
    cmd = ["gcc", "-O3", *arch_flags, "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    return _gcc(LIB, [], verbose)


def build_native(verbose: bool = False) -> str:
    return _gcc(LIB_NATIVE, ["-march=native"], verbose)


if __name__ == "__main__":
    print(build(verbose=True))
