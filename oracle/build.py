"""Build the CPU oracle shared libraries (FP64, and FP32 for the round-off floor).

Test infrastructure: compiled with gcc, plain -O2 + OpenMP, no fast-math and
no FMA contraction, so the oracle's arithmetic is exactly what its C source
says.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wave_oracle.c")
OUT = os.path.join(HERE, "_build")
LIBS = {"f64": "liboracle_f64.so", "f32": "liboracle_f32.so"}


def lib_path(precision: str = "f64") -> str:
    return os.path.join(OUT, LIBS[precision])


def build(verbose: bool = False) -> None:
    os.makedirs(OUT, exist_ok=True)
    for prec, name in LIBS.items():
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-ffp-contract=off", "-Wall", "-Wno-unused-function"]
        if prec == "f32":
            cmd.append("-DORACLE_REAL_FLOAT")
        cmd += [SRC, "-o", os.path.join(OUT, name), "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose=True)
