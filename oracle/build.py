"""Build the oracle's C library with the host compiler (test infrastructure)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblam_oracle.so")


def build() -> str:
    src = os.path.join(HERE, "lam_oracle.c")
    tmp = LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                    src, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_native(path: str) -> str:
    """The same source built with -O3 -march=native, for the CPU-baseline timing on the machine
    it runs on (built there, at the time of the measurement; never shipped elsewhere)."""
    src = os.path.join(HERE, "lam_oracle.c")
    tmp = path + ".tmp"
    subprocess.run(["gcc", "-O3", "-march=native", "-std=c11", "-Wall", "-fopenmp", "-fPIC",
                    "-shared", "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, path)
    return path


if __name__ == "__main__":
    print(build())
