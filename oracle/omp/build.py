"""Builds oracle/omp/liboracle_omp.so (the host-parallel oracle) with g++ and
OpenMP: `python oracle/omp/build.py`."""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cheb_omp.cpp")
LIB = os.path.join(HERE, "liboracle_omp.so")


def build() -> str:
    cxx = shutil.which("g++") or "g++"
    tmp = LIB + ".tmp"
    subprocess.run([cxx, "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
