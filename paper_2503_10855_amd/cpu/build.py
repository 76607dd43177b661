"""Build step for the tuned CPU comparison library (cpu/libhx_cpu.so):
g++ -O3 for x86-64-v3 (AVX2 + FMA), so the row loops vectorise."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhx_cpu.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", os.path.join(HERE, "edge_cpu.cpp"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
