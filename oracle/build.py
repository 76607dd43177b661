"""Build step for the oracle library (oracle/libhx_oracle.so).

Test infrastructure: the oracle is compiled with plain gcc, -O2, no fast-math
and no FP contraction, so that every double operation is the one written in
edge_oracle.c.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhx_oracle.so")


def build(verbose: bool = False, out: str = LIB, srcdir: str = HERE) -> str:
    """Compile the oracle sources in `srcdir` into `out` (by default this
    directory's sources into LIB)."""
    srcs = [os.path.join(srcdir, f) for f in ("edge_oracle.c", "srad_oracle.c")]
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           *srcs, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
