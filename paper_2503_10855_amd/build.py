"""Build step for libhx.so: compiles the HIP kernels and the C ABI for
gfx950 with hipcc and links them in-tree (paper_2503_10855_amd/libhx.so).

Flags: -ffp-contract=off (the only fused multiply-adds are the explicit
fmaf calls, so every kernel variant rounds identically), packed fp32
disabled, and private arrays kept out of LDS (they become registers once
the sweep loops are unrolled).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhx.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++20", "-fPIC", "-Wall",
         "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-disable-promote-alloca-to-lds",
         "-I" + CSRC, "-I" + os.path.join(ROOT, "include")]

PLAIN = ["k_stages.hip", "k_sweep.hip", "k_batch.hip", "hx_api.cpp",
         "hx_tune.hip", "hx_serve.cpp", "hx_sched.cpp", "k_srad.hip", "hx_log.cpp"]
SWEEP_KS = (3, 5, 7)
SWEEP_MODES = (0, 1, 2, 3, 4)


def _units():
    for f in PLAIN:
        yield f, os.path.join(OUT, f.rsplit(".", 1)[0] + ".o"), []
    for k in SWEEP_KS:
        for m in SWEEP_MODES:
            yield ("sweep_inst.hip", os.path.join(OUT, f"sweep_k{k}_m{m}.o"),
                   [f"-DHX_KS={k}", f"-DHX_MODE={m}"])


def _deps_mtime():
    t = 0.0
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in os.listdir(d):
            if f.endswith((".h", ".hip", ".cpp")):
                t = max(t, os.path.getmtime(os.path.join(d, f)))
    return t


def _compile(unit, incremental, dep_t, verbose):
    src, obj, extra = unit
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) >= dep_t:
        return obj
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} {extra} failed:\n{r.stderr}")
    return obj


def build(verbose: bool = False, incremental: bool = False, jobs: int = 0) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    dep_t = _deps_mtime()
    units = list(_units())
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, incremental, dep_t, verbose), units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-ldl", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
