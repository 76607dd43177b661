"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer, on
the CPU: the oracle (plain C), the tuned CPU library (C++ over threads) and
the scheduling-language compiler (the one part of libhx.so that is pure host
logic) are rebuilt with the sanitizers into a temporary directory and run on
small inputs, including the degenerate shapes; any report fails the test.
The sanitizers instrument host code only (-Xarch_host on the hipcc line)."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
HIPCC = "/opt/rocm/bin/hipcc"


def libasan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                       text=True).stdout.strip()
    return p if p and os.path.isabs(p) and os.path.exists(p) else None


def run_child(code, env_extra, tmp):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, cwd=tmp,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "AddressSanitizer" not in out, \
        out[-4000:]
    return out


pytestmark = pytest.mark.skipif(libasan() is None or shutil.which("gcc") is None,
                                reason="gcc sanitizer runtime not available")

SHAPES = "[(1, 1), (1, 7), (7, 1), (2, 3), (5, 5), (3, 300), (67, 41), (130, 97)]"


def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("edge_oracle.c", "srad_oracle.c")]
    subprocess.run(["gcc", "-std=c11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
                    *SAN, *srcs, "-o", lib, "-lm"], check=True)
    out = run_child(f"""
        import numpy as np, oracle
        from paper_2503_10855_amd import synth
        for i, (h, w) in enumerate({SHAPES}):
            img = synth.image(h, w, 31, i)
            for ks, sg in ((3, 0.8), (5, 1.0), (7, 1.5)):
                oracle.edge_detect(img, ks, sg, 0.1, stages=True)
            oracle.srad(synth.speckle(h, w), 2, 0.5)
        imgs = [synth.image(h, w, 32, i) for i, (h, w) in enumerate({SHAPES})]
        oracle.edge_detect_many(imgs, 5, 1.0, 0.1, nthreads=4)
        print("oracle ok")
        """, {"HXO_ORACLE_LIB": lib, "LD_PRELOAD": libasan()}, str(tmp_path))
    assert "oracle ok" in out


def test_cpu_library_under_sanitizers(tmp_path):
    lib = str(tmp_path / "libhx_cpu_san.so")
    subprocess.run(["g++", "-std=c++17", "-fPIC", "-shared", "-pthread", *SAN,
                    os.path.join(ROOT, "paper_2503_10855_amd", "cpu", "edge_cpu.cpp"),
                    "-o", lib], check=True)
    out = run_child(f"""
        import ctypes
        from paper_2503_10855_amd import cpu, synth
        cpu._lib = ctypes.CDLL({lib!r})
        cpu._lib.hx_cpu_edge_detect_many.restype = ctypes.c_int
        imgs = [synth.image(h, w, 33, i) for i, (h, w) in enumerate({SHAPES})]
        for ks, sg in ((3, 0.8), (5, 1.0), (7, 1.5)):
            cpu.edge_detect_many(imgs, ks, sg, 0.1, nthreads=4)
        print("cpu ok")
        """, {"LD_PRELOAD": libasan()}, str(tmp_path))
    assert "cpu ok" in out


DRIVER = r'''
#include <cstdarg>
#include <cstdio>
#include <string>
#include "hx_pipeline.h"
namespace hx {
hx_status fail(hx_status st, const char* fmt, ...) {
    char b[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(b, sizeof b, fmt, ap);
    va_end(ap);
    return st;
}
}  // namespace hx
int main() {
    const char* progs[] = {
        "",
        "fork-tile[16, 64](blur, laplacian, zero_cross, sobel); warp-reduce(max_gradient);",
        "fork-fuse(blur, sobel, laplacian, zero_cross); fork-tile[64, 256](blur); "
        "warp-reduce(max_gradient); pass[speculate](threshold);",
        "fork-fuse(blur, sobel); fork-fuse(laplacian, zero_cross); fork-tile[32, 128](blur);",
        "reduction_tree![4096](max_gradient);",
        "fork-chunk[4096](max_gradient); fork-reshape(max_gradient); "
        "monoid-reassociate(max_gradient); fork-fission(max_gradient);",
        "fork-fission(max_gradient);", "fork-fuse(blur, laplacian);", "fork-tile[", ";;;",
        "pass[bogus](threshold);", "fork-tile[-1, 99999999999](blur);",
        "let (a, b) = blur(c);", "fork-tile[16, 16](nothing);",
    };
    int ok = 0;
    for (const char* t : progs) {
        hx_schedule s{};
        if (hx::compile_schedule(t, &s) == HX_OK) {
            const std::string back = hx::schedule_text(s);
            hx_schedule s2{};
            if (hx::compile_schedule(back.c_str(), &s2) != HX_OK) return 2;
            ++ok;
        }
    }
    std::printf("schedules ok %d\n", ok);
    return 0;
}
'''


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_schedule_compiler_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2503_10855_amd", "csrc")
    drv = tmp_path / "drv.cpp"
    drv.write_text(DRIVER)
    exe = str(tmp_path / "sched_san")
    flags = ["--offload-arch=gfx950", "-std=c++20", "-g", "-O1", "-I" + csrc,
             "-I" + os.path.join(ROOT, "include"),
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.run([HIPCC, *flags, os.path.join(csrc, "hx_sched.cpp"), str(drv), "-o", exe],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "schedules ok" in out and "runtime error" not in out, out[-3000:]
