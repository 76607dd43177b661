"""The library's diagnostics on the CPU: HX_LOG=1 prints every failing call
with its hx_last_error() text to stderr, nothing is printed without it, and
HX_TRACE=1 (roctx ranges) leaves the calls' results unchanged.  Each case
runs in a fresh process, since the settings are read once per process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2503_10855_amd", "libhx.so")

PROBE = r"""
import ctypes, sys
lib = ctypes.CDLL(sys.argv[1])
lib.hx_last_error.restype = ctypes.c_char_p
out = (ctypes.c_int32 * 5)()
st1 = lib.hx_schedule_compile(b"no-such-statement(blur);", out)
st2 = lib.hx_srad(None, None, 8, 8, 8, 1, ctypes.c_float(0.5), 1, None, None)
print(st1, st2, lib.hx_last_error().decode(), flush=True)
"""


def run_probe(env_extra):
    env = {k: v for k, v in os.environ.items() if k not in ("HX_LOG", "HX_TRACE")}
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", PROBE, LIB], env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout.strip(), [l for l in r.stderr.splitlines() if l.startswith("[hx]")]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhx.so not built")
def test_log_levels_and_trace():
    quiet_out, quiet = run_probe({})
    assert quiet == []
    out, lines = run_probe({"HX_LOG": "1"})
    assert out == quiet_out
    st1, st2 = (int(x) for x in out.split()[:2])
    assert st1 != 0 and st2 != 0
    assert len(lines) == 2, lines
    assert lines[0].startswith("[hx] error HX_E_")
    assert lines[1] == "[hx] error HX_E_INVALID: pipeline is NULL"
    t_out, t_lines = run_probe({"HX_LOG": "1", "HX_TRACE": "1"})
    assert t_out == quiet_out
    # Tracing adds no line unless the roctx library cannot be opened.
    assert t_lines == lines or (len(t_lines) == 3 and "roctx" in t_lines[0]), t_lines
