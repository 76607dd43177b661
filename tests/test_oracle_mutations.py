"""The pins are strong enough: each plausible mistake planted in a copy of
the oracle's C source (on the CPU, in a temporary directory) makes at least
one pin fail.  Every mutation keeps all memory accesses in bounds, so a
failure is a wrong value caught by a pin, never a crash."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = ["tests/test_oracle_pins.py", "tests/test_srad_oracle_pins.py"]

# (file, text, replacement, what the mistake is)
MUTATIONS = [
    ("edge_oracle.c", "exp(-(double)(i * i) /", "exp(-(double)(i) /", "Gaussian exponent linear"),
    ("edge_oracle.c", "(2.0 * sigma * sigma)", "(sigma * sigma)", "Gaussian width off by sqrt 2"),
    ("edge_oracle.c", "(double)I[yy * pitch + xx]", "(double)I[yy * pitch + (W - 1 - xx)]",
     "blur reads the mirrored column"),
    ("edge_oracle.c", "clampi(y + i, 0, H - 1)", "((y + i) % H + H) % H",
     "wrap-around instead of clamped rows"),
    ("edge_oracle.c", "- 4.0 * at(B, H, W, y, x)", "- 3.0 * at(B, H, W, y, x)",
     "Laplacian centre weight"),
    ("edge_oracle.c", "x + dx) > 0.0 ? 1 : 0", "x + dx) >= 0.0 ? 1 : 0",
     "zero counted as positive"),
    ("edge_oracle.c", "{1.0, 2.0, 1.0}", "{1.0, 1.0, 1.0}", "Sobel smoothing weights"),
    ("edge_oracle.c", "(at(B, H, W, y + 1, x + d) - at(B, H, W, y - 1, x + d))",
     "(at(B, H, W, y + 1, x) - at(B, H, W, y - 1, x))", "Sobel gy ignores the column offset"),
    ("edge_oracle.c", "if (G[i] > m) m = G[i];", "if (G[i] < m) m = G[i];", "max becomes min"),
    ("edge_oracle.c", "G[y * W + x] > tau", "G[y * W + x] >= tau", "threshold not strict"),
    ("srad_oracle.c", "s2 += J[i] * J[i];", "s2 += J[i];", "second moment of J"),
    ("srad_oracle.c", "const double v = s2 / n - m * m;", "const double v = s2 / n;",
     "variance drops the mean term"),
    ("srad_oracle.c", "*q0sqr = v / (m * m);", "*q0sqr = v / m;", "q0^2 divides by the mean"),
    ("srad_oracle.c", "(l * l) / 16.0", "(l * l) / 4.0", "q^2 Laplacian weight"),
    ("srad_oracle.c", "1.0 + 0.25 * l", "1.0 + l", "q^2 denominator"),
    ("srad_oracle.c", "if (cv > 1.0) cv = 1.0;", "", "c not clamped to 1"),
    ("srad_oracle.c", "at(c, H, W, y + 1, x) * dS", "cc * dS", "c_S replaced by c"),
    ("srad_oracle.c", "at(c, H, W, y, x + 1) * dE", "cc * dE", "c_E replaced by c"),
    ("srad_oracle.c", "j + 0.25 * lambda * D", "j + lambda * D", "step lambda instead of lambda/4"),
]


def _run_pins(tmp, sources):
    """Build `sources` (file -> text) into tmp and run the pins against it;
    returns pytest's exit code."""
    from oracle.build import build
    for f in os.listdir(ORACLE):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(ORACLE, f), tmp)
    for f, text in sources.items():
        with open(os.path.join(tmp, f), "w") as fh:
            fh.write(text)
    out = build(out=os.path.join(tmp, "libhx_oracle.so"), srcdir=tmp)
    env = dict(os.environ, HXO_ORACLE_LIB=out)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    return r.returncode


def _mutated(f, old, new):
    with open(os.path.join(ORACLE, f)) as fh:
        text = fh.read()
    assert text.count(old) == 1, (f, old)   # the mutation applies, once
    return {f: text.replace(old, new)}


def test_unmutated_copy_passes(tmp_path):
    """The harness itself: an unchanged copy built the same way passes."""
    assert _run_pins(str(tmp_path), {}) == 0


def test_every_mutation_fails_a_pin(tmp_path):
    jobs = []
    for i, (f, old, new, what) in enumerate(MUTATIONS):
        d = tmp_path / f"m{i}"
        d.mkdir()
        jobs.append((what, str(d), _mutated(f, old, new)))
    with ThreadPoolExecutor(max_workers=4) as ex:
        codes = list(ex.map(lambda j: _run_pins(j[1], j[2]), jobs))
    survivors = [what for (what, _, _), rc in zip(jobs, codes) if rc != 1]
    assert not survivors, f"mutations no pin catches (or that crashed): {survivors}"
