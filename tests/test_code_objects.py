"""The gfx950 code objects built into libhx.so: every kernel keeps its
per-lane values in registers.  A kernel with a private (scratch) segment
stores and reloads values through memory, and each reload waits for every
load in flight, which undoes the sweeps' row prefetch (a compiler turning a
select chain into an indexed array did exactly that once).  Reads only the
kernel metadata of this repository's own build."""
import os
import re
import struct
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2503_10855_amd", "libhx.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def gfx950_code_objects(lib):
    """The gfx950 entries of every offload bundle in lib's .hip_fatbin."""
    with tempfile.TemporaryDirectory() as td:
        fb = os.path.join(td, "fatbin.bin")
        subprocess.run([f"{LLVM}/llvm-objcopy", f"--dump-section=.hip_fatbin={fb}", lib,
                        os.path.join(td, "discard.so")], check=True, capture_output=True)
        data = open(fb, "rb").read()
    out = []
    for m in re.finditer(re.escape(MAGIC), data):
        base = m.start()
        pos = base + len(MAGIC)
        (n,) = struct.unpack_from("<Q", data, pos)
        pos += 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", data, pos)
            pos += 24
            triple = data[pos:pos + tlen].decode()
            pos += tlen
            if "gfx950" in triple and size:
                out.append(data[base + off:base + off + size])
    return out


def kernel_private_sizes(co):
    """{kernel name: private segment bytes} from a code object's notes."""
    with tempfile.NamedTemporaryFile(suffix=".co") as f:
        f.write(co)
        f.flush()
        notes = subprocess.run([f"{LLVM}/llvm-readelf", "--notes", f.name], check=True,
                               capture_output=True, text=True).stdout
    sizes, name = {}, None
    for line in notes.splitlines():
        s = line.strip()
        if s.startswith(".name:"):
            name = s.split(":", 1)[1].strip()
        elif s.startswith(".private_segment_fixed_size:") and name:
            sizes[name] = int(s.split(":", 1)[1])
            name = None
    return sizes


@pytest.mark.skipif(not os.path.exists(LIB) or not os.path.exists(f"{LLVM}/llvm-readelf"),
                    reason="libhx.so not built or LLVM tools missing")
def test_no_kernel_uses_scratch():
    cos = gfx950_code_objects(LIB)
    assert cos, "no gfx950 code object in libhx.so"
    sizes = {}
    for co in cos:
        sizes.update(kernel_private_sizes(co))
    assert any("k_batch_p1s" in k for k in sizes), sorted(sizes)[:5]
    spill = {k: v for k, v in sizes.items() if v}
    assert not spill, spill
