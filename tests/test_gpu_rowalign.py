"""Row alignment and right edges of the vector sweep.

Rows that start on a word boundary but not on a 16-byte one, mask rows that
are not word aligned, and right edges that fall inside a lane (widths not a
multiple of 4) all run the vector sweep; a right edge whose straddling lane
has no lane after it in the strip falls back to the per-element variant.
Widths here put the edge at each position within a lane, in the second,
third and fifth 248-column strip, and on both sides of that fallback
(W = 494 keeps the vector path, 497 and 499 do not), and images narrower
than one strip, whose two edges lie in the same strip.  Each mask is compared
with the fp64 oracle, with the same image in dense buffers, and bytes
outside the mask view must stay untouched; per image and batched, under
every pass structure."""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import oracle
import parity
from paper_2503_10855_amd import synth

pytestmark = pytest.mark.gpu
THETA = 0.1
SHAPES = [(83, 757), (61, 998), (45, 1003), (70, 500), (40, 494), (40, 497),
          (40, 499), (37, 1241), (29, 253),
          # narrower than one strip: both edges in it (the vector path
          # from W = 8 up to the width the strip's right edge allows)
          (50, 61), (33, 130), (41, 247), (35, 248), (30, 245), (30, 249),
          (20, 9), (20, 8), (20, 7)]
SENTINEL = 7


@pytest.fixture(scope="module")
def hx():
    from paper_2503_10855_amd import hx as mod
    return mod


def offset_src(a, lead, pad):
    """a in a float buffer whose rows start `lead` floats in and are `pad`
    floats longer than the image (lead 1 and an odd pitch: word-aligned,
    not 16-byte aligned rows)."""
    h, w = a.shape
    buf = torch.zeros((h, w + lead + pad), dtype=torch.float32, device="cuda")
    view = buf[:, lead:lead + w]
    view.copy_(torch.from_numpy(a))
    return view


def offset_mask(h, w, lead, pad):
    buf = torch.full((h, w + lead + pad), SENTINEL, dtype=torch.uint8, device="cuda")
    return buf, buf[:, lead:lead + w]


def check_outside(buf, lead, w, what):
    b = buf.cpu().numpy()
    assert np.all(b[:, :lead] == SENTINEL), what
    assert np.all(b[:, lead + w:] == SENTINEL), what


@pytest.mark.parametrize("ks,sigma", [(3, 0.8), (5, 1.0), (7, 1.5)])
def test_unaligned_rows_and_ragged_right_edges(hx, ks, sigma):
    imgs = [synth.image(h, w, 61, i) for i, (h, w) in enumerate(SHAPES)]
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 4)) as ex:
        oras = list(ex.map(lambda a: oracle.edge_detect(a, ks, sigma, THETA, stages=True),
                           imgs))
    dense = [torch.from_numpy(a).cuda() for a in imgs]
    # Source rows 1 float in with pitch W+6 (odd W: odd pitch), mask rows 1
    # byte in with pitch W+4: every mask row has its own alignment.
    srcs = [offset_src(a, 1, 5) for a in imgs]
    mbufs = [offset_mask(a.shape[0], a.shape[1], 1, 3) for a in imgs]
    npx = sum(a.size for a in imgs)
    for pm in (1, 2, 3):
        with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA, max_pixels=npx,
                         max_images=len(imgs), pass_mode=pm) as p:
            print(f"row alignment ks={ks} pass={pm}: batched", flush=True)
            p.edge_detect_batched(srcs, [m for _, m in mbufs])
            ref = p.edge_detect_batched(dense)
            print(f"row alignment ks={ks} pass={pm}: per image", flush=True)
            one = []
            for s in srcs:
                buf, m = offset_mask(s.shape[0], s.shape[1], 1, 3)
                p.edge_detect(s, m)
                one.append((buf, m))
            p.sync()
            torch.cuda.synchronize()
        for i, (a, o) in enumerate(zip(imgs, oras)):
            what = (ks, pm, SHAPES[i])
            buf, m = mbufs[i]
            check_outside(buf, 1, a.shape[1], what)
            got = m.cpu().numpy()
            assert np.array_equal(got, ref[i].cpu().numpy()), what
            r = parity.compare_mask(got, o, THETA)
            assert r["mismatch"] == 0, (what, r)
            assert parity.exempt_bounded(r), (what, r)
            b1, m1 = one[i]
            check_outside(b1, 1, a.shape[1], ("per image",) + what)
            assert np.array_equal(m1.cpu().numpy(), got), ("per image",) + what
