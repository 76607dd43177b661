"""Seeded random cases: shapes, row pitches, blur sizes, value ranges and
pass structures drawn from one generator, each image checked against the
fp64 oracle per image and in one ragged batch, and the maxima against the
oracle's M.  Complements the hand-picked shapes of test_gpu_parity."""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import oracle
import parity

pytestmark = pytest.mark.gpu
THETA = 0.1


@pytest.fixture(scope="module")
def hx():
    from paper_2503_10855_amd import hx as mod
    return mod


def cases(seed, n):
    """n images: sides log-uniform in [1, 900], values either the usual
    scene or wide-range noise (negative values included), each in a buffer
    whose row pitch has 0-7 extra floats."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 99]))
    out = []
    for i in range(n):
        h = int(round(np.exp(rng.uniform(0, np.log(900)))))
        w = int(round(np.exp(rng.uniform(0, np.log(900)))))
        if rng.random() < 0.5:
            from paper_2503_10855_amd import synth
            a = synth.image(h, w, seed, i)
        else:
            a = (rng.standard_normal((h, w)) * 10.0 ** rng.uniform(-2, 2)).astype(np.float32)
        out.append((a, int(rng.integers(0, 8))))
    return out


def pitched(a, pad):
    h, w = a.shape
    buf = torch.zeros((h, w + pad), dtype=torch.float32, device="cuda")
    view = buf[:, :w]
    view.copy_(torch.from_numpy(a))
    return view


@pytest.mark.parametrize("ks,sigma,seed", [(5, 1.0, 501), (3, 0.8, 502), (7, 1.5, 503)])
def test_random_images_per_image_and_batched(hx, ks, sigma, seed):
    imgs = cases(seed, 24)
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 4)) as ex:
        oras = list(ex.map(lambda c: oracle.edge_detect(c[0], ks, sigma, THETA, stages=True),
                           imgs))
    srcs = [pitched(a, pad) for a, pad in imgs]
    npx = sum(a.size for a, _ in imgs)
    for pm in (1, 2, 3):
        with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA, max_pixels=npx,
                         max_images=len(imgs), pass_mode=pm) as p:
            print(f"random k{ks} seed {seed} pass {pm}: {len(imgs)} images", flush=True)
            dmax = torch.zeros(len(imgs), device="cuda")
            masks = p.edge_detect_batched(srcs, dmax=dmax)
            one = [p.edge_detect(s) for s in srcs]
            torch.cuda.synchronize()
            dm = dmax.cpu().numpy()
            for i, ((a, pad), o) in enumerate(zip(imgs, oras)):
                mb = masks[i].cpu().numpy()
                m1 = one[i].cpu().numpy()
                assert np.array_equal(mb, m1), (i, a.shape, pad)
                r = parity.compare_mask(mb, o, THETA)
                assert r["mismatch"] == 0, (i, a.shape, pad, r)
                assert parity.exempt_bounded(r), (i, a.shape, pad, r)
                M = float(dm[i])
                assert abs(M - o["M"]) <= parity.REL * o["M"] if o["M"] > 0 else M == 0.0, \
                    (i, a.shape, M, o["M"])
