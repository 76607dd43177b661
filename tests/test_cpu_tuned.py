"""The tuned multi-core fp32 CPU implementation (the host comparison point)
against the oracle: masks match outside the exemption bands, M within
1e-5, and the result does not depend on the thread count."""
import numpy as np
import pytest

import oracle
import parity
from paper_2503_10855_amd import synth

THETA = 0.1


@pytest.fixture(scope="module")
def cpu():
    from paper_2503_10855_amd.cpu import build as b
    import os
    if not os.path.exists(b.LIB):
        b.build()
    from paper_2503_10855_amd import cpu as mod
    return mod


SHAPES = [(1, 1), (1, 9), (9, 1), (2, 3), (5, 5), (130, 257), (300, 61), (129, 128), (260, 300)]


@pytest.mark.parametrize("ks,sigma", [(3, 0.8), (5, 1.0), (7, 1.5)])
def test_cpu_tuned_matches_oracle(cpu, ks, sigma):
    imgs = [synth.image(h, w, 29, i) for i, (h, w) in enumerate(SHAPES)]
    masks, Ms = cpu.edge_detect_many(imgs, ks, sigma, THETA, nthreads=4)
    for a, m, M in zip(imgs, masks, Ms):
        o = oracle.edge_detect(a, ks, sigma, THETA, stages=True)
        assert abs(M - o["M"]) <= 1e-5 * max(o["M"], 1e-30), (a.shape, M, o["M"])
        r = parity.compare_mask(m, o, THETA)
        assert r["mismatch"] == 0, (a.shape, r)


def test_cpu_tuned_thread_count_invariant(cpu):
    imgs = [synth.image(h, w, 30, i) for i, (h, w) in enumerate([(700, 300), (50, 900)])]
    m1, M1 = cpu.edge_detect_many(imgs, 5, 1.0, THETA, nthreads=1)
    m8, M8 = cpu.edge_detect_many(imgs, 5, 1.0, THETA, nthreads=8)
    assert all(np.array_equal(a, b) for a, b in zip(m1, m8))
    assert np.array_equal(M1, M8)


def test_cpu_tuned_degenerate(cpu):
    imgs = [np.zeros((7, 9), np.float32), np.full((40, 33), 0.3, np.float32)]
    masks, Ms = cpu.edge_detect_many(imgs, 5, 1.0, THETA, nthreads=2)
    assert all(int(m.sum()) == 0 for m in masks) and np.all(Ms == 0)
