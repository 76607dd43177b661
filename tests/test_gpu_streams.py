"""Batched calls in flight on several streams at once (the way the
benchmark and the server issue them): each call has its own output buffers
and must give exactly the masks and maxima of the per-image calls, whatever
else runs beside it, under every pass structure."""
import numpy as np
import pytest
import torch

from paper_2503_10855_amd import synth

pytestmark = pytest.mark.gpu

THETA = 0.1
SIZES = [(1080, 1920), (300, 700), (64, 64), (517, 259), (1, 300), (777, 1025)]


@pytest.fixture(scope="module")
def hx():
    from paper_2503_10855_amd import hx as mod
    return mod


def images(seed):
    return [torch.from_numpy(synth.image(h, w, seed, i)).cuda()
            for i, (h, w) in enumerate(SIZES)]


@pytest.mark.parametrize("pass_mode", [1, 2, 3])
@pytest.mark.parametrize("nstreams", [2, 3])
def test_overlapping_batches_match_per_image(hx, pass_mode, nstreams):
    # Two different image sets, so concurrent calls also differ in content.
    sets = [images(40), images(41)]
    npx = sum(h * w for h, w in SIZES)
    with hx.Pipeline(ksize=5, sigma=1.0, theta=THETA, max_pixels=npx,
                     max_images=len(SIZES), pass_mode=pass_mode) as p:
        ref = []
        for srcs in sets:
            dm = torch.zeros(len(srcs), device="cuda")
            ms = []
            for j, s in enumerate(srcs):
                ms.append(p.edge_detect(s, dmax=dm[j:j + 1]))
            torch.cuda.synchronize()
            ref.append(([m.cpu() for m in ms], dm.cpu()))
        streams = [torch.cuda.Stream() for _ in range(nstreams)]
        preps = []
        for k in range(nstreams):
            srcs = sets[k % 2]
            masks = [torch.full(s.shape, 7, dtype=torch.uint8, device="cuda") for s in srcs]
            preps.append(p.prepare_batch(srcs, masks, torch.zeros(len(srcs), device="cuda")))
        print(f"pass {pass_mode}, {nstreams} streams", flush=True)
        for i in range(4 * nstreams):      # more calls than the pipeline has contexts
            preps[i % nstreams].run(streams[i % nstreams])
        torch.cuda.synchronize()
        for k, q in enumerate(preps):
            rm, rd = ref[k % 2]
            for j, (a, b) in enumerate(zip(q.masks, rm)):
                assert torch.equal(a.cpu(), b), (k, j, SIZES[j])
            assert torch.equal(q.dmax.cpu(), rd), k
