"""hx_edge_detect_static, the entry point that allocates nothing (its
scratch is a fixed device array): through the C ABI it gives the bits of
hx_edge_detect in the same fused STORE form, on two calls in a row (the
second on a smaller image, so the array keeps the first call's larger
contents), allocates nothing, and refuses an image beyond its capacity."""
import numpy as np
import pytest
import torch

import oracle
import parity
from paper_2503_10855_amd import synth

pytestmark = pytest.mark.gpu
THETA = 0.1


@pytest.fixture(scope="module")
def hx():
    from paper_2503_10855_amd import hx as mod
    return mod


@pytest.mark.parametrize("ks,sigma", [(5, 1.0), (7, 1.5), (3, 1.0)])
def test_static_entry_matches_per_image(hx, ks, sigma):
    big = synth.image(1500, 2100, 95, 0)
    small = synth.image(333, 517, 95, 1)
    tb, ts = torch.from_numpy(big).cuda(), torch.from_numpy(small).cuda()
    with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA, max_pixels=big.size) as p:
        before = p.memory()
        print(f"static entry, k{ks}: 1500x2100 then 333x517", flush=True)
        outs = []
        for t in (tb, ts):
            dm = torch.zeros(1, device="cuda")
            m = torch.full(t.shape, 7, dtype=torch.uint8, device="cuda")
            p.edge_detect_static(t, m, dmax=dm)
            outs.append((m, dm))
        torch.cuda.synchronize()
        assert p.memory() == before
        p.set_schedule(256, 32, 4, hx.PASS_STORE)
        refs = []
        for t in (tb, ts):
            dm = torch.zeros(1, device="cuda")
            refs.append((p.edge_detect(t, dmax=dm), dm))
        torch.cuda.synchronize()
    for (m, dm), (rm, rdm) in zip(outs, refs):
        assert torch.equal(m.cpu(), rm.cpu())
        assert torch.equal(dm.cpu(), rdm.cpu())
    o = oracle.edge_detect(small, ks, sigma, THETA, stages=True)
    assert parity.compare_mask(outs[1][0].cpu().numpy(), o, THETA)["mismatch"] == 0


def test_static_entry_refuses_oversized_image(hx):
    side = 4096  # 4096 x 4096 = 16 Mi code elements > the 8 Mi the array holds
    src = torch.zeros((side, side), dtype=torch.float32, device="cuda")
    with hx.Pipeline(theta=THETA, max_pixels=side * side, forms=hx.FORM_BATCH,
                     batch_contexts=1) as p:
        with pytest.raises(hx.HxError) as ei:
            p.edge_detect_static(src)
        assert ei.value.status == hx.HX_E_INVALID
