"""The pipeline's scratch: all of it is allocated when the pipeline is
created (no call allocates), per-image calls on different streams are
ordered so they never share scratch mid-flight, and a batch larger than a
batch context's descriptor table still gives the oracle's masks."""
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


def test_no_call_allocates(hx):
    """Every call form, every pass structure and fusion depth, the stage hook
    and SRAD: the pipeline's allocation count and device bytes are those of
    hx_pipeline_create afterwards."""
    sizes = [(300, 700), (1080, 1920), (17, 5)]
    srcs = [torch.from_numpy(synth.image(h, w, 91, i)).cuda() for i, (h, w) in enumerate(sizes)]
    npx = sum(h * w for h, w in sizes)
    with hx.Pipeline(theta=THETA, max_pixels=npx, max_images=8) as p:
        before = p.memory()
        print(f"pipeline memory {before}", flush=True)
        assert before[0] > 0 and before[2] > 0
        for sched in [(64, 16, 1), (256, 32, 2), (256, 32, 3), (256, 64, 4, hx.PASS_STORE),
                      (256, 16, 4, hx.PASS_RECOMPUTE), (256, 64, 4, hx.PASS_SPECULATE)]:
            p.set_schedule(*sched)
            for s in srcs:
                p.edge_detect(s)
            p.edge_detect_batched(srcs)
        p.set_schedule()
        p.edge_detect_stages(srcs[0])
        J = torch.from_numpy(synth.speckle(256, 320)).cuda()
        p.srad(J, 3, 0.5, fused=True)
        p.srad(J, 2, 0.5, fused=False)
        p.sync()
        assert p.memory() == before


def test_per_image_calls_on_two_streams(hx):
    """Two different images in flight on two streams at once through the
    per-image form: each equals its lone result and the oracle."""
    a = synth.image(1080, 1920, 92, 0)
    b = synth.image(900, 1300, 92, 1)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    with hx.Pipeline(theta=THETA, max_pixels=1080 * 1920) as p:
        for sched in [(256, 32, 4, hx.PASS_STORE), (64, 16, 1)]:
            p.set_schedule(*sched)
            lone_a = p.edge_detect(ta).cpu().numpy()
            lone_b = p.edge_detect(tb).cpu().numpy()
            s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
            print(f"two streams, schedule {sched}", flush=True)
            outs = []
            for _ in range(4):
                ma = torch.full(ta.shape, 7, dtype=torch.uint8, device="cuda")
                mb = torch.full(tb.shape, 7, dtype=torch.uint8, device="cuda")
                p.edge_detect(ta, ma, stream=s1)
                p.edge_detect(tb, mb, stream=s2)
                outs.append((ma, mb))
            torch.cuda.synchronize()
            for ma, mb in outs:
                assert np.array_equal(ma.cpu().numpy(), lone_a)
                assert np.array_equal(mb.cpu().numpy(), lone_b)
        p.set_schedule()
    for img, m in ((a, lone_a), (b, lone_b)):
        o = oracle.edge_detect(img, 5, 1.0, THETA, stages=True)
        r = parity.compare_mask(m, o, THETA)
        assert r["mismatch"] == 0, r


@pytest.mark.parametrize("pass_mode", [1, 2, 3])
def test_batch_larger_than_its_table(hx, pass_mode):
    """Tall one-column images have many tiles per pixel.  Here a context's
    table holds about 4300 pass-1 tiles (the batch's pixels in full tiles,
    twice, plus 16 per image plus 4096): six 2^15 x 1 images (512 tiles
    each) fit together, the 300000 x 1 image (4688 tiles) alone does not
    (it runs in the per-image form) and the 3 x 20000 one follows in a
    group of its own.  Every mask matches the oracle and the maxima are
    exact."""
    heights = [1 << 15] * 6 + [300000]
    imgs = [synth.image(h, 1, 93, i) for i, h in enumerate(heights)]
    imgs.append(synth.image(3, 20000, 93, 99))
    srcs = [torch.from_numpy(x).cuda() for x in imgs]
    npx = sum(x.size for x in imgs)
    with hx.Pipeline(theta=THETA, max_pixels=npx, max_images=len(imgs),
                     pass_mode=pass_mode) as p:
        before = p.memory()
        dmax = torch.zeros(len(srcs), device="cuda")
        print(f"pass {pass_mode}: {len(srcs)} images, {npx} px", flush=True)
        masks = p.edge_detect_batched(srcs, dmax=dmax)
        p.sync()
        assert p.memory() == before
        got = [m.cpu().numpy() for m in masks]
        dm = dmax.cpu().numpy()
    for x, m, M in zip(imgs, got, dm):
        o = oracle.edge_detect(x, 5, 1.0, THETA, stages=True)
        r = parity.compare_mask(m, o, THETA)
        assert r["mismatch"] == 0 and parity.exempt_bounded(r), (x.shape, r)
        assert abs(M - o["M"]) <= 1e-5 * max(o["M"], 1e-30), (x.shape, M, o["M"])


def test_forms_not_created_are_refused(hx):
    """A pipeline created for batched calls only refuses the per-image fused
    form, the stage hook and SRAD (nothing is enqueued), and still serves
    batched calls."""
    src = torch.from_numpy(synth.image(200, 300, 94, 0)).cuda()
    with hx.Pipeline(theta=THETA, max_pixels=1 << 18, max_images=4, forms=hx.FORM_BATCH,
                     batch_contexts=1) as p:
        p.set_schedule(256, 32, 4, hx.PASS_STORE)
        with pytest.raises(hx.HxError) as ei:
            p.edge_detect(src)
        assert ei.value.status == hx.HX_E_UNSUPPORTED
        p.set_schedule()
        with pytest.raises(hx.HxError) as ei:
            p.edge_detect_stages(src)
        assert ei.value.status == hx.HX_E_UNSUPPORTED
        J = torch.from_numpy(synth.speckle(64, 64)).cuda()
        with pytest.raises(hx.HxError) as ei:
            p.srad(J, 1, 0.5)
        assert ei.value.status == hx.HX_E_UNSUPPORTED
        m = p.edge_detect_batched([src])[0].cpu().numpy()
    o = oracle.edge_detect(src.cpu().numpy(), 5, 1.0, THETA, stages=True)
    assert parity.compare_mask(m, o, THETA)["mismatch"] == 0
