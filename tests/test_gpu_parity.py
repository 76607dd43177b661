"""Parity of the HIP path (through the C ABI) with the fp64 oracle.

Every input is a seeded synthetic image (paper_2503_10855_amd.synth); the
oracle and the HIP path see the same array.  Tolerances: tests/parity.py.
"""
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


@pytest.fixture(scope="module")
def hx():
    from paper_2503_10855_amd import hx as mod
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ora(img, ks=5, sigma=1.0):
    return oracle.edge_detect(img, ks, sigma, THETA, stages=True)


def ora_many(imgs, ks=5, sigma=1.0):
    n = min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(n) as ex:
        return list(ex.map(lambda a: ora(a, ks, sigma), imgs))


def assert_mask(mask, o, what=""):
    r = parity.compare_mask(mask, o, THETA)
    print(f"{what} mask: {r}", flush=True)
    assert r["mismatch"] == 0, (what, r)
    # Exempt pixels may differ by the reading of the tolerance; on these
    # seeded inputs none does.
    assert parity.exempt_bounded(r), (what, r)


# Sizes spanning several sweep strips/bands plus ragged tails, and the
# degenerate shapes of the method (one row, one column, one pixel).
SIZES = [(1, 1), (1, 7), (7, 1), (2, 2), (5, 5), (3, 300), (67, 300),
         (130, 517), (256, 256), (64, 249), (65, 250), (66, 252), (67, 253),
         (200, 1000), (300, 61)]

SCHEDULES = [
    (16, 16, 1, 1, 0), (32, 16, 1, 1, 0), (64, 32, 1, 1, 0), (16, 32, 1, 1, 0),
    (64, 16, 2, 1, 0), (128, 32, 2, 1, 0), (256, 64, 2, 1, 0),
    (64, 32, 3, 1, 0), (128, 16, 3, 1, 0), (256, 128, 3, 1, 0),
    (64, 16, 4, 1, 0), (64, 128, 4, 1, 0), (128, 32, 4, 1, 0),
    (256, 16, 4, 1, 0), (256, 64, 4, 1, 0), (256, 128, 4, 1, 0), (256, 8, 4, 1, 0),
    (128, 8, 3, 1, 0),
    (64, 64, 4, 2, 0), (128, 16, 4, 2, 0), (256, 32, 4, 2, 0), (256, 64, 4, 2, 0),
    (256, 64, 4, 3, 0), (256, 32, 4, 3, 0), (256, 48, 4, 3, 0), (256, 96, 4, 3, 0),
    (256, 16, 4, 3, 0), (256, 24, 4, 3, 0),
    (256, 160, 4, 3, 0),
    (64, 16, 1, 1, 1), (32, 32, 1, 1, 2),
]


@pytest.mark.parametrize("ks,sigma", [(5, 1.0), (7, 1.5), (3, 0.8)])
@pytest.mark.parametrize("shape", SIZES)
def test_stage_parity(hx, shape, ks, sigma):
    img = synth.image(*shape, config_seed=21, index=shape[0] * 1000 + shape[1])
    o = ora(img, ks, sigma)
    with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA) as p:
        st = p.edge_detect_stages(dev(img))
        torch.cuda.synchronize()
        st = {k: v.cpu().numpy() for k, v in st.items()}
    st["M"] = st["M"][0]
    r = parity.compare_stages(st, o, THETA)
    print(shape, ks, r, flush=True)
    for k in ("B", "L", "G"):
        assert r[k][0] == 0, (k, r[k])
    assert r["M_ok"], (st["M"], o["M"])
    assert r["Z_mismatch"] == 0
    assert r["mask"]["mismatch"] == 0, r["mask"]
    assert parity.exempt_bounded(r["mask"]), r["mask"]


@pytest.mark.parametrize("ks,sigma", [(5, 1.0), (7, 1.5)])
@pytest.mark.parametrize("shape", [(1, 1), (7, 1), (3, 300), (130, 517),
                                   (256, 256), (300, 61), (70, 1100)])
def test_every_schedule_bit_identical(hx, shape, ks, sigma):
    """Every schedule (tile shape x fusion depth x pass mode x reduction)
    computes each pixel with the same operation sequence, so masks and M
    must be bit-identical; a halo, clamp or race bug breaks this."""
    img = synth.image(*shape, config_seed=22, index=shape[0] + shape[1])
    src = dev(img)
    ref_mask = ref_m = None
    with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA) as p:
        for sch in SCHEDULES:
            p.set_schedule(*sch)
            dmax = torch.full((1,), -1.0, device="cuda")
            mask = torch.full(shape, 7, dtype=torch.uint8, device="cuda")
            p.edge_detect(src, mask, dmax)
            torch.cuda.synchronize()
            m, M = mask.cpu().numpy(), float(dmax.cpu()[0])
            if ref_mask is None:
                ref_mask, ref_m = m, M
                assert_mask(m, ora(img, ks, sigma), f"{shape} {sch}")
            assert np.array_equal(m, ref_mask), (shape, sch)
            assert M == ref_m, (shape, sch, M, ref_m)


@pytest.mark.parametrize("ks,sigma", [(5, 1.0), (7, 1.5)])
@pytest.mark.parametrize("pass_mode", [1, 2, 3])
def test_batched_equals_per_image(hx, ks, sigma, pass_mode):
    sizes = [(1, 1), (64, 64), (5, 900), (333, 17), (256, 256), (130, 517),
             (1080, 1920), (2, 3), (700, 65), (64, 249)]
    imgs = [synth.image(h, w, 23, i) for i, (h, w) in enumerate(sizes)]
    srcs = [dev(a) for a in imgs]
    with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA, pass_mode=pass_mode) as p:
        dmax = torch.zeros(len(imgs), device="cuda")
        print(f"batched ks={ks} pass={pass_mode}: launching", flush=True)
        masks = p.edge_detect_batched(srcs, dmax=dmax)
        p.sync()
        print("batched: done; per-image calls", flush=True)
        one = []
        for s in srcs:
            d1 = torch.zeros(1, device="cuda")
            m1 = p.edge_detect(s, dmax=d1)
            torch.cuda.synchronize()
            one.append((m1.cpu().numpy(), float(d1.cpu()[0])))
    os_ = ora_many(imgs, ks, sigma)
    for i, (m, (m1, M1), o) in enumerate(zip(masks, one, os_)):
        m = m.cpu().numpy()
        assert np.array_equal(m, m1), (i, sizes[i])
        assert float(dmax[i].cpu()) == M1
        assert abs(M1 - o["M"]) <= 1e-5 * o["M"]
        assert_mask(m, o, f"batched {sizes[i]}")


def weak_bound_images():
    """Images on which the sampled bands of SPECULATE (8 rows at the top of
    every H // 4 rows for these heights) see a poor lower bound of the max,
    or none at all, so pass 1 lists many or most pixels: the strongest edge
    sits between the bands, or the bands are flat (bound 0: every pixel
    with Z = 1 and G > 0 is listed)."""
    out = []
    a = synth.image(300, 700, 26, 0) * 0.2  # bands at rows 0, 75, 150, 225
    a[30:60, 200:260] += 5.0            # the strongest edge, between bands
    out.append(a.astype(np.float32))
    b = synth.image(290, 513, 26, 1)
    for y0 in range(0, 290, 72):        # flat over each band and its halo
        b[max(0, y0 - 4):y0 + 20] = 0.3
    out.append(b.astype(np.float32))
    rng = np.random.default_rng(np.random.SeedSequence([26, 2]))
    out.append(rng.uniform(0, 1, (200, 333)).astype(np.float32))  # pure noise
    c = np.full((140, 260), 0.5, np.float32)
    c[:, 130:] = 0.25                   # one vertical step through every band
    out.append(c)
    return out


@pytest.mark.parametrize("ks,sigma", [(5, 1.0), (3, 0.8), (7, 1.5)])
def test_speculate_with_weak_bound(hx, ks, sigma):
    """SPECULATE is exact whatever its bound: per image and batched, its
    masks equal RECOMPUTE's bit for bit and the oracle's."""
    imgs = weak_bound_images()
    srcs = [dev(a) for a in imgs]
    res = {}
    for pm in (2, 3):
        with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA, pass_mode=pm) as p:
            dmax = torch.zeros(len(imgs), device="cuda")
            print(f"weak bound ks={ks} pass={pm}: batched", flush=True)
            masks = p.edge_detect_batched(srcs, dmax=dmax)
            p.sync()
            one = [p.edge_detect(s).cpu().numpy() for s in srcs]
            torch.cuda.synchronize()
            res[pm] = ([m.cpu().numpy() for m in masks], one, dmax.cpu().numpy())
    for i, a in enumerate(imgs):
        assert np.array_equal(res[3][0][i], res[2][0][i]), i
        assert np.array_equal(res[3][1][i], res[2][0][i]), i
        assert res[3][2][i] == res[2][2][i], i
        assert_mask(res[3][0][i], ora(a, ks, sigma), f"weak bound {i} {a.shape}")


def test_speculate_bounds_never_leak_between_batches(hx):
    """SPECULATE's bounds persist in each batch context and are told apart
    by an epoch; a bound left by an earlier batch with a brighter image in
    the same slot must never be used (it would exceed the dim image's max
    and clear its edges).  Alternate bright and dim batches over every
    context, twice, and compare with the per-image result each time."""
    bright = synth.image(200, 300, 27, 0) * 8.0
    dim = synth.image(200, 300, 27, 1) * 0.5
    refs = {}
    with hx.Pipeline(theta=THETA, pass_mode=3) as p:
        for name, a in (("bright", bright), ("dim", dim)):
            p.set_schedule(64, 16, 1)  # depth 1: no bound involved
            refs[name] = p.edge_detect(dev(a)).cpu().numpy()
            p.set_schedule()
        for call in range(14):
            name, a = (("bright", bright), ("dim", dim))[call % 2]
            print(f"epoch test call {call}: {name}", flush=True)
            m = p.edge_detect_batched([dev(a), dev(dim)])
            p.sync()
            assert np.array_equal(m[0].cpu().numpy(), refs[name]), (call, name)
            assert np.array_equal(m[1].cpu().numpy(), refs["dim"]), call
    assert refs["dim"].sum() > 0
    assert_mask(refs["dim"], ora(dim), "dim")


@pytest.mark.skip(reason="the single-kernel batched variant, in which pass-2 "
                  "workgroups spin until their image's pass-1 items are done, "
                  "went silent on the GPU twice (the second time after its "
                  "per-poll L2 invalidate was removed) and is switched off; "
                  "batches now run as wait-free pass-1 / pass-2 kernels")
def test_single_kernel_wait_queue_batch(hx):
    raise AssertionError("switched off")


@pytest.mark.parametrize("pass_mode", [2, 3])
def test_batched_graph_replay_with_changing_batches(hx, pass_mode):
    """Batches of different compositions on one pipeline: the first call of
    a composition on a batch context launches directly, a repeat replays a
    captured graph (re-captured when the item counts change).  Each
    composition runs 8 times (more calls than contexts), with eager work
    on the outputs between the calls; every result must be the first one,
    which must match the oracle."""
    with hx.Pipeline(theta=THETA, pass_mode=pass_mode) as p:
        for rep, sizes in enumerate([[(100, 200), (50, 50)],
                                     [(1, 1), (300, 301), (64, 64), (7, 900)],
                                     [(100, 200)],
                                     [(100, 200), (50, 50)]]):
            imgs = [synth.image(h, w, 24 + rep, i) for i, (h, w) in enumerate(sizes)]
            srcs = [dev(a) for a in imgs]
            masks = [torch.empty(a.shape, dtype=torch.uint8, device="cuda") for a in imgs]
            dmax = torch.zeros(len(imgs), device="cuda")
            batch = p.prepare_batch(srcs, masks, dmax)
            first = None
            for call in range(8):
                print(f"replay {rep} call {call}: launching", flush=True)
                for m in masks:
                    m.fill_(7)
                dmax.fill_(-1.0)
                batch.run()
                p.sync()
                got = ([m.cpu().numpy() for m in masks], dmax.cpu().numpy())
                if first is None:
                    first = got
                    for a, m in zip(imgs, got[0]):
                        assert_mask(m, ora(a), f"replay {rep} {a.shape}")
                else:
                    for m0, m1 in zip(first[0], got[0]):
                        assert np.array_equal(m0, m1), (rep, call)
                    assert np.array_equal(first[1], got[1]), (rep, call)


@pytest.mark.parametrize("sched", [(256, 64, 4, 1, 0), (64, 16, 1, 1, 0),
                                   (128, 32, 4, 2, 0), (256, 64, 4, 3, 0)])
def test_pitch_and_misalignment(hx, sched):
    """Padded row pitches and bases that are not 16-byte aligned take the
    scalar load/store paths; results must not change and bytes outside the
    image must stay untouched."""
    H, W = 97, 301
    img = synth.image(H, W, 25, 0)
    big = torch.zeros((H, W + 13 + 1), dtype=torch.float32, device="cuda")
    src = big[:, 1:W + 1]
    src.copy_(dev(img))
    mbuf = torch.full((H, W + 6), 9, dtype=torch.uint8, device="cuda")
    mask = mbuf[:, 1:W + 1]
    with hx.Pipeline(theta=THETA) as p:
        p.set_schedule(*sched)
        p.edge_detect(src, mask)
        ref = p.edge_detect(dev(img))
        torch.cuda.synchronize()
    mb = mbuf.cpu().numpy()
    assert np.all(mb[:, 0] == 9) and np.all(mb[:, W + 1:] == 9)
    assert np.array_equal(mask.cpu().numpy(), ref.cpu().numpy())
    assert_mask(ref.cpu().numpy(), ora(img), "pitch")


@pytest.mark.parametrize("ks,sigma", [(5, 1.0), (7, 1.5)])
def test_extreme_aspect_ratios(hx, ks, sigma):
    """One-row, one-column and very thin images, far longer than a sweep
    strip or band in one direction: per image, and batched under every pass
    structure, against the oracle."""
    shapes = [(1, 70001), (70001, 1), (2, 40000), (40000, 3), (5, 4099), (4099, 6)]
    imgs = [synth.image(h, w, 28, i) for i, (h, w) in enumerate(shapes)]
    os_ = ora_many(imgs, ks, sigma)
    srcs = [dev(a) for a in imgs]
    for pm in (1, 2, 3):
        with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA, pass_mode=pm) as p:
            print(f"extreme shapes ks={ks} pass={pm}", flush=True)
            masks = p.edge_detect_batched(srcs)
            one = [p.edge_detect(s) for s in srcs]
            p.sync()
            torch.cuda.synchronize()
            for i, (m, m1, o) in enumerate(zip(masks, one, os_)):
                m = m.cpu().numpy()
                assert np.array_equal(m, m1.cpu().numpy()), (pm, shapes[i])
                assert_mask(m, o, f"pass {pm} {shapes[i]}")


def test_degenerate_images(hx):
    with hx.Pipeline(theta=THETA) as p:
        for val in (0.0, 0.37):
            for shape in ((1, 1), (9, 9), (300, 513)):
                src = torch.full(shape, val, dtype=torch.float32, device="cuda")
                dmax = torch.full((1,), -1.0, device="cuda")
                mask = p.edge_detect(src, dmax=dmax)
                torch.cuda.synchronize()
                assert int(mask.sum()) == 0 and float(dmax[0]) == 0.0


def test_abi_rejects_bad_arguments(hx):
    import ctypes
    lib = hx.raw()
    with hx.Pipeline(theta=THETA, max_pixels=10000, max_images=4) as p:
        src = torch.zeros((50, 60), device="cuda")
        mask = torch.full((50, 60), 5, dtype=torch.uint8, device="cuda")
        good = hx.image_desc(src, mask)

        def call(**kw):
            d = hx.Image(good.src, good.height, good.width, good.src_pitch,
                         good.mask, good.mask_pitch)
            for k, v in kw.items():
                setattr(d, k, v)
            return lib.hx_edge_detect(p.handle, ctypes.byref(d), None, None)

        assert call(src=None) == hx.HX_E_INVALID
        assert call(mask=None) == hx.HX_E_INVALID
        assert call(height=0) == hx.HX_E_INVALID
        assert call(width=-3) == hx.HX_E_INVALID
        assert call(src_pitch=59) == hx.HX_E_INVALID
        assert call(mask_pitch=10) == hx.HX_E_INVALID
        assert call(height=200, width=60, src_pitch=60, mask_pitch=60) == hx.HX_E_INVALID
        assert lib.hx_edge_detect(p.handle, None, None, None) == hx.HX_E_INVALID
        arr = (hx.Image * 5)(*([good] * 5))
        assert lib.hx_edge_detect_batched(p.handle, arr, 5, None, None) == hx.HX_E_INVALID
        assert lib.hx_edge_detect_batched(p.handle, arr, 0, None, None) == hx.HX_E_INVALID
        assert lib.hx_edge_detect_batched(p.handle, arr, 4, None, None) == hx.HX_E_INVALID
        bad = hx.Schedule(48, 16, 1, 1, 0)
        assert lib.hx_pipeline_set_schedule(p.handle, ctypes.byref(bad)) == hx.HX_E_INVALID
        bad = hx.Schedule(256, 64, 4, 1, 2)
        assert lib.hx_pipeline_set_schedule(p.handle, ctypes.byref(bad)) == hx.HX_E_INVALID
        bad = hx.Schedule(128, 64, 4, 3, 0)  # SPECULATE needs the 256x64 tile
        assert lib.hx_pipeline_set_schedule(p.handle, ctypes.byref(bad)) == hx.HX_E_INVALID
        bad = hx.Schedule(256, 64, 4, 4, 0)
        assert lib.hx_pipeline_set_schedule(p.handle, ctypes.byref(bad)) == hx.HX_E_INVALID
        torch.cuda.synchronize()
        assert int((mask != 5).sum()) == 0  # nothing was enqueued
    with pytest.raises(hx.HxError):
        hx.Pipeline(ksize=9).set_schedule(256, 64, 4)


FUSED_STAGE_SCHEDULES = [
    ((64, 16, 2, 1, 0), ("B", "Z", "G")), ((256, 64, 2, 1, 0), ("B", "Z", "G")),
    ((128, 32, 2, 1, 0), ("B", "Z", "G")),
    ((64, 32, 3, 1, 0), ("L", "Z", "G")), ((256, 16, 3, 1, 0), ("L", "Z", "G")),
    ((256, 128, 3, 1, 0), ("L", "Z", "G")),
]


@pytest.mark.parametrize("ks,sigma", [(5, 1.0), (7, 1.5), (3, 0.8)])
@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (3, 300), (130, 517),
                                   (256, 256), (70, 1100), (40, 251), (40, 252)])
def test_fused_depth_stages(hx, shape, ks, sigma):
    """The stage planes the fused depths keep in memory -- B, Z and G at
    depth 2 (its register sweep writes B and G^2, its LDS kernel Z), L, Z
    and G at depth 3 -- equal depth 1's bit for bit under every tile shape,
    and the oracle's within the stated tolerance."""
    img = synth.image(*shape, config_seed=24, index=shape[0] * 7 + shape[1])
    o = ora(img, ks, sigma)
    with hx.Pipeline(ksize=ks, sigma=sigma, theta=THETA) as p:
        ref = {k: v.cpu().numpy() for k, v in p.edge_detect_stages(dev(img)).items()}
        for sched, keys in FUSED_STAGE_SCHEDULES:
            p.set_schedule(*sched)
            st = {k: v.cpu().numpy() for k, v in
                  p.edge_detect_stages(dev(img), stages=keys).items()}
            for k in keys + ("M", "mask"):
                assert np.array_equal(st[k], ref[k]), (shape, sched, k)
            for k in keys:
                if k in ("B", "L", "G"):
                    bad, err = parity.float_stage_ok(st[k], o[k])
                    assert bad == 0, (shape, sched, k, err)
        p.set_schedule()
    band, amb = parity.exemptions(o, THETA)
    assert int(((ref["Z"] != o["Z"]) & ~amb).sum()) == 0
