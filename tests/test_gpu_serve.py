"""The serving loop: continuous batching under an HBM budget.  Each
request's mask must be the same served alone and served in a mix (bit for
bit), match the per-image call, and match the oracle."""
import time

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


def collect(srv, tickets, shapes, timeout=60.0):
    out = {}
    t_end = time.time() + timeout
    while len(out) < len(tickets):
        assert time.time() < t_end, f"{len(tickets) - len(out)} requests never completed"
        for t, sh in zip(tickets, shapes):
            if t in out:
                continue
            r = srv.poll(t, sh)
            if r is not None:
                out[t] = r
        time.sleep(0.001)
    return [out[t] for t in tickets]


def test_serve_alone_equals_in_mix(hx):
    sizes = synth.log_uniform_sizes(48, 64, 1024, 77)
    imgs = [synth.image(h, w, 78, i) for i, (h, w) in enumerate(sizes)]
    picks = [0, 17, 40]
    with hx.Pipeline(theta=THETA, max_pixels=1 << 24, max_images=64,
                     forms=hx.FORM_BATCH) as p:
        alone = {}
        for i in picks:
            with hx.Server(p, hbm_budget=256 << 20, streams=2, max_batch=16) as srv:
                print(f"serve alone {i} {sizes[i]}", flush=True)
                t = srv.submit(imgs[i])
                alone[i] = collect(srv, [t], [sizes[i]])[0][0]
        print("serve mix of 48", flush=True)
        with hx.Server(p, hbm_budget=256 << 20, streams=3, max_batch=16) as srv:
            tickets = []
            for a in imgs:
                tickets.append(srv.submit(a))
                time.sleep(0.0005)  # arrivals spread over the run
            res = collect(srv, tickets, sizes)
            st = srv.stats()
        print(f"stats {st}", flush=True)
        assert st["completed"] == len(imgs) and st["batches"] >= 2
    with hx.Pipeline(theta=THETA, max_pixels=1 << 24, max_images=64) as q:
        per_image = [q.edge_detect(torch.from_numpy(a).cuda()).cpu().numpy() for a in imgs]
    for i in picks:
        assert np.array_equal(alone[i], res[i][0]), i
    for i, ((m, lat), ref) in enumerate(zip(res, per_image)):
        assert np.array_equal(m, ref), i
        assert lat > 0
    for i in range(0, len(imgs), 6):
        o = oracle.edge_detect(imgs[i], 5, 1.0, THETA, stages=True)
        r = parity.compare_mask(res[i][0], o, THETA)
        assert r["mismatch"] == 0, (i, r)


def test_serve_admission_respects_budget(hx):
    """The budget covers the pipeline's own scratch and the request buffers:
    with room for about two 512x512 requests beyond the scratch, the peak
    of the two together stays within it, and a request that could never
    fit is refused."""
    sizes = [(512, 512)] * 12 + [(300, 700)] * 4
    imgs = [synth.image(h, w, 79, i) for i, (h, w) in enumerate(sizes)]
    with hx.Pipeline(theta=THETA, max_pixels=1 << 20, max_images=16, forms=hx.FORM_BATCH,
                     batch_contexts=2) as p:
        own, _, allocs = p.memory()
        budget = own + (3 << 20)
        with hx.Server(p, hbm_budget=budget, streams=2, max_batch=8) as srv:
            print(f"serve under a budget of {budget} bytes ({own} of pipeline scratch)",
                  flush=True)
            tickets = [srv.submit(a) for a in imgs]
            res = collect(srv, tickets, sizes)
            st = srv.stats()
            with pytest.raises(hx.HxError) as ei:  # 5 MiB: within max_pixels, not the arena
                srv.submit(np.zeros((1024, 1024), np.float32))
            assert ei.value.status == hx.HX_E_BUSY
        # A budget that does not exceed the scratch is refused.
        with pytest.raises(hx.HxError) as ei:
            hx.Server(p, hbm_budget=own, streams=2, max_batch=8)
        assert ei.value.status == hx.HX_E_INVALID
        assert p.memory() == (own, p.memory()[1], allocs)
    with hx.Pipeline(theta=THETA, max_pixels=1 << 22, max_images=16) as q:
        refs = [q.edge_detect(torch.from_numpy(a).cuda()).cpu().numpy() for a in imgs]
    print(f"stats {st}", flush=True)
    assert own + st["peak_bytes"] <= budget and st["completed"] == len(imgs)
    for (m, _), ref in zip(res, refs):
        assert np.array_equal(m, ref)


def test_serve_submit_never_blocks(hx):
    """A full pinned pool makes submit return at once (pending), not wait:
    the pool is freed only by polling, which a single-threaded caller could
    then never reach.  After the finished requests are collected the same
    request goes in."""
    side = 2048  # 16 MiB in + 4 MiB mask per request; the pool holds 64 MiB
    imgs = [synth.image(side, side, 80, i) for i in range(5)]
    with hx.Pipeline(theta=THETA, max_pixels=1 << 23, max_images=4, forms=hx.FORM_BATCH,
                     batch_contexts=2) as p:
        own = p.memory()[0]
        with hx.Server(p, hbm_budget=own + (48 << 20), streams=2, max_batch=2) as srv:
            print("serve: filling the pinned pool", flush=True)
            tickets = []
            refused = None
            for i, a in enumerate(imgs):
                t = srv.try_submit(a)
                if t is None:
                    refused = i
                    break
                tickets.append(t)
            assert refused is not None and refused >= 2, refused
            with pytest.raises(hx.HxError) as ei:
                srv.submit(imgs[refused])
            assert ei.value.status == hx.HX_E_PENDING
            shapes = [(side, side)] * len(tickets)
            res = collect(srv, tickets, shapes)
            t = srv.submit(imgs[refused])
            last = collect(srv, [t], [(side, side)])[0]
    with hx.Pipeline(theta=THETA, max_pixels=1 << 23, max_images=4) as q:
        ref = q.edge_detect(torch.from_numpy(imgs[refused]).cuda()).cpu().numpy()
        refs = [q.edge_detect(torch.from_numpy(a).cuda()).cpu().numpy() for a in imgs[:refused]]
    assert np.array_equal(last[0], ref)
    for (m, _), r in zip(res, refs):
        assert np.array_equal(m, r)


def test_serve_zero_copy_slots(hx):
    """Reserve / commit / view / release: the caller writes each request into
    its pinned slot and reads the mask where it lies; the masks equal the
    per-image ones.  A cancelled slot gives its room back, and tickets in
    the wrong state are refused."""
    sizes = [(300, 500), (1080, 1920), (64, 64), (517, 259), (1, 300)]
    imgs = [synth.image(h, w, 83, i) for i, (h, w) in enumerate(sizes)]
    with hx.Pipeline(theta=THETA, max_pixels=1 << 23, max_images=8, forms=hx.FORM_BATCH,
                     batch_contexts=2) as p:
        own = p.memory()[0]
        with hx.Server(p, hbm_budget=own + (256 << 20), streams=2, max_batch=4) as srv:
            print("serve: zero-copy slots", flush=True)
            t0, slot0 = srv.reserve((2048, 2048))
            srv.cancel(t0)
            with pytest.raises(hx.HxError) as ei:
                srv.commit(t0)
            assert ei.value.status == hx.HX_E_NOT_FOUND
            tickets = []
            for a in imgs:
                t, slot = srv.reserve(a.shape)
                assert slot.shape == a.shape and slot.dtype == np.float32
                slot[...] = a
                tickets.append(t)
            with pytest.raises(hx.HxError) as ei:
                srv.view(tickets[0], sizes[0])
            assert ei.value.status == hx.HX_E_INVALID
            for t in tickets:
                srv.commit(t)
            with pytest.raises(hx.HxError) as ei:
                srv.commit(tickets[0])
            assert ei.value.status == hx.HX_E_INVALID
            got = {}
            deadline = time.time() + 60
            while len(got) < len(tickets) and time.time() < deadline:
                for t, shp in zip(tickets, sizes):
                    if t in got:
                        continue
                    r = srv.view(t, shp)
                    if r is not None:
                        m, lat, svc = r
                        assert not m.flags.writeable and lat >= svc >= 0
                        got[t] = m.copy()
                        srv.release(t)
                time.sleep(1e-4)
            assert len(got) == len(tickets)
            with pytest.raises(hx.HxError) as ei:
                srv.release(tickets[0])
            assert ei.value.status == hx.HX_E_NOT_FOUND
    with hx.Pipeline(theta=THETA, max_pixels=1 << 23, max_images=8) as q:
        refs = [q.edge_detect(torch.from_numpy(a).cuda()).cpu().numpy() for a in imgs]
    for t, ref in zip(tickets, refs):
        assert np.array_equal(got[t], ref)
