"""GPU parity at the full sizes the benchmark runs, in the launch
configuration it times (one frame of all views through the library's
graph):

  - 1080p: every work item, coefficient and texel, and the whole frame;
  - batched 16 views: every work item (blocks shared across views decoded
    once); sampled coefficients, texels and pixels;
  - heavy 4K trilinear with the LRU cache over 8 drifting frames: per frame
    the decoded set, evictions and resident set against the oracle's
    simulator; sampled coefficients, texels and pixels.

The 1080p frame and the sampled checks of the other two run in the fused
decode the benchmark times as well as in the two-kernel MFMA decode.

Sampled pixels are checked bit-exactly against the oracle's resolve over the
GPU's texels (only the blocks the sampled taps read are assembled); the
texels themselves are checked against the oracle's decode on sampled
blocks.  Slow: the workloads take minutes to generate.
"""
import time

import numpy as np
import pytest

import oracle
from oracle import parity
from paper_2510_08166_amd.synth import configs

from gpu_common import full_parity

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def log(msg):
    print(msg, flush=True)


def graph_frame(r):
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = r.capture(s)
    g.launch()
    s.synchronize()
    g.close()


def gather_tiles(r, slots):
    """Texel tiles of the given cache slots, [n, 256] RGBA8, gathered on the GPU."""
    import torch
    idx = torch.from_numpy(np.asarray(slots, np.int64)).to(r.cache.texels.device)
    return r.cache.texels.view(-1, 256)[idx].cpu().numpy().view(np.uint32)


def sampled_pixels(osc, r, frame, gbuf, filt, n, rng, slot_of):
    """Compare n random non-background pixels of a view's frame with the
    oracle's resolve over the GPU's own texels of the blocks they read."""
    fg = np.argwhere(gbuf["tex"] != oracle.BACKGROUND)
    if len(fg) == 0:
        return 0
    pick = fg[rng.choice(len(fg), min(n, len(fg)), replace=False)]
    g = np.ascontiguousarray(gbuf[pick[:, 0], pick[:, 1]]).reshape(1, -1)
    lv, x, y, w, bad = osc.taps(g, filt)
    assert bad == 0
    need = {}
    for L, xx, yy, ww in zip(lv.ravel(), x.ravel(), y.ravel(), w.ravel()):
        if ww == 0:
            continue
        L = int(L)
        bx, by = int(xx) >> 4, int(yy) >> 4
        need[(L, bx, by)] = int(osc.blk_base[L]) + by * int(osc.blk_cols[L]) + bx
    keys = list(need)
    slots = slot_of[np.array([need[k] for k in keys], np.int64)]
    assert not np.any(slots == 0xFFFFFFFF), "a tap's block has no slot"
    tiles = gather_tiles(r, slots)
    imgs = {}
    for (L, bx, by), t in zip(keys, tiles):
        if L not in imgs:
            imgs[L] = np.zeros((int(osc.lev_h[L]), int(osc.lev_w[L]), 3), np.uint8)
        t = t.reshape(16, 16).view(np.uint8).reshape(16, 16, 4)[:, :, :3]
        h = min(16, int(osc.lev_h[L]) - 16 * by); wd = min(16, int(osc.lev_w[L]) - 16 * bx)
        imgs[L][16 * by:16 * by + h, 16 * bx:16 * bx + wd] = t[:h, :wd]
    ref, bad = osc.resolve(g, filt, imgs)
    assert bad == 0
    got = frame[pick[:, 0], pick[:, 1]]
    assert np.array_equal(got, ref.ravel()), "sampled pixels differ from the oracle's resolve of the GPU texels"
    return len(pick)


def test_frame1080_full_size(gpu):
    import torch
    from paper_2510_08166_amd import jpt
    t0 = time.time()
    wl = configs.frame1080()
    log("1080p generated in %.1f s" % (time.time() - t0))
    r, osc, blocks = full_parity(wl)
    # the benchmark's configuration: fused decode, the frame captured;
    # bit-exact against the eager fused frame, the same work list as above
    items = r.frame.work_items()
    rf = jpt.Renderer(wl.textures, wl.views, wl.filter, idct_mode=jpt.IDCT_FUSED_F32, host=r.host)
    rf.render()
    torch.cuda.synchronize()
    tex0 = rf.cache.texels[: len(blocks) * 256].cpu().numpy()
    frame0 = rf.views.frame_host(0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = rf.capture(s)
    rf.cache.texels.zero_()
    rf.frame.work.zero_()
    torch.cuda.synchronize()
    g.launch()
    s.synchronize()
    g.close()
    ctr = rf.frame.counters_host()
    assert ctr[jpt.CTR_ERROR] == 0 and ctr[jpt.CTR_ITEMS] == len(items)
    assert np.array_equal(rf.frame.work_items(), items)
    assert np.array_equal(rf.cache.texels[: len(blocks) * 256].cpu().numpy(), tex0)
    assert np.array_equal(rf.views.frame_host(0), frame0)
    log("1080p captured fused frame: bit-exact with the eager frame")
    # and the fused frame against the oracle itself: every texel within
    # 1 LSB, the frame bit-exact against the oracle's resolve of these
    # texels and within 1 LSB of the oracle's full render
    lc = parity.LevelCache(osc)
    tiles = tex0.view(np.uint32).reshape(len(blocks), 256)
    maxd, nmis, tie, dist, nch = parity.check_texels(lc, blocks, tiles)
    log("fused texels: max diff %d, %d of %d channels differ, worst tie distance %.2e (%.2f of its tolerance)"
        % (maxd, nmis, nch, dist, tie))
    assert maxd <= 1 and tie <= 1.0
    ref, bad = osc.resolve(wl.views[0], wl.filter, parity.levels_from_tiles(osc, blocks, tiles))
    assert bad == 0 and np.array_equal(frame0, ref)
    full, _, _ = osc.render(wl.views[0], wl.filter)
    assert parity.frame_diff(frame0, full) <= 1
    log("1080p fused frame: oracle parity")


def test_batched16_sampled(gpu):
    import torch
    from paper_2510_08166_amd import jpt
    t0 = time.time()
    wl = configs.batched16(log=log)
    log("batched16 generated in %.1f s" % (time.time() - t0))
    r = jpt.Renderer(wl.textures, wl.views, wl.filter)
    graph_frame(r)
    ctr = r.frame.counters_host()
    assert ctr[jpt.CTR_ERROR] == 0
    osc = oracle.Scene(wl.textures)
    # (the MFMA two-kernel decode first, then the fused decode the benchmark times)
    blocks = parity.visible_blocks(osc, wl.views, wl.filter)
    log("visible blocks %d (GPU %d); pixels %d" % (len(blocks), ctr[jpt.CTR_VISIBLE], wl.n_pixels))
    assert ctr[jpt.CTR_VISIBLE] == len(blocks) and ctr[jpt.CTR_NEW] == len(blocks)
    items = r.frame.work_items()
    assert np.array_equal(items, parity.expected_items(osc, blocks))
    rng = np.random.default_rng(0)
    n = len(items)
    sample = np.sort(rng.choice(n, 120, replace=False))
    coef = r.frame.coef[: n * jpt.ITEM_COEFS].cpu().numpy().reshape(n, 6, 64)
    lc = parity.LevelCache(osc)
    assert parity.check_coefs(lc, items, coef, sample) == []
    slot_of = r.cache.slot_of.cpu().numpy().view(np.uint32)
    tb = blocks[np.sort(rng.choice(len(blocks), 120, replace=False))]
    maxd, nmis, tie, dist, nch = parity.check_texels(lc, tb, gather_tiles(r, slot_of[tb]))
    log("texels: max diff %d, %d of %d channels differ, worst tie distance %.2e (%.2f of its tolerance)"
        % (maxd, nmis, nch, dist, tie))
    assert maxd <= 1 and tie <= 1.0
    for v, g in enumerate(wl.views):
        sampled_pixels(osc, r, r.views.frame_host(v), g, wl.filter, 400, rng, slot_of)
    log("16 views: sampled pixels bit-exact")
    r.idct_mode = jpt.IDCT_FUSED_F32
    r.cache.texels.zero_()
    graph_frame(r)
    ctr = r.frame.counters_host()
    assert ctr[jpt.CTR_ERROR] == 0 and ctr[jpt.CTR_NEW] == len(blocks)
    assert np.array_equal(r.frame.work_items(), items)
    tb = blocks[np.sort(rng.choice(len(blocks), 120, replace=False))]
    maxd, nmis, tie, dist, nch = parity.check_texels(lc, tb, gather_tiles(r, slot_of[tb]))
    log("fused texels: max diff %d, %d of %d channels differ, worst tie distance %.2e (%.2f of its tolerance)"
        % (maxd, nmis, nch, dist, tie))
    assert maxd <= 1 and tie <= 1.0
    for v, g in enumerate(wl.views):
        sampled_pixels(osc, r, r.views.frame_host(v), g, wl.filter, 400, rng, slot_of)
    log("16 views, fused decode: sampled pixels bit-exact")


def test_heavy_lru_sequence_sampled(gpu):
    import torch
    from paper_2510_08166_amd import jpt
    t0 = time.time()
    wl = configs.heavy(log=log)
    log("heavy generated in %.1f s" % (time.time() - t0))
    slots = (2 << 30) // 1024
    r = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, policy=jpt.CACHE_LRU, n_slots=slots, max_items=1 << 20)
    views = [jpt.Views([g]) for g in wl.views]
    osc = oracle.Scene(wl.textures)
    lc = parity.LevelCache(osc)
    rng = np.random.default_rng(1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    for mode in (jpt.IDCT_MFMA_F16, jpt.IDCT_FUSED_F32):
        r.idct_mode = mode
        r.cache.reset(r.scene)
        sim = oracle.LruSim(slots)
        torch.cuda.synchronize()
        graphs = [r.capture(s, v) for v in views]
        for f, g in enumerate(wl.views):
            graphs[f].launch()
            s.synchronize()
            ctr = r.frame.counters_host()
            vis = parity.visible_blocks(osc, [g], wl.filter)
            new, ev = sim.step(f, vis)
            log("mode %d frame %d: visible %d new %d evicted %d" % (mode, f, ctr[jpt.CTR_VISIBLE], ctr[jpt.CTR_NEW],
                                                                   ctr[jpt.CTR_EVICTED]))
            assert ctr[jpt.CTR_ERROR] == 0
            assert ctr[jpt.CTR_VISIBLE] == len(vis)
            items = r.frame.work_items()
            assert np.array_equal(items, parity.expected_items(osc, np.array(new, np.uint32)))
            assert ctr[jpt.CTR_EVICTED] == len(ev)
            if f in (0, 7):
                assert np.array_equal(r.cache.resident_blocks(), np.array(sorted(sim.last_used), np.uint32))
            n = len(items)
            slot_of = r.cache.slot_of.cpu().numpy().view(np.uint32)
            if n and mode != jpt.IDCT_FUSED_F32:  # (the fused decode writes texels only)
                coef = r.frame.coef[: n * jpt.ITEM_COEFS].cpu().numpy().reshape(n, 6, 64)
                sample = np.sort(rng.choice(n, min(n, 40 if f == 0 else 10), replace=False))
                assert parity.check_coefs(lc, items, coef, sample) == []
            if f in (0, 7):
                vb = np.array(vis, np.uint32)
                tb = vb[np.sort(rng.choice(len(vb), 40, replace=False))]
                maxd, nmis, tie, dist, nch = parity.check_texels(lc, tb, gather_tiles(r, slot_of[tb]))
                log("frame %d texels: max diff %d, %d of %d channels differ, worst tie distance %.2e (%.2f of its "
                    "tolerance)" % (f, maxd, nmis, nch, dist, tie))
                assert maxd <= 1 and tie <= 1.0
                sampled_pixels(osc, r, views[f].frame_host(0), g, wl.filter, 2000, rng, slot_of)
                log("frame %d: sampled pixels bit-exact" % f)
        for gr in graphs:
            gr.close()
