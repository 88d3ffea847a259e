"""jpt_mark_blocks_static (the mark entry point that allocates nothing: its
scan scratch is a device array inside the library) against jpt_mark_blocks
with the caller's frame->scan, through the C ABI.

Both run on identical inputs and state; every integer output must be
identical: the counters, the work list, the block -> slot table and, for
the LRU cache, its whole per-slot state; the frames decoded and resolved
from them must be identical bit for bit.  Calls come in a row on the same
device and scratch: a larger scene first, then a smaller one (fewer scan
entries, so stale contents of the larger call would show), then an LRU
sequence."""
import numpy as np
import pytest

from paper_2510_08166_amd.synth import configs

pytestmark = pytest.mark.gpu


def same_state(rA, rB, lru):
    import torch
    torch.cuda.synchronize()
    from paper_2510_08166_amd import jpt
    cA, cB = rA.frame.counters_host(), rB.frame.counters_host()
    assert np.array_equal(cA, cB), (cA, cB)
    n = int(cA[jpt.CTR_ITEMS])
    assert np.array_equal(rA.frame.work_items(), rB.frame.work_items())
    assert torch.equal(rA.frame.vis, rB.frame.vis)
    assert torch.equal(rA.cache.slot_of, rB.cache.slot_of)
    if lru:
        for name in ("owner", "last_used", "resident", "free_stack", "meta"):
            assert torch.equal(getattr(rA.cache, name), getattr(rB.cache, name)), name
    return n


def pair(wl, policy=0, n_slots=None):
    from paper_2510_08166_amd import jpt
    rA = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, policy=policy, n_slots=n_slots,
                      idct_mode=jpt.IDCT_FUSED_F32)
    rB = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, policy=policy, n_slots=n_slots, host=rA.host,
                      idct_mode=jpt.IDCT_FUSED_F32)
    # rB's own scan buffer is never used: poison it
    rB.frame.scan.fill_(-1)
    return rA, rB


def frame_pair(rA, rB, lru=False):
    import torch
    from paper_2510_08166_amd import jpt
    rA.mark()
    rB.frame.c.frame_no = rB.frame_no
    jpt.mark_blocks_static(rB.scene, rB.views, rB.filter, rB.frame, rB.cache, rB.tuning)
    rB.frame_no += 1
    n = same_state(rA, rB, lru)
    for r in (rA, rB):
        r.decode()
        r.resolve()
    torch.cuda.synchronize()
    assert rA.frame.counters_host()[jpt.CTR_ERROR] == 0
    assert np.array_equal(rA.views.frame_host(), rB.views.frame_host())
    return n


def test_static_scratch_mark_matches_caller_scratch(gpu):
    # 1. a larger scene (several textures and levels, bilinear)
    big = configs.quad_scene(81, 6, 256, 50, 90, 5, 320, 200, 30, filt=configs.FILTER_BILINEAR)
    rA, rB = pair(big)
    n1 = frame_pair(rA, rB)
    print("larger scene: %d blocks, %d items" % (rA.scene.n_blocks, n1), flush=True)
    assert n1 > 0
    # 2. right after it, on the same scratch, a smaller scene (fewer block ids)
    small = configs.tiny()
    sA, sB = pair(small)
    assert sA.scene.n_blocks < rA.scene.n_blocks
    n2 = frame_pair(sA, sB)
    print("smaller scene: %d blocks, %d items" % (sA.scene.n_blocks, n2), flush=True)
    assert n2 == 256
    # 3. an LRU sequence (the scratch also holds the two per-tile scans)
    import oracle
    from oracle import parity
    from paper_2510_08166_amd import jpt
    wl = configs.heavy(seed=33, n_tex=8, sides=(64, 128, 256), W=256, H=160, n_quads=30, n_frames=4)
    osc = oracle.Scene(wl.textures)
    cap = max(len(parity.visible_blocks(osc, [g], wl.filter)) for g in wl.views) + 4  # evictions every frame
    lA = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, n_slots=cap, policy=jpt.CACHE_LRU,
                      idct_mode=jpt.IDCT_FUSED_F32)
    lB = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, n_slots=cap, policy=jpt.CACHE_LRU, host=lA.host,
                      idct_mode=jpt.IDCT_FUSED_F32)
    lB.frame.scan.fill_(-1)
    evicted = 0
    for g in wl.views:
        lA.set_views([g])
        lB.set_views([g])
        n = frame_pair(lA, lB, lru=True)
        evicted += int(lA.frame.counters_host()[jpt.CTR_EVICTED])
        print("LRU frame: %d items, evicted %d" % (n, lA.frame.counters_host()[jpt.CTR_EVICTED]), flush=True)
    assert evicted > 0
