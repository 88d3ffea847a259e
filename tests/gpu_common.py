"""Shared helpers of the GPU parity tests: run one frame through the C ABI
and compare everything it produced with the oracle."""
import numpy as np

import oracle
from oracle import parity


def run(wl, idct_mode=0, **kw):
    import torch
    from paper_2510_08166_amd import jpt
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, **kw)
    r.mark()
    r.decode(idct_mode=idct_mode)
    r.resolve()
    torch.cuda.synchronize()
    ctr = r.frame.counters_host()
    items = r.frame.work_items()
    n = len(items)
    coef = r.frame.coef[: n * jpt.ITEM_COEFS].cpu().numpy().reshape(n, 6, 64)
    n_new = min(int(ctr[jpt.CTR_NEW]), r.cache.n_slots)
    tiles = r.cache.texels[: n_new * 256].cpu().numpy().view(np.uint32).reshape(n_new, 256)
    frames = [r.views.frame_host(i) for i in range(r.views.n)]
    return r, ctr, items, coef, tiles, frames


def full_parity(wl, coef_sample=None, texel_sample=None, full_render=True, idct_mode=0, tuning=None, host=None):
    from paper_2510_08166_amd import jpt
    osc = oracle.Scene(wl.textures)
    r, ctr, items, coef, tiles, frames = run(wl, idct_mode, tuning=tuning, host=host)
    print("%s: items %d new %d visible %d err %x" % (wl.name, ctr[jpt.CTR_ITEMS], ctr[jpt.CTR_NEW],
                                                     ctr[jpt.CTR_VISIBLE], ctr[jpt.CTR_ERROR]), flush=True)
    assert ctr[jpt.CTR_ERROR] == 0
    blocks = parity.visible_blocks(osc, wl.views, wl.filter)
    assert ctr[jpt.CTR_NEW] == len(blocks) and ctr[jpt.CTR_VISIBLE] == len(blocks)
    assert np.array_equal(items, parity.expected_items(osc, blocks))
    lc = parity.LevelCache(osc)
    if idct_mode != jpt.IDCT_FUSED_F32:   # (the fused decode writes texels only)
        assert parity.check_coefs(lc, items, coef, coef_sample) == []
    maxd, nmis, tie, dist, n = parity.check_texels(lc, blocks, tiles, texel_sample)
    print("texels: max diff %d, %d of %d channels differ, worst tie distance %.2e (%.2f of its tolerance)"
          % (maxd, nmis, n, dist, tie))
    assert maxd <= 1 and tie <= 1.0
    imgs = parity.levels_from_tiles(osc, blocks, tiles)
    for g, f in zip(wl.views, frames):
        ref, bad = osc.resolve(g, wl.filter, imgs)
        assert bad == 0
        assert np.array_equal(f, ref), "frame differs from the oracle's resolve of the GPU texels"
        if full_render:
            full, _, _ = osc.render(g, wl.filter)
            assert parity.frame_diff(f, full) <= 1
    return r, osc, blocks
