"""The BC1 fixed-rate baseline on the GPU (jpt_bc1_resolve) against the
oracle: BC1 levels decoded by definition, then the oracle's resolve;
frames bit-exact for every filter, with and without mip mapping."""
import numpy as np
import pytest

import oracle
from paper_2510_08166_amd import synth
from paper_2510_08166_amd.synth import configs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("filt", [configs.FILTER_NEAREST, configs.FILTER_BILINEAR, configs.FILTER_TRILINEAR,
                                  configs.FILTER_BILINEAR | oracle.NO_MIP])
def test_bc1_resolve_matches_oracle(gpu, filt):
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.quad_scene(51, 3, 200, 50, 90, 5, 320, 200, 24, keep_rgb=True, name="bc1")
    levels = [[(synth.bc1_encode(l), l.shape[1], l.shape[0]) for l in t.rgb_levels] for t in wl.textures]
    sc = jpt.Bc1Scene(levels)
    views = jpt.Views(wl.views)
    jpt.bc1_resolve(sc, views, filt)
    torch.cuda.synchronize()
    got = views.frame_host(0)
    osc = oracle.Scene(wl.textures)
    imgs = {}
    L = 0
    for t in levels:
        for blk, w, h in t:
            imgs[L] = oracle.bc1_decode(blk, w, h)
            L += 1
    ref, bad = osc.resolve(wl.views[0], filt, imgs)
    assert bad == 0
    assert np.array_equal(got, ref)
