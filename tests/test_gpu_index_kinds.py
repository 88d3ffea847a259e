"""The two readings of the paper's index on the GPU: a predictor index
(untouched entropy segment, DC predictors per MCU) decodes through the same
entropy kernel to coefficients bit-identical to the spliced index's, and to
the oracle's, with identical texels and frames."""
import numpy as np
import pytest

from paper_2510_08166_amd.synth import configs

from gpu_common import full_parity, run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["420 bilinear", "444 ragged trilinear"])
@pytest.mark.parametrize("mode", [0, 2])
def test_predictor_index_equals_spliced(gpu, case, mode):
    from paper_2510_08166_amd import jpt
    if case == "420 bilinear":
        wl = configs.reduced(seed=17, filt=configs.FILTER_BILINEAR)
    else:
        wl = configs.quad_scene(23, 3, 200, 40, 95, 4, 160, 120, 12, sampling=444, filt=configs.FILTER_TRILINEAR)
    alt = jpt.HostScene(wl.textures, index_kind=jpt.INDEX_PREDICTORS)
    r_alt, osc, blocks = full_parity(wl, idct_mode=mode, host=alt)
    assert r_alt.scene.c.flags & jpt.SCENE_PREDICTOR_INDEX
    _, ctr_a, items_a, coef_a, tiles_a, frames_a = run(wl, mode, host=alt)
    _, ctr_s, items_s, coef_s, tiles_s, frames_s = run(wl, mode)
    assert np.array_equal(items_a, items_s)
    if mode != jpt.IDCT_FUSED_F32:
        assert np.array_equal(coef_a, coef_s)
    assert np.array_equal(tiles_a, tiles_s)
    for a, b in zip(frames_a, frames_s):
        assert np.array_equal(a, b)
    bound, eff, stored = alt.overhead()
    sb, se, ss = jpt.HostScene(wl.textures).overhead()
    print("%s: overhead bound %.4f bpp; predictor index effective %.4f, spliced %.4f" % (case, bound, eff, se))
    assert abs(eff - bound) < 1e-9 and se < eff


def test_predictor_level_without_scene_flag_fails_loudly(gpu):
    """A predictor-index level in a scene launched without
    JPT_SCENE_PREDICTOR_INDEX is flagged corrupt, never decoded wrongly."""
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.reduced(seed=18)
    alt = jpt.HostScene(wl.textures, index_kind=jpt.INDEX_PREDICTORS)
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, host=alt)
    r.scene.c.flags = 0
    r.render()
    torch.cuda.synchronize()
    assert r.frame.counters_host()[jpt.CTR_ERROR] & jpt.ERR_CORRUPT
