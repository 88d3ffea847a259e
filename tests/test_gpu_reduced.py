"""Reduced-resolution decode on the GPU (jpt_decode_reduced) against the
oracle's definition (orc_mcu_reduced): every work item's tile within 1 LSB,
mismatches only within a rounding tie's tolerance (max(1e-3, an fp32 error
bound of the reduced sums)); coefficient decode shared with the plain path."""
import numpy as np
import pytest

import oracle
from oracle import parity
from paper_2510_08166_amd.synth import configs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("s", [1, 2, 3])
@pytest.mark.parametrize("sampling,kind", [(420, 0), (444, 0), (420, 1)])
def test_reduced_decode_matches_oracle(gpu, s, sampling, kind):
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.quad_scene(61 + s, 3, 192, 40, 95, 1, 160, 120, 10, sampling=sampling,
                            filt=configs.FILTER_NEAREST, name="reduced decode")
    host = jpt.HostScene(wl.textures, index_kind=kind)
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, host=host)
    r.mark()
    torch.cuda.synchronize()
    items = r.frame.work_items()
    side = 16 >> s
    out = torch.zeros(max(1, len(items)) * side * side, dtype=torch.int32, device="cuda")
    jpt.decode_reduced(r.scene, r.frame, s, out)
    torch.cuda.synchronize()
    assert r.frame.counters_host()[jpt.CTR_ERROR] == 0
    tiles = out.cpu().numpy().view(np.uint32).reshape(-1, side * side)
    osc = oracle.Scene(wl.textures)
    lc = parity.LevelCache(osc)
    maxd, nmis, worst = 0, 0, 0.0
    for i, it in enumerate(items):
        L, m = lc.item_mcu(int(it))
        if m is None:
            continue
        j = osc.jpegs[L]
        ref, f = oracle.mcu_reduced(j, lc.coef(L)[m], s, want_f64=True)
        t = ref.shape[0]
        got = tiles[i][: t * t].reshape(t, t).view(np.uint8).reshape(t, t, 4)[:, :, :3].astype(int)
        d = np.abs(got - ref.astype(int))
        maxd = max(maxd, int(d.max()))
        mis = d > 0
        if mis.any():
            nmis += int(mis.sum())
            fv = f[mis]
            assert not ((fv > 255.49) | (fv < -0.49)).any(), "a clamped texel differs"
            comp = [0, 0, 0, 0, 1, 1] if j.n_du == 6 else [0, 1, 1]
            F = np.abs(lc.coef(L)[m].astype(np.float64) * j.quant[comp])
            tol = max(1e-3, 72 * 2.0 ** -24 * F.sum() / 4 + 4096 * 2.0 ** -24)
            dist = np.abs(np.abs(fv - np.floor(fv)) - 0.5)
            worst = max(worst, float(dist.max() / tol))
    print("scale 1/%d %d %s: %d items, max diff %d, %d channels differ, worst %.2f of tolerance" % (
        1 << s, sampling, "predictors" if kind else "spliced", len(items), maxd, nmis, worst))
    assert maxd <= 1 and worst <= 1.0
