"""Pins of the float64 differentiable-form reference (oracle.grad).

  - texels: equal to the sequential oracle's unrounded MCU pixels (C code,
    IDCT by definition) wherever that path does not clamp;
  - frame: equal to the oracle's resolve (C code) applied to the same
    unrounded texels, so taps, weights and levels agree;
  - gradient: the closed form of one nearest-filtered pixel (a product of two
    1-D DCT basis functions times the colour matrix entry, chroma at the
    half-resolution sample), central differences of the L2 loss (exact for a
    quadratic up to rounding), and the adjoint identity <J d, y> = <d, J^T y>.
A transposed basis, a wrong chroma index, a wrong colour coefficient, a
wrong tap weight or a dropped 2x2 chroma sum fails at least one of them.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import grad, parity
from paper_2510_08166_amd.synth import GPIXEL_DTYPE, configs, make_textures, target_frame
from paper_2510_08166_amd.synth.configs import quad_scene


def scene_items(wl):
    osc = oracle.Scene(wl.textures)
    blocks = parity.visible_blocks(osc, wl.views, wl.filter)
    items = parity.expected_items(osc, blocks)
    return osc, items


@pytest.fixture(scope="module")
def mixed():
    """4:2:0 and 4:4:4 textures with odd sizes (ragged MCUs), bilinear."""
    tex = make_textures([(31, 72, 56, 70, 420, 3), (32, 60, 44, 85, 444, 3)])
    rng = np.random.default_rng(5)
    H, W = 40, 52
    g = np.zeros((H, W), GPIXEL_DTYPE)
    g["u"] = rng.uniform(-1, 2, (H, W)).astype(np.float32)
    g["v"] = rng.uniform(-1, 2, (H, W)).astype(np.float32)
    g["tex"] = rng.integers(0, 2, (H, W))
    g["lod"] = rng.uniform(-0.5, 2.5, (H, W)).astype(np.float32)
    g["tex"][:3, :] = oracle.BACKGROUND
    return g, tex


@pytest.mark.parametrize("filt", [oracle.NEAREST, oracle.BILINEAR, oracle.TRILINEAR])
def test_texels_and_frame_match_oracle(mixed, filt):
    g, tex = mixed
    osc = oracle.Scene(tex)
    blocks = parity.visible_blocks(osc, [g], filt)
    items = parity.expected_items(osc, blocks)
    lc = parity.LevelCache(osc)
    F = grad.dequantized(osc, items, lc)
    samp = grad.item_sampling(osc, items)
    assert set(samp) == {420, 444}
    t420, t444, (y420, y444) = grad.item_texels(torch.as_tensor(F), samp)
    k = {420: 0, 444: 0}
    n_cmp = n_all = 0
    for it, s in zip(items, samp):
        b, q = int(it) >> 2, int(it) & 3
        L, m = lc.item_mcu(int(it))
        if m is None:
            k[s] += 1
            continue
        _, ref = osc.jpegs[L].mcu_pixels(lc.coef(L)[m], want_f64=True)
        tile = (t420 if s == 420 else t444)[k[s]].numpy()
        ycc = (y420 if s == 420 else y444)[k[s]].numpy()
        k[s] += 1
        ycc8 = ycc + np.array([0.0, 128.0, 128.0])             # chroma as the 8-bit path stores it
        ok = np.all((ycc8 >= 0) & (ycc8 <= 255), axis=-1)     # texels the 8-bit path does not clamp
        assert np.abs(tile[ok] - ref[ok]).max(initial=0) < 1e-9
        n_cmp += ok.sum(); n_all += ok.size
    assert n_cmp > 0.9 * n_all
    # frame: the oracle's C resolve over the same unrounded texels
    imgs = grad.level_images(osc, items, F)
    zeros = {L: np.zeros(im.shape, np.uint8) for L, im in imgs.items()}
    _, ff, bad = osc.resolve(g, filt, zeros, imgs, want_f64=True)
    assert bad == 0
    fr = grad.forward(osc, items, torch.as_tensor(F), g, filt).numpy()
    assert not np.isnan(ff).any()
    assert np.abs(fr - ff).max() < 1e-9


def test_single_pixel_gradient_closed_form():
    """One nearest-filtered pixel on texel (tx, ty) of a 4:2:0 MCU: dR/dF_Y(v,u)
    = B[ty%8][v] B[tx%8][u] in the texel's luma unit, dR/dF_Cr = 1.402 times
    the basis at the chroma sample (ty/2, tx/2), dR/dF_Cb = 0; likewise for G
    and B with their matrix entries."""
    tex = make_textures([(41, 32, 32, 75, 420, 1)])
    osc = oracle.Scene(tex)
    B = np.array([[(np.sqrt(0.5) if u == 0 else 1.0) / 2 * np.cos((2 * x + 1) * u * np.pi / 16)
                   for u in range(8)] for x in range(8)])
    for (tx, ty) in [(3, 5), (12, 9), (0, 15), (15, 0)]:
        g = np.zeros((1, 1), GPIXEL_DTYPE)
        g["u"], g["v"], g["tex"], g["lod"] = (tx + 0.5) / 32, (ty + 0.5) / 32, 0, 0.0
        items = np.array([0 << 2], np.uint32)  # block (0, 0)
        F = grad.dequantized(osc, items)
        coef = {"R": (1.0, 0.0, 1.402), "G": (1.0, -0.344136, -0.714136), "B": (1.0, 1.772, 0.0)}
        for ch, (cy, cb, cr) in enumerate(coef.values()):
            d = np.zeros((1, 1, 3)); d[0, 0, ch] = 1.0
            _, dF = grad.vjp(osc, items, F, g, oracle.NEAREST, d)
            exp = np.zeros((6, 8, 8))
            exp[(ty // 8) * 2 + tx // 8] = np.outer(B[ty % 8], B[tx % 8])
            exp[4] = cb * np.outer(B[ty // 2], B[tx // 2])
            exp[5] = cr * np.outer(B[ty // 2], B[tx // 2])
            assert np.abs(dF[0].reshape(6, 8, 8) - exp).max() < 1e-12


def test_central_differences_and_adjoint():
    wl = configs.reduced(seed=11, n_tex=3, side=128, W=96, H=64, n_quads=10, n_levels=4)
    osc, items = scene_items(wl)
    g = wl.views[0]
    F = grad.dequantized(osc, items)
    target = target_frame(3, *g.shape).astype(np.float64)
    L0, dF = grad.l2_loss_grad(osc, items, F, g, wl.filter, target)
    rng = np.random.default_rng(0)
    nz = np.argwhere(np.abs(dF) > 0)
    pick = nz[rng.choice(len(nz), 64, replace=False)]
    for i, d, k in pick:
        Fp = F.copy(); Fp[i, d, k] += 1.0
        Fm = F.copy(); Fm[i, d, k] -= 1.0
        fd = (grad.l2_loss(osc, items, Fp, g, wl.filter, target) -
              grad.l2_loss(osc, items, Fm, g, wl.filter, target)) / 2.0
        assert abs(fd - dF[i, d, k]) <= 1e-6 * max(1.0, abs(dF[i, d, k])) + 1e-9 * abs(L0)
    # adjoint identity
    y = rng.standard_normal(g.shape + (3,))
    delta = rng.standard_normal(F.shape)
    samp = grad.item_sampling(osc, items)
    delta[samp == 444, 3:] = 0.0
    f0, Jty = grad.vjp(osc, items, F, g, wl.filter, y)
    with torch.no_grad():
        f1 = grad.forward(osc, items, torch.as_tensor(F + delta), g, wl.filter).numpy()
    lhs = float(((f1 - f0) * y).sum())
    rhs = float((delta * Jty).sum())
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs))


def test_quad_scene_444_gradient_sums_chroma_once():
    """4:4:4 chroma has no 2x2 sum: the colour-matrix part of the gradient of
    a nearest pixel lands on the texel's own sample."""
    wl = quad_scene(9, 2, 64, 70, 80, 2, 48, 32, 4, sampling=444, filt=oracle.NEAREST)
    osc, items = scene_items(wl)
    g = wl.views[0]
    F = grad.dequantized(osc, items)
    rng = np.random.default_rng(1)
    y = rng.standard_normal(g.shape + (3,))
    _, dF = grad.vjp(osc, items, F, g, wl.filter, y)
    assert np.all(dF[:, 3:] == 0.0)
    # the luma gradient and the Cb / Cr gradients follow the colour matrix:
    # dL/dY = sum of channel adjoints, dL/dCb = -0.344136 gG + 1.772 gB
    Binv = grad.basis()
    for i in range(min(len(items), 20)):
        dS = (Binv @ torch.as_tensor(dF[i, :3].reshape(3, 8, 8)) @ Binv.T).numpy()   # back to sample space
        # every sample gradient is a linear image of the channel adjoints; Y and
        # Cb/Cr gradients must be zero exactly where no pixel reads the texel
        zero_y = np.abs(dS[0]) < 1e-12
        assert np.all(np.abs(dS[1][zero_y]) < 1e-9) and np.all(np.abs(dS[2][zero_y]) < 1e-9)
