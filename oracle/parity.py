"""Comparison of GPU results with the oracle (test infrastructure).

All inputs are plain numpy arrays read back from the device; nothing here
calls the GPU library.  The bar:
  - visible blocks, work items, coefficients: bit-exact;
  - texels: within 1 LSB per RGB channel of the fp64 oracle, and every
    mismatch within max(1e-3, an a-priori fp32 error bound) of a rounding
    tie of the fp64 value (texel_tolerance);
  - frames: bit-exact against the oracle's resolve applied to the GPU's own
    texels, within 1 LSB against the oracle's full render.
"""
from __future__ import annotations

import numpy as np

from . import ZIGZAG, Scene, unpack_frame


def expected_items(osc: Scene, blocks: np.ndarray) -> np.ndarray:
    out = []
    for b in blocks:
        L = osc.level_of_block(int(b))
        n = 4 if osc.jpegs[L].sampling == 444 else 1
        out.extend((int(b) << 2) | q for q in range(n))
    return np.array(out, np.uint32)


def visible_blocks(osc: Scene, gbufs, filt) -> np.ndarray:
    s = set()
    for g in gbufs:
        v, _ = osc.mark(g, filt)
        s.update(int(x) for x in v)
    return np.array(sorted(s), np.uint32)


class LevelCache:
    """Sequentially decoded coefficients of each level, decoded once."""

    def __init__(self, osc: Scene):
        self.osc = osc
        self._coef = {}

    def coef(self, L):
        if L not in self._coef:
            self._coef[L] = self.osc.jpegs[L].decode()[0]
        return self._coef[L]

    def item_mcu(self, item: int):
        b, q = item >> 2, item & 3
        L, bx, by = self.osc.block_coords(b)
        j = self.osc.jpegs[L]
        if j.sampling == 420:
            return L, by * j.mcu_cols + bx
        mx, my = 2 * bx + (q & 1), 2 * by + (q >> 1)
        if mx >= j.mcu_cols or my >= j.mcu_rows:
            return L, None
        return L, my * j.mcu_cols + mx

    def block_tile(self, b: int, want_f64=False):
        """16x16 tile of a block (rgb uint8, optional f64) from per-MCU oracle pixels."""
        L, bx, by = self.osc.block_coords(b)
        j = self.osc.jpegs[L]
        rgb = np.zeros((16, 16, 3), np.uint8)
        f = np.zeros((16, 16, 3)) if want_f64 else None
        coef = self.coef(L)
        if j.sampling == 420:
            r = j.mcu_pixels(coef[by * j.mcu_cols + bx], want_f64)
            if want_f64:
                rgb[:], f[:] = r
            else:
                rgb[:] = r
        else:
            for q in range(4):
                mx, my = 2 * bx + (q & 1), 2 * by + (q >> 1)
                if mx >= j.mcu_cols or my >= j.mcu_rows:
                    continue
                r = j.mcu_pixels(coef[my * j.mcu_cols + mx], want_f64)
                ys, xs = slice(8 * (q >> 1), 8 * (q >> 1) + 8), slice(8 * (q & 1), 8 * (q & 1) + 8)
                if want_f64:
                    rgb[ys, xs], f[ys, xs] = r
                else:
                    rgb[ys, xs] = r
        return (rgb, f) if want_f64 else rgb


def check_coefs(lc: LevelCache, items: np.ndarray, coef_zz: np.ndarray, sample=None):
    """coef_zz: [n_items, 6, 64] in zigzag order.  Returns indices of mismatching items."""
    bad = []
    idx = range(len(items)) if sample is None else sample
    for i in idx:
        it = int(items[i])
        L, m = lc.item_mcu(it & 0x7FFFFFFF)
        if m is None:
            if np.any(coef_zz[i]):
                bad.append(i)
            continue
        ref = lc.coef(L)[m]
        n_du = ref.shape[0]
        nat = np.zeros((n_du, 64), np.int16)
        nat[:, ZIGZAG] = coef_zz[i, :n_du]
        if not np.array_equal(nat, ref) or np.any(coef_zz[i, n_du:]):
            bad.append(i)
    return bad


# Colour-matrix magnitudes per output channel (R, G, B) applied to the
# errors of the Y, Cb and Cr samples (JFIF full-range inverse).
_MIX = np.array([[1.0, 0.0, 1.402], [1.0, 0.344136, 0.714136], [1.0, 1.772, 0.0]])
_U = 2.0 ** -24
TIE_FLOOR = 1e-3


def texel_tolerance(lc: LevelCache, b: int) -> np.ndarray:
    """[16, 16, 3] distance to a rounding tie within which either neighbour
    is a correct 8-bit texel: max(1e-3, an a-priori bound on the fp32 error
    of the GPU paths).  A sample is s = sum F_uv K_uv with |K_uv| <= 1/4;
    its fp32 evaluation errs by at most 72 u sum|F| / 4 (u = 2^-24: up to 64
    accumulation roundings, the fp16 hi/lo basis split worth 4 u |K|, the
    recombination and the basis rounding), and the colour matrix, its fp32
    constants and the +0.5 of the rounding add at most 4096 u.  sum|F| is
    taken over the data unit feeding each sample."""
    L, bx, by = lc.osc.block_coords(b)
    j = lc.osc.jpegs[L]
    coef = lc.coef(L)
    S = np.zeros((16, 16, 3))                     # sum |F| of the Y, Cb, Cr unit of each texel
    qt = j.quant.astype(np.float64)               # natural order, [luma, chroma]

    def du_sum(m, d, comp):
        return float(np.abs(coef[m, d].astype(np.float64) * qt[1 if comp else 0]).sum())

    if j.sampling == 420:
        m = by * j.mcu_cols + bx
        for ty in range(16):
            for tx in range(16):
                S[ty, tx] = (du_sum(m, (ty // 8) * 2 + tx // 8, 0), du_sum(m, 4, 1), du_sum(m, 5, 2))
    else:
        for q in range(4):
            mx, my = 2 * bx + (q & 1), 2 * by + (q >> 1)
            if mx >= j.mcu_cols or my >= j.mcu_rows:
                continue
            m = my * j.mcu_cols + mx
            S[8 * (q >> 1):8 * (q >> 1) + 8, 8 * (q & 1):8 * (q & 1) + 8] = (du_sum(m, 0, 0), du_sum(m, 1, 1),
                                                                              du_sum(m, 2, 2))
    bound = 72.0 * _U * (S @ _MIX.T) / 4.0 + 4096.0 * _U
    return np.maximum(TIE_FLOOR, bound)


def check_texels(lc: LevelCache, blocks: np.ndarray, tiles: np.ndarray, sample=None):
    """tiles: [n_blocks, 256] RGBA8 u32 in slot order (= block order).  Returns
    (max abs diff, n mismatching channels, worst ratio of a mismatch's
    distance to a rounding tie over its tolerance (texel_tolerance; <= 1
    passes, clamped values count as infinitely far), the worst such distance
    itself, n channels compared)."""
    maxd, nmis, ratio, dmax, n = 0, 0, 0.0, 0.0, 0
    idx = range(len(blocks)) if sample is None else sample
    for i in idx:
        b = int(blocks[i])
        L, bx, by = lc.osc.block_coords(b)
        j = lc.osc.jpegs[L]
        ref, f = lc.block_tile(b, want_f64=True)
        got = tiles[i].reshape(16, 16).view(np.uint8).reshape(16, 16, 4)[:, :, :3].astype(int)
        # texels outside the image belong to no pixel; compare the image part
        h = min(16, j.height - 16 * by); w = min(16, j.width - 16 * bx)
        d = np.abs(got[:h, :w] - ref[:h, :w].astype(int))
        n += d.size
        maxd = max(maxd, int(d.max()))
        mis = d > 0
        if mis.any():
            nmis += int(mis.sum())
            fv = f[:h, :w][mis]
            clamped = (fv > 255.49) | (fv < -0.49)
            dist = np.abs(np.abs(fv - np.floor(fv)) - 0.5)
            dist[clamped] = np.inf
            tol = texel_tolerance(lc, b)[:h, :w][mis]
            ratio = max(ratio, float((dist / tol).max()))
            dmax = max(dmax, float(dist.max()))
    return maxd, nmis, ratio, dmax, n


def levels_from_tiles(osc: Scene, blocks: np.ndarray, tiles: np.ndarray) -> dict:
    """Level images holding the GPU's decoded blocks (other texels zero)."""
    imgs = {}
    for i, b in enumerate(blocks):
        L, bx, by = osc.block_coords(int(b))
        j = osc.jpegs[L]
        if L not in imgs:
            imgs[L] = np.zeros((j.height, j.width, 3), np.uint8)
        t = tiles[i].reshape(16, 16).view(np.uint8).reshape(16, 16, 4)[:, :, :3]
        h = min(16, j.height - 16 * by); w = min(16, j.width - 16 * bx)
        imgs[L][16 * by:16 * by + h, 16 * bx:16 * bx + w] = t[:h, :w]
    return imgs


def frame_diff(a: np.ndarray, b: np.ndarray) -> int:
    return int(np.abs(unpack_frame(a).astype(int) - unpack_frame(b).astype(int)).max()) if a.size else 0
