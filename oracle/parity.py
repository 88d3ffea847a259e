"""Comparison of GPU results with the oracle (test infrastructure).

All inputs are plain numpy arrays read back from the device; nothing here
calls the GPU library.  The bar:
  - visible blocks, work items, coefficients: bit-exact;
  - texels: within 1 LSB per RGB channel of the fp64 oracle, and every
    mismatch within 0.01 of a rounding tie of the fp64 value;
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


def check_texels(lc: LevelCache, blocks: np.ndarray, tiles: np.ndarray, sample=None):
    """tiles: [n_blocks, 256] RGBA8 u32 in slot order (= block order).  Returns
    (max abs diff, n mismatching channels, max distance of a mismatch to a
    rounding tie, n channels compared)."""
    maxd, nmis, tie, n = 0, 0, 0.0, 0
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
            dist[clamped] = 1.0
            tie = max(tie, float(dist.max()))
    return maxd, nmis, tie, n


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
