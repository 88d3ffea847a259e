"""Float64 reference of the differentiable form (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the GPU library.

The frame as a function of the dequantised DCT coefficients F of a set of
work items, with the rounding and clamping of the 8-bit path dropped and the
integer filter weights of the resolve held constant (paper: Decode, whose
stages are dequantisation, the 8x8 inverse DCT and the colour transform;
Resolve, the filtered lookup of the decoded texels):

    s      = IDCT(F)                                 (T.81 A.3.3, by definition)
    ycc    = s + (128, 0, 0); chroma replicated over 2x2 texels for 4:2:0
    texel  = M ycc,  M the JFIF full-range inverse    (R = Y + 1.402 Cr,
             G = Y - 0.344136 Cb - 0.714136 Cr, B = Y + 1.772 Cb)
    frame  = sum over the taps of (tap weight / 65536) (level weight / 256) texel

A work item is (block << 2) | quadrant: one item per 16x16 block of a 4:2:0
level (its MCU), four per block of a 4:4:4 level (one 8x8 MCU per quadrant).
F is [n_items, 6, 64] in natural order (index v*8+u, v the vertical
frequency); a 4:4:4 item uses units 0..2 (Y, Cb, Cr).  Gradients come from
torch autograd in float64 on the CPU.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Scene
from .parity import LevelCache

M = ((1.0, 0.0, 1.402), (1.0, -0.344136, -0.714136), (1.0, 1.772, 0.0))


def basis() -> torch.Tensor:
    """B[x][u] = C(u)/2 cos((2x+1) u pi / 16), C(0) = 1/sqrt(2), else 1, so that
    s = B F B^T is the 2-D inverse DCT of T.81 A.3.3."""
    x = np.arange(8)[:, None]
    u = np.arange(8)[None, :]
    C = np.where(u == 0, 1.0 / np.sqrt(2.0), 1.0)
    return torch.tensor(C / 2.0 * np.cos((2 * x + 1) * u * np.pi / 16.0), dtype=torch.float64)


def item_sampling(osc: Scene, items: np.ndarray) -> np.ndarray:
    return np.array([osc.jpegs[osc.level_of_block(int(it) >> 2)].sampling for it in items], np.int64)


def dequantized(osc: Scene, items: np.ndarray, lc: LevelCache | None = None) -> np.ndarray:
    """F of each item from the oracle's sequential decode: coefficient x
    quantiser (paper: Decode, dequantisation).  Items whose 4:4:4 MCU lies
    beyond the image get zeros."""
    lc = lc or LevelCache(osc)
    F = np.zeros((len(items), 6, 64), np.float64)
    for i, it in enumerate(items):
        L, m = lc.item_mcu(int(it))
        if m is None:
            continue
        j = osc.jpegs[L]
        coef = lc.coef(L)[m].astype(np.float64)
        comps = (0, 0, 0, 0, 1, 1) if j.sampling == 420 else (0, 1, 1)
        for d, c in enumerate(comps):
            F[i, d] = coef[d] * j.quant[c]
    return F


def item_texels(F: torch.Tensor, sampling: np.ndarray):
    """Texels of every item, unrounded: (tiles420 [n, 16, 16, 3], tiles444
    [n, 8, 8, 3], ycc of both before the colour transform).  F [n_items, 6, 64]."""
    B = basis()
    s = B @ F.reshape(-1, 6, 8, 8) @ B.T                       # [n, 6, y, x]
    i420 = torch.from_numpy(np.nonzero(sampling == 420)[0])
    i444 = torch.from_numpy(np.nonzero(sampling == 444)[0])
    Mt = torch.tensor(M, dtype=torch.float64)
    out = []
    for idx, kind in ((i420, 420), (i444, 444)):
        S = s.index_select(0, idx)
        if kind == 420:
            top = torch.cat([S[:, 0], S[:, 1]], dim=2)           # [n, 8, 16]
            bot = torch.cat([S[:, 2], S[:, 3]], dim=2)
            Y = torch.cat([top, bot], dim=1) + 128.0              # [n, 16, 16]
            Cb = S[:, 4].repeat_interleave(2, 1).repeat_interleave(2, 2)
            Cr = S[:, 5].repeat_interleave(2, 1).repeat_interleave(2, 2)
        else:
            Y, Cb, Cr = S[:, 0] + 128.0, S[:, 1], S[:, 2]
        ycc = torch.stack([Y, Cb, Cr], dim=-1)
        out.append((ycc @ Mt.T, ycc))
    return out[0][0], out[1][0], (out[0][1], out[1][1])


def tap_rows(osc: Scene, items: np.ndarray, sampling: np.ndarray, g: np.ndarray, filt: int):
    """Per pixel and tap: the row of the flat texel table (420 tiles first,
    then 444 quadrant tiles, one row per texel) and the weight.  Raises if a
    tap with non-zero weight reads a block that is not a work item."""
    lv, x, y, w, bad = osc.taps(g, filt)
    if bad:
        raise ValueError("%d invalid pixels" % bad)
    order = np.argsort(items, kind="stable")
    sorted_items = items[order].astype(np.int64)
    n420 = int((sampling == 420).sum())
    rank = np.zeros(len(items), np.int64)          # position of each item inside its kind
    rank[sampling == 420] = np.arange(n420)
    rank[sampling == 444] = np.arange(len(items) - n420)
    used = w != 0
    L = np.where(used, lv, 0)
    xx, yy = x.astype(np.int64), y.astype(np.int64)
    base = osc.blk_base.astype(np.int64)[L]
    cols = osc.blk_cols.astype(np.int64)[L]
    blk = base + (yy >> 4) * cols + (xx >> 4)
    s444 = np.array([osc.jpegs[i].sampling == 444 for i in range(len(osc.jpegs))])[L]
    q = np.where(s444, ((yy >> 3) & 1) * 2 + ((xx >> 3) & 1), 0)
    code = (blk << 2) | q
    pos = np.searchsorted(sorted_items, code)
    pos = np.minimum(pos, len(sorted_items) - 1)
    found = sorted_items[pos] == code
    if np.any(used & ~found):
        raise ValueError("a tap reads a block that is not a work item")
    it = order[pos]
    row = np.where(s444, n420 * 256 + rank[it] * 64 + (yy & 7) * 8 + (xx & 7),
                   rank[it] * 256 + (yy & 15) * 16 + (xx & 15))
    return np.where(used, row, 0), np.where(used, w, 0.0)


def forward(osc: Scene, items: np.ndarray, F: torch.Tensor, g: np.ndarray, filt: int) -> torch.Tensor:
    """frame [H, W, 3] float64 as a differentiable function of F."""
    samp = item_sampling(osc, items)
    t420, t444, _ = item_texels(F, samp)
    flat = torch.cat([t420.reshape(-1, 3), t444.reshape(-1, 3)], dim=0)
    row, w = tap_rows(osc, items, samp, g, filt)
    if flat.shape[0] == 0:
        return torch.zeros(g.shape + (3,), dtype=torch.float64)
    gathered = flat.index_select(0, torch.from_numpy(row.reshape(-1))).reshape(row.shape + (3,))
    return (gathered * torch.from_numpy(w)[..., None]).sum(dim=-2)


def vjp(osc: Scene, items: np.ndarray, F: np.ndarray, g: np.ndarray, filt: int, dframe: np.ndarray):
    """(frame, dF = J^T dframe) in float64."""
    Ft = torch.tensor(F, dtype=torch.float64, requires_grad=True)
    frame = forward(osc, items, Ft, g, filt)
    frame.backward(torch.as_tensor(np.asarray(dframe, np.float64)))
    return frame.detach().numpy(), Ft.grad.numpy()


def l2_loss_grad(osc: Scene, items: np.ndarray, F: np.ndarray, g: np.ndarray, filt: int, target: np.ndarray):
    """(L, dL/dF) for L = sum (frame - target)^2."""
    Ft = torch.tensor(F, dtype=torch.float64, requires_grad=True)
    frame = forward(osc, items, Ft, g, filt)
    L = ((frame - torch.as_tensor(np.asarray(target, np.float64))) ** 2).sum()
    L.backward()
    return float(L.detach()), Ft.grad.numpy()


def l2_loss(osc: Scene, items: np.ndarray, F: np.ndarray, g: np.ndarray, filt: int, target: np.ndarray) -> float:
    with torch.no_grad():
        frame = forward(osc, items, torch.as_tensor(np.asarray(F, np.float64)), g, filt)
        return float(((frame - torch.as_tensor(np.asarray(target, np.float64))) ** 2).sum())


def level_images(osc: Scene, items: np.ndarray, F: np.ndarray) -> dict:
    """Unrounded texels of the items pasted into their levels (NaN where no
    item covers a texel): {level: [h, w, 3] float64}."""
    samp = item_sampling(osc, items)
    with torch.no_grad():
        t420, t444, _ = item_texels(torch.as_tensor(F, dtype=torch.float64), samp)
    t420, t444 = t420.numpy(), t444.numpy()
    out = {}
    k420 = k444 = 0
    for it, s in zip(items, samp):
        b, q = int(it) >> 2, int(it) & 3
        L, bx, by = osc.block_coords(b)
        img = out.setdefault(L, np.full((int(osc.lev_h[L]), int(osc.lev_w[L]), 3), np.nan))
        if s == 420:
            tile, y0, x0 = t420[k420], 16 * by, 16 * bx
            k420 += 1
        else:
            tile, y0, x0 = t444[k444], 16 * by + 8 * (q >> 1), 16 * bx + 8 * (q & 1)
            k444 += 1
        h = max(0, min(tile.shape[0], img.shape[0] - y0))
        w = max(0, min(tile.shape[1], img.shape[1] - x0))
        img[y0:y0 + h, x0:x0 + w] = tile[:h, :w]
    return out
