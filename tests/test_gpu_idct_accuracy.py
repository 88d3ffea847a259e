"""IEEE-1180-style accuracy of the GPU inverse DCTs against the oracle's
fp64 IDCT (by definition).

Random 8x8 sample blocks uniform in [-L, L] are forward-transformed in fp64
and rounded to integer coefficients (the procedure of IEEE 1180-1990); the
coefficients are written straight into a frame's coefficient buffer (a
quality-100 texture, so every quantiser is 1, with zero chroma so that R = G
= B = the luma sample) and run through jpt_idct_color.  The red channel of
each texel is then round(clamp(IDCT + 128, 0, 255)), compared with the same
expression over the oracle's fp64 IDCT.  The ranges stay within what the
8-bit output can hold (L = 5 and L = 100).  Bounds are the standard's:
peak error <= 1, mean square error per position <= 0.06 and overall
<= 0.02, mean error per position <= 0.015 and overall <= 0.0015.
"""
import numpy as np
import pytest

import oracle
from paper_2510_08166_amd import synth

pytestmark = pytest.mark.gpu

# JPT_IDCT_* of the 8-bit paths
MODES = {"mfma_f16": 0, "scalar_f32": 1, "mfma_bf16": 3}


def fdct_matrix():
    x = np.arange(8)[:, None]
    u = np.arange(8)[None, :]
    C = np.where(u == 0, 1 / np.sqrt(2), 1.0)
    return C / 2 * np.cos((2 * x + 1) * u * np.pi / 16)   # B[x][u]; s = B F B^T, F = B^T s B


def setup(seed, side=816):
    """A quality-100 texture (every quantiser 1) sampled at texel centres:
    the frame's work items are all of its 51 x 51 = 2,601 MCUs (10,404 luma
    data units)."""
    import torch
    from paper_2510_08166_amd import jpt
    rgb = synth.texture(seed, side, side)
    tex = synth.EncodedTexture(0, side, side, 100, 420, [synth.encode(rgb, 100, 420)])
    y, x = np.mgrid[0:side, 0:side]
    g = np.zeros((side, side), synth.GPIXEL_DTYPE)
    g["u"] = ((x + 0.5) / side).astype(np.float32)
    g["v"] = ((y + 0.5) / side).astype(np.float32)
    g["tex"] = 0
    r = jpt.Renderer([tex], [g], jpt.FILTER_NEAREST)
    assert (r.host.quants[0] == 1).all()
    r.mark()
    torch.cuda.synchronize()
    return r


def ieee_blocks(n, lo, hi, sign, seed):
    """IEEE 1180-1990 input: sample blocks uniform in [-lo, hi] (times sign),
    their fp64 forward DCT rounded to integers and clipped to 12 bits."""
    rng = np.random.default_rng(seed)
    B = fdct_matrix()
    samples = sign * rng.integers(-lo, hi + 1, (n, 4, 8, 8)).astype(np.float64)   # S[y][x]
    F = np.matmul(np.matmul(B.T, samples), B)                  # F[v][u] = sum B[y][v] S[y][x] B[x][u]
    return np.clip(np.round(F), -2048, 2047).astype(np.int16)


def stats(got, ref):
    e = (got - ref).reshape(-1, 64).astype(np.float64)
    return dict(peak=int(np.abs(e).max()), pmse=float((e ** 2).mean(0).max()), omse=float((e ** 2).mean()),
                pme=float(np.abs(e.mean(0)).max()), ome=float(abs(e.mean())), blocks=e.shape[0])


def within_bounds(st):
    return (st["peak"] <= 1 and st["pmse"] <= 0.06 and st["omse"] <= 0.02 and st["pme"] <= 0.015
            and st["ome"] <= 0.0015)


def run_case(L, mode, seed):
    import torch
    from paper_2510_08166_amd import jpt
    side = 512
    rgb = synth.texture(seed, side, side)
    tex = synth.EncodedTexture(0, side, side, 100, 420, [synth.encode(rgb, 100, 420)])
    y, x = np.mgrid[0:side, 0:side]
    g = np.zeros((side, side), synth.GPIXEL_DTYPE)
    g["u"] = ((x + 0.5) / side).astype(np.float32)
    g["v"] = ((y + 0.5) / side).astype(np.float32)
    g["tex"] = 0
    r = jpt.Renderer([tex], [g], jpt.FILTER_NEAREST)
    assert (r.host.quants[0] == 1).all()
    r.mark()
    torch.cuda.synchronize()
    items = r.frame.work_items()
    n = len(items)
    rng = np.random.default_rng(seed)
    B = fdct_matrix()
    samples = rng.integers(-L, L + 1, (n, 4, 8, 8)).astype(np.float64)   # S[y][x]
    F = np.matmul(np.matmul(B.T, samples), B)                  # F[v][u] = sum B[y][v] S[y][x] B[x][u]
    F = np.clip(np.round(F), -2048, 2047).astype(np.int16)
    coef = np.zeros((n, 6, 64), np.int16)
    coef[:, :4] = F.reshape(n, 4, 64)[:, :, oracle.ZIGZAG]      # natural -> zigzag order
    r.frame.coef[: n * 384].copy_(torch.from_numpy(coef.reshape(-1)))
    jpt.idct_color(r.scene, r.frame, r.cache, mode)
    torch.cuda.synchronize()
    tiles = r.cache.texels[: n * 256].cpu().numpy().view(np.uint8).reshape(n, 16, 16, 4)
    got = np.zeros((n, 4, 8, 8), np.int64)
    for k in range(4):
        got[:, k] = tiles[:, 8 * (k >> 1):8 * (k >> 1) + 8, 8 * (k & 1):8 * (k & 1) + 8, 0]
    ref = np.zeros_like(got)
    Fn = F.astype(np.float64)
    for i in range(n):
        for k in range(4):
            s = oracle.idct(Fn[i, k].reshape(64))
            ref[i, k] = np.floor(np.clip(s + 128.0, 0.0, 255.0) + 0.5)
    e = (got - ref).reshape(-1, 64).astype(np.float64)
    return dict(peak=int(np.abs(e).max()), pmse=float((e ** 2).mean(0).max()), omse=float((e ** 2).mean()),
                pme=float(np.abs(e.mean(0)).max()), ome=float(abs(e.mean())), blocks=e.shape[0])


@pytest.mark.parametrize("lo,hi", [(256, 255), (5, 5), (300, 300)])
@pytest.mark.parametrize("sign", [1, -1])
def test_ieee1180_float_path_full_ranges(gpu, lo, hi, sign):
    """The standard's three ranges, and their negations, on the fp32
    separable IDCT before any clamp: the float texels of jpt_fwd_float with
    zero chroma are R = G = B = IDCT + 128, so IDCT = R - 128, rounded and
    clipped to [-256, 255] as the standard's output."""
    import torch
    from paper_2510_08166_amd import jpt
    r = setup(seed=60 + lo)
    items = r.frame.work_items()
    n = len(items)
    F = ieee_blocks(n, lo, hi, sign, seed=lo * 3 + (sign > 0))
    diff = jpt.DiffFrame(r)
    Fd = torch.zeros((n, 6, 64), dtype=torch.float32, device="cuda")
    Fd[:, :4] = torch.from_numpy(F.reshape(n, 4, 64).astype(np.float32)).cuda()
    diff._scratch()
    diff.forward(Fd)
    torch.cuda.synchronize()
    tf = diff.texel_f[: n * 768].cpu().numpy().reshape(n, 16, 16, 3)
    got = np.zeros((n, 4, 8, 8), np.int64)
    for k in range(4):
        blk = tf[:, 8 * (k >> 1):8 * (k >> 1) + 8, 8 * (k & 1):8 * (k & 1) + 8, 0] - 128.0
        got[:, k] = np.clip(np.floor(blk + 0.5), -256, 255)
    ref = np.zeros_like(got)
    Fn = F.astype(np.float64)
    for i in range(n):
        for k in range(4):
            ref[i, k] = np.clip(np.floor(oracle.idct(Fn[i, k].reshape(64)) + 0.5), -256, 255).reshape(8, 8)
    st = stats(got, ref)
    print("IDCT fp32 separable [-%d, %d] sign %+d: %s" % (lo, hi, sign, st), flush=True)
    assert st["blocks"] >= 10000 and within_bounds(st)


@pytest.mark.parametrize("mode_name", ["mfma_f16", "mfma_bf16", "scalar_f32", "float"])
def test_ieee1180_zero_in_zero_out(gpu, mode_name):
    """All-zero coefficients give exactly zero samples (texels of 128 on the
    8-bit paths, float texels of exactly 128.0)."""
    import torch
    from paper_2510_08166_amd import jpt
    r = setup(seed=70, side=256)
    n = len(r.frame.work_items())
    if mode_name == "float":
        diff = jpt.DiffFrame(r)
        diff._scratch()
        diff.forward(torch.zeros((n, 6, 64), dtype=torch.float32, device="cuda"))
        torch.cuda.synchronize()
        assert (diff.texel_f[: n * 768].cpu().numpy() == 128.0).all()
        return
    r.frame.coef[: n * 384].zero_()
    jpt.idct_color(r.scene, r.frame, r.cache, MODES[mode_name])
    torch.cuda.synchronize()
    t = r.cache.texels[: n * 256].cpu().numpy().view(np.uint8).reshape(-1, 4)
    assert (t[:, :3] == 128).all()


@pytest.mark.parametrize("L", [5, 100])
@pytest.mark.parametrize("mode_name", ["mfma_f16", "mfma_bf16", "scalar_f32"])
def test_ieee1180_style(gpu, L, mode_name):
    mode = MODES[mode_name]
    st = run_case(L, mode, seed=40 + L)
    print("IDCT %s L=%d: %s" % (mode_name, L, st), flush=True)
    assert st["peak"] <= 1 and st["pmse"] <= 0.06 and st["omse"] <= 0.02
    assert st["pme"] <= 0.015 and st["ome"] <= 0.0015
