"""Pins of the oracle's JPEG decoding against things other than itself:
PIL/libjpeg (run, never inspected), scipy's orthonormal DCT, closed forms,
the paper's worked MCU/DU counts, and brute force on tiny images."""
import io

import numpy as np
import pytest
import scipy.fft
from PIL import Image

import oracle
from paper_2510_08166_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def pil_encode(rgb, q, sub):
    b = io.BytesIO()
    Image.fromarray(rgb).save(b, format="JPEG", quality=q, subsampling=sub, optimize=False)
    return b.getvalue()


def pil_decode(data, mode="RGB"):
    im = Image.open(io.BytesIO(data))
    if mode == "YCbCr":
        im.draft("YCbCr", im.size)
        return np.asarray(im)
    return np.asarray(im.convert("RGB"))


# ------------------------------------------------------------------ IDCT
def test_idct_equals_orthonormal_dct3():
    """The JPEG IDCT (1/4 C(u)C(v) normalisation) is scipy's orthonormal 2-D DCT-III."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        F = rng.integers(-1024, 1024, (8, 8)).astype(np.float64) * (rng.random((8, 8)) < 0.5)
        ref = scipy.fft.idctn(F, type=2, norm="ortho")     # F[v][u] -> s[y][x]
        assert np.abs(oracle.idct(F) - ref).max() < 1e-9


def test_idct_dc_only_is_flat():
    for dc in (-1024.0, -1.0, 8.0, 1016.0):
        F = np.zeros((8, 8)); F[0, 0] = dc
        assert np.allclose(oracle.idct(F), dc / 8.0, atol=1e-12)


def test_idct_single_coefficient_is_separable_basis():
    """A single coefficient gives an outer product of two 1-D basis vectors
    (rank one), and the (v,u) coefficient oscillates u times along x."""
    for v in range(8):
        for u in range(8):
            F = np.zeros((8, 8)); F[v, u] = 100.0
            s = oracle.idct(F)
            sv = np.linalg.svd(s, compute_uv=False)
            assert sv[1] < 1e-9 * max(sv[0], 1)
            row = s[np.argmax(np.abs(s).sum(1))]
            sign_changes = int(np.sum(np.diff(np.sign(np.round(row, 9))) != 0))
            assert sign_changes == u


def test_idct_parseval_and_inverse():
    rng = np.random.default_rng(1)
    for _ in range(20):
        F = rng.normal(0, 200, (8, 8))
        s = oracle.idct(F)
        assert abs((s ** 2).sum() - (F ** 2).sum()) < 1e-6 * (F ** 2).sum()
        F2 = scipy.fft.dctn(s, type=2, norm="ortho")
        assert np.abs(F2 - F).max() < 1e-9


# ---------------------------------------------------------------- counts
def test_paper_mcu_and_du_counts_4096():
    """4096x4096 with 4:2:0 -> 65,536 MCUs and 393,216 data units (JPEG background section)."""
    data = bytearray(synth.encode(synth.texture(3, 16, 16), 75, 420))
    i = data.index(b"\xff\xc0")
    data[i + 5:i + 7] = (4096).to_bytes(2, "big"); data[i + 7:i + 9] = (4096).to_bytes(2, "big")
    j = oracle.Jpeg(bytes(data))
    assert (j.n_mcu, j.n_mcu * j.n_du) == (65536, 393216)


# --------------------------------------------------- against PIL/libjpeg
@pytest.mark.parametrize("q", [10, 50, 75, 95, 100])
def test_oracle_decodes_pil_444_like_pil(q):
    rgb = synth.texture(100 + q, 72, 56)
    data = pil_encode(rgb, q, 0)       # 4:4:4
    ours = oracle.Jpeg(data)
    coef, _, _, _ = ours.decode()
    px = ours.pixels(coef).astype(int)
    ref = pil_decode(data).astype(int)
    d = np.abs(px - ref)
    # libjpeg uses an integer IDCT and integer colour conversion
    assert d.max() <= 3 and d.mean() < 0.6


@pytest.mark.parametrize("q", [30, 75, 95])
def test_oracle_luma_420_like_pil(q):
    """4:2:0: luma does not depend on chroma upsampling, compare Y with PIL's YCbCr output."""
    rgb = synth.texture(200 + q, 80, 48)
    data = pil_encode(rgb, q, 2)       # 4:2:0
    ours = oracle.Jpeg(data)
    coef, _, _, _ = ours.decode()
    _, f = ours.pixels(coef, want_f64=True)
    y = 0.299 * f[..., 0] + 0.587 * f[..., 1] + 0.114 * f[..., 2]     # undo the colour matrix
    ref = pil_decode(data, "YCbCr")[..., 0].astype(float)
    assert np.abs(np.floor(y + 0.5) - ref).max() <= 2


def test_pil_decodes_synth_files():
    rgb = synth.texture(9, 96, 80)
    for smp in (420, 444):
        data = synth.encode(rgb, 80, smp)
        im = pil_decode(data)
        assert im.shape == rgb.shape


# --------------------------------------------- encoder / decoder pairing
@pytest.mark.parametrize("smp", [420, 444])
@pytest.mark.parametrize("q", [1, 25, 50, 75, 90, 100])
@pytest.mark.parametrize("size", [(8, 8), (16, 16), (40, 24), (33, 17), (97, 65)])
def test_decoder_returns_encoder_coefficients(smp, q, size):
    """Independent encoder (synth) and decoder (oracle): quantised
    coefficients must come back bit for bit, sequentially and by random access."""
    w, h = size
    rgb = synth.texture(w * 1000 + h + q, w, h)
    data, ref = synth.encode(rgb, q, smp, want_coef=True)
    j = oracle.Jpeg(data)
    coef, mb, pred, _ = j.decode()
    assert np.array_equal(coef, ref)
    for m in range(j.n_mcu):
        rc, out, end = j.decode_mcu_at(int(mb[m]), pred[m])
        assert rc == 0 and np.array_equal(out, coef[m]) and end == mb[m + 1]


def test_q100_420_pixels_match_encoder_input():
    """At quality 100 (all quantisers 1) the decode reproduces the encoder's
    YCbCr planes up to DCT rounding; chroma must sit replicated over each 2x2."""
    rgb = synth.texture(5, 64, 48)
    data = synth.encode(rgb, 100, 420)
    j = oracle.Jpeg(data)
    coef, _, _, _ = j.decode()
    _, f = j.pixels(coef, want_f64=True)
    r, g, b = [rgb[..., c].astype(float) for c in range(3)]
    Y = np.clip(np.floor(0.299 * r + 0.587 * g + 0.114 * b + 0.5), 0, 255)
    Cb = np.clip(np.floor(-0.168736 * r - 0.331264 * g + 0.5 * b + 128 + 0.5), 0, 255)
    Cr = np.clip(np.floor(0.5 * r - 0.418688 * g - 0.081312 * b + 128 + 0.5), 0, 255)
    box = lambda p: np.floor((p[0::2, 0::2] + p[1::2, 0::2] + p[0::2, 1::2] + p[1::2, 1::2] + 2) / 4)
    rep = lambda p: np.repeat(np.repeat(p, 2, 0), 2, 1)
    Cb2, Cr2 = rep(box(Cb)), rep(box(Cr))
    # decoded YCbCr from the oracle's (unclamped) RGB
    y = 0.299 * f[..., 0] + 0.587 * f[..., 1] + 0.114 * f[..., 2]
    cb = -0.168736 * f[..., 0] - 0.331264 * f[..., 1] + 0.5 * f[..., 2] + 128
    cr = 0.5 * f[..., 0] - 0.418688 * f[..., 1] - 0.081312 * f[..., 2] + 128
    assert np.abs(y - Y).max() < 1.5
    assert np.abs(cb - Cb2).max() < 1.5 and np.abs(cr - Cr2).max() < 1.5


def test_flat_images_every_value_brute_force():
    """One-MCU flat images at Q=1: every 8-bit grey level comes back exactly
    (DC = 8 (v - 128), every AC zero)."""
    for v in range(256):
        rgb = np.full((16, 16, 3), v, np.uint8)
        data, ref = synth.encode(rgb, 100, 420, want_coef=True)
        j = oracle.Jpeg(data)
        coef, _, _, _ = j.decode()
        assert coef[0, 0, 0] == 8 * (v - 128) and not coef[0, :, 1:].any()
        assert np.array_equal(j.pixels(coef), rgb)


# ------------------------------------------------------------ robustness
def test_truncated_and_garbage_are_rejected():
    data = synth.encode(synth.texture(1, 64, 64), 75, 420)
    with pytest.raises(oracle.OracleError):
        oracle.Jpeg(b"not a jpeg at all")
    j = oracle.Jpeg(data[: len(data) // 2])        # scan cut in half
    with pytest.raises(oracle.OracleError):
        j.decode()


def test_progressive_is_unsupported():
    b = io.BytesIO()
    Image.fromarray(synth.texture(2, 32, 32)).save(b, format="JPEG", quality=75, progressive=True)
    with pytest.raises(oracle.OracleError):
        oracle.Jpeg(b.getvalue())
