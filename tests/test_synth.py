"""The seeded input generator: deterministic, and its baseline JPEG files
carry the Annex K tables exactly as libjpeg (run through PIL) writes them at
the same quality."""
import io

import numpy as np
import pytest
from PIL import Image

from paper_2510_08166_amd import synth
from paper_2510_08166_amd.synth import configs


def segments(data: bytes):
    """(marker, payload) pairs up to SOS."""
    out, p = [], 2
    while p < len(data):
        m = data[p + 1]
        L = int.from_bytes(data[p + 2:p + 4], "big")
        out.append((m, data[p + 4:p + 2 + L]))
        if m == 0xDA:
            break
        p += 2 + L
    return out


def tables(data: bytes):
    dqt, dht = {}, {}
    for m, s in segments(data):
        o = 0
        if m == 0xDB:
            while o < len(s):
                dqt[s[o] & 15] = bytes(s[o + 1:o + 65]); o += 65
        elif m == 0xC4:
            while o < len(s):
                n = sum(s[o + 1:o + 17])
                dht[s[o]] = bytes(s[o + 1:o + 17 + n]); o += 17 + n
    return dqt, dht


@pytest.mark.parametrize("q", [1, 10, 25, 50, 51, 75, 90, 99, 100])
def test_tables_equal_libjpeg(q):
    rgb = synth.texture(1, 32, 32)
    b = io.BytesIO()
    Image.fromarray(rgb).save(b, format="JPEG", quality=q, subsampling=2, optimize=False)
    pq, ph = tables(b.getvalue())
    oq, oh = tables(synth.encode(rgb, q, 420))
    assert pq == oq
    assert ph == oh


def test_deterministic_and_seeded():
    a = synth.texture(5, 64, 48); b = synth.texture(5, 64, 48); c = synth.texture(6, 64, 48)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert synth.encode(a, 75, 420) == synth.encode(b, 75, 420)
    g1 = configs.reduced(seed=3).views[0]; g2 = configs.reduced(seed=3).views[0]
    assert g1.tobytes() == g2.tobytes()


def test_mip_chain_box_filter():
    rgb = synth.texture(2, 64, 32)
    ch = synth.mip_chain(rgb)
    assert [l.shape[:2] for l in ch] == [(32, 64), (16, 32), (8, 16), (4, 8), (2, 4), (1, 2), (1, 1)]
    a = rgb.astype(int)
    want = (a[0::2, 0::2] + a[1::2, 0::2] + a[0::2, 1::2] + a[1::2, 1::2] + 2) >> 2
    assert np.array_equal(ch[1], want)


def test_gbuffer_recipe():
    wl = configs.reduced(seed=9, W=200, H=120, n_quads=30)
    g = wl.views[0]
    fg = g["tex"] != 0xFFFFFFFF
    assert fg.mean() > 0.5
    assert np.isfinite(g["lod"][fg]).all() and np.isfinite(g["u"][fg]).all()
    assert set(np.unique(g["tex"][fg])) <= set(range(len(wl.textures)))
