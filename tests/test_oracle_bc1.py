"""Pins of the oracle's BC1 decoder (the fixed-rate baseline; the paper's
Background: BC1): hand-built blocks in both palette modes, the bit layout of
the indices, endpoint widening by bit replication, and the encoder's
exactness on colours RGB565 represents."""
import numpy as np

import oracle
from paper_2510_08166_amd import synth


def block(c0, c1, idx):
    bits = sum(int(k) << (2 * i) for i, k in enumerate(np.asarray(idx).ravel()))
    return bytes([c0 & 255, c0 >> 8, c1 & 255, c1 >> 8]) + bits.to_bytes(4, "little")


def test_four_colour_block_by_hand():
    # c0 = pure red 31<<11 -> (255, 0, 0); c1 = blue 31 -> (0, 0, 255)
    idx = np.array([[0, 1, 2, 3]] * 4)
    img = oracle.bc1_decode(block(31 << 11, 31, idx), 4, 4)
    want = np.array([[255, 0, 0], [0, 0, 255], [170, 0, 85], [85, 0, 170]])   # (2*255+0+1)//3 = 170 ...
    assert np.array_equal(img[0], want) and np.array_equal(img[3], want)


def test_three_colour_block_and_black():
    # c0 <= c1: palette {c0, c1, (c0 + c1 + 1) // 2, black}
    c0, c1 = (8 << 11) | (16 << 5) | 4, (9 << 11) | (17 << 5) | 5
    idx = np.array([[3, 2, 1, 0]] * 4).T                    # rows: index 3, 2, 1, 0
    img = oracle.bc1_decode(block(c0, c1, idx), 4, 4)
    e0 = np.array([(8 << 3) | (8 >> 2), (16 << 2) | (16 >> 4), (4 << 3) | (4 >> 2)])
    e1 = np.array([(9 << 3) | (9 >> 2), (17 << 2) | (17 >> 4), (5 << 3) | (5 >> 2)])
    assert (img[0] == 0).all()
    assert np.array_equal(img[1, 0], (e0 + e1 + 1) // 2)
    assert np.array_equal(img[2, 0], e1) and np.array_equal(img[3, 0], e0)


def test_ragged_image_and_exact_colours():
    rng = np.random.default_rng(3)
    # colours whose 8-bit channels come from 5/6-bit values by replication are exact
    r = rng.integers(0, 32, (10, 7)); g = rng.integers(0, 64, (10, 7)); b = rng.integers(0, 32, (10, 7))
    img = np.stack([(r << 3) | (r >> 2), (g << 2) | (g >> 4), (b << 3) | (b >> 2)], -1).astype(np.uint8)
    img[:, :, :] = img[:1, :1, :]           # one colour per image: the encoder's endpoints are that colour
    dec = oracle.bc1_decode(synth.bc1_encode(img), 7, 10)
    assert np.array_equal(dec, img)
    # a two-colour block whose endpoints are exact decodes exactly
    two = np.zeros((4, 4, 3), np.uint8)
    two[:, :2] = (255, 0, 0)
    two[:, 2:] = (0, 0, 255)
    assert np.array_equal(oracle.bc1_decode(synth.bc1_encode(two), 4, 4), two)
