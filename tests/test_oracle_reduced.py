"""Pins of the oracle's reduced-resolution decode (the paper's Discussion:
lower resolutions from the DC and the first ACs instead of stored mips).

Closed forms: at full scale it is the MCU's texels; at 1/8 the DC alone, the
block mean; in general, for a single coefficient (u, v), the box average of
the full-resolution samples over M x M (M = 8 / N) is the reduced sample
times D_M(u) D_M(v), D_M(u) = sin(M u pi / 16) / (M sin(u pi / 16)) (the
Dirichlet kernel of averaging M neighbouring cosines), D_M(0) = 1."""
import numpy as np
import pytest

import oracle

from jpeg_writer import write_jpeg

Q1 = np.ones(64, np.int64)


def jpeg_for(sampling):
    n_du = 6 if sampling == 420 else 3
    side = 16 if sampling == 420 else 8
    return oracle.Jpeg(write_jpeg(side, side, sampling, Q1, Q1, [[(0, [(0x00, 0)])] * n_du]))


@pytest.mark.parametrize("sampling", [420, 444])
def test_full_scale_is_the_mcu(sampling):
    j = jpeg_for(sampling)
    rng = np.random.default_rng(1)
    c = (rng.integers(-40, 41, (j.n_du, 64)) * (rng.random((j.n_du, 64)) < 0.3)).astype(np.int16)
    a, fa = oracle.mcu_reduced(j, c, 0, want_f64=True)
    b, fb = j.mcu_pixels(c, want_f64=True)
    assert np.array_equal(a, b) and np.allclose(fa, fb, atol=1e-12)


def dirichlet(M, u):
    return 1.0 if u == 0 else np.sin(M * u * np.pi / 16) / (M * np.sin(u * np.pi / 16))


@pytest.mark.parametrize("s", [1, 2, 3])
@pytest.mark.parametrize("uv", [(0, 0), (1, 0), (0, 1), (1, 1), (3, 2), (2, 3)])
def test_single_coefficient_box_average(s, uv):
    N, M = 8 >> s, 1 << s
    u, v = uv
    if u >= N or v >= N:
        pytest.skip("frequency above the reduced band")
    j = jpeg_for(444)
    c = np.zeros((3, 64), np.int16)
    c[0, v * 8 + u] = 40                                  # luma only: R = G = B = Y
    _, f = oracle.mcu_reduced(j, c, s, want_f64=True)
    r = f[:, :, 0] - 128.0
    F = np.zeros(64)
    F[v * 8 + u] = 40.0
    full = oracle.idct(F)                                 # pinned to scipy's DCT-III elsewhere
    avg = full.reshape(N, M, N, M).mean(axis=(1, 3))
    assert np.allclose(r * dirichlet(M, u) * dirichlet(M, v), avg, atol=1e-9)


def test_dc_only_is_the_block_mean_420():
    j = jpeg_for(420)
    rng = np.random.default_rng(2)
    c = (rng.integers(-30, 31, (6, 64))).astype(np.int16)
    c[4:] = 0                                              # no chroma: colour = Y
    _, f = oracle.mcu_reduced(j, c, 3, want_f64=True)
    assert f.shape == (2, 2, 3)
    for d in range(4):
        mean = oracle.idct(c[d].astype(np.float64)).mean()
        want = np.clip(mean + 128.0, 0, 255)
        assert abs(f[d // 2, d % 2, 1] - want) < 1e-9
