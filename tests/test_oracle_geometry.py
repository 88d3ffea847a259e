"""Pins of the oracle's geometry pass (the pass before Mark): closed forms of
a fronto-parallel quad (uv linear in the pixel centre, lod = log2 of the
texels per pixel), occlusion by depth, background, and the lower index on
equal depth."""
import numpy as np

import oracle
from paper_2510_08166_amd import synth

W, H = 64, 48


def front_camera(fov=60.0):
    return synth.camera((0.0, 0.0, 0.0), 0.0, 0.0, fov, W, H)


def test_fronto_parallel_quad_closed_form():
    D, X, Y, su, sv, tw, th = 5.0, 4.0, 3.0, 2.0, 1.5, 512, 256
    tris = synth.quad_triangles((-X, -Y, -D), (2 * X, 0, 0), (0, 2 * Y, 0), (su, sv), 7)
    cam = front_camera()
    g = oracle.geometry(tris, cam, W, H, [1] * 7 + [tw], [1] * 7 + [th])
    tx, ty = float(cam["tan_half_x"][0]), float(cam["tan_half_y"][0])
    x, y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    sx = (2 * x / W - 1) * tx
    sy = (1 - 2 * y / H) * ty
    a = (sx * D + X) / (2 * X)
    b = (sy * D + Y) / (2 * Y)
    inside = (a >= 0) & (a <= 1) & (b >= 0) & (b <= 1)
    assert inside.all()                      # the quad fills the view (tan 30 deg * 5 < 4)
    assert (g["tex"] == 7).all()
    assert np.allclose(g["u"], a * su, atol=1e-6) and np.allclose(g["v"], b * sv, atol=1e-6)
    rho = max(2 * tx / W * D / (2 * X) * su * tw, 2 * ty / H * D / (2 * Y) * sv * th)
    assert np.allclose(g["lod"], np.log2(rho), atol=1e-5)


def test_nearer_quad_occludes_and_misses_are_background():
    back = synth.quad_triangles((-10, -10, -9), (20, 0, 0), (0, 20, 0), (1, 1), 1)
    front = synth.quad_triangles((0, -10, -4), (10, 0, 0), (0, 20, 0), (1, 1), 2)   # right half, nearer
    tris = np.concatenate([back, front])
    g, hit = oracle.geometry(tris, front_camera(), W, H, [64] * 3, [64] * 3, want_tri=True)
    assert (g["tex"][:, W // 2 + 1:] == 2).all() and (g["tex"][:, : W // 2 - 1] == 1).all()
    # nothing behind the camera or beside the quads: background
    g2 = oracle.geometry(synth.quad_triangles((-1, -1, 5), (2, 0, 0), (0, 2, 0), (1, 1), 0), front_camera(), W, H,
                         [64], [64])
    assert (g2["tex"] == oracle.BACKGROUND).all()


def test_equal_depth_takes_the_lower_index():
    a = synth.quad_triangles((-10, -10, -6), (20, 0, 0), (0, 20, 0), (1, 1), 3)
    b = synth.quad_triangles((-10, -10, -6), (20, 0, 0), (0, 20, 0), (1, 1), 5)
    g, hit = oracle.geometry(np.concatenate([a, b]), front_camera(), W, H, [64] * 6, [64] * 6, want_tri=True)
    assert (g["tex"] == 3).all() and (hit < 2).all()
