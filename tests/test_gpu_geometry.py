"""GPU geometry pass (jpt_geometry_pass) against the oracle's fp64 ray cast,
and the frame rendered from the GPU's G-buffer against the oracle.

fp32 against fp64: a pixel whose centre ray passes within rounding of a
triangle edge or of a depth tie may take the other triangle, so texture ids
must agree on all but a tiny share of pixels; where they agree, uv agrees to
1e-4 and lod to 2e-3 (the footprint is a difference of neighbouring uv,
which loses the leading digits)."""
import numpy as np
import pytest

import oracle
from paper_2510_08166_amd import synth
from paper_2510_08166_amd.synth import configs

from gpu_common import full_parity

pytestmark = pytest.mark.gpu


def room(n_tex=6, side=256):
    tex = synth.make_textures([(90 + i, side, side, 60 + 5 * i, 420 if i % 2 else 444, None) for i in range(n_tex)])
    tris = synth.room_scene(3, n_tex, tex_side=side, texels_per_unit=64.0)
    return tex, tris


def gpu_gbuffer(tex, tris, cam, W, H):
    import torch
    from paper_2510_08166_amd import jpt
    host = jpt.HostScene(tex)
    scene = jpt.DeviceScene(host)
    views = jpt.Views([np.zeros((H, W), synth.GPIXEL_DTYPE)])
    t = torch.from_numpy(np.ascontiguousarray(tris).view(np.uint8).copy()).cuda()
    jpt.geometry_pass(scene, t, cam, views)
    torch.cuda.synchronize()
    return views.gbufs[0].cpu().numpy().view(synth.GPIXEL_DTYPE).reshape(H, W), host


@pytest.mark.parametrize("yaw", [0.0, 37.0, 200.0])
def test_geometry_matches_oracle(gpu, yaw):
    W, H = 320, 180
    tex, tris = room()
    cam = synth.camera((0.3, 1.7, -0.2), yaw, -8.0, 90.0, W, H)
    g, _ = gpu_gbuffer(tex, tris, cam, W, H)
    ref = oracle.geometry(tris, cam, W, H, [t.width for t in tex], [t.height for t in tex])
    same = g["tex"] == ref["tex"]
    fg = ref["tex"] != oracle.BACKGROUND
    print("yaw %.0f: %d of %d pixels differ in texture, %d foreground" % (yaw, (~same).sum(), same.size, fg.sum()))
    assert (~same).sum() <= same.size // 2000
    m = same & fg
    du = np.abs(g["u"][m] - ref["u"][m]).max(); dv = np.abs(g["v"][m] - ref["v"][m]).max()
    dl = np.abs(g["lod"][m] - ref["lod"][m]).max()
    print("max |du| %.2e |dv| %.2e |dlod| %.2e" % (du, dv, dl))
    assert du <= 1e-4 and dv <= 1e-4 and dl <= 2e-3


def test_frame_from_gpu_geometry(gpu):
    """The whole frame from triangles: GPU geometry, then mark, decode and
    resolve, checked against the oracle on the GPU's own G-buffer."""
    W, H = 256, 144
    tex, tris = room()
    cam = synth.camera((0.0, 1.7, 0.0), 120.0, -10.0, 90.0, W, H)
    g, _ = gpu_gbuffer(tex, tris, cam, W, H)
    wl = configs.Workload("room from triangles", tex, [g], configs.FILTER_TRILINEAR)
    full_parity(wl)
