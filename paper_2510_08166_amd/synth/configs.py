"""Seeded workloads.  They stand in for the paper's Sponza / Graffiti scenes
(evaluation section, test-scene table), which are not available: same frame
sizes (1920x1080 desktop), textures of 1k-8k texels per side, mip chains,
and repeated as well as non-repeating uv mappings.

  tiny      one 256x256 texture, q75, 4:2:0, single level; a 256x256 frame
            that maps pixel centres 1:1 onto texel centres, nearest filter.
  1080p     32 textures of 2048x2048, q ~ U{50..90}, 4:2:0, 8 levels each
            (2048 .. 16); 1920x1080 frame from 200 random quads, bilinear.
  reduced   the 1080p recipe at a size the CPU checker finishes quickly
            (used by tests only).
"""
from __future__ import annotations

import numpy as np

from . import GPIXEL_DTYPE, make_textures, random_quads, rasterise, seed_ints

FILTER_NEAREST, FILTER_BILINEAR, FILTER_TRILINEAR = 0, 1, 2


class Workload:
    def __init__(self, name, textures, views, filt, extra=None):
        self.name = name
        self.textures = textures          # list[EncodedTexture]
        self.views = views                # list of G-buffers (H, W) GPIXEL_DTYPE
        self.filter = filt
        self.extra = extra or {}

    @property
    def n_pixels(self):
        return sum(v.shape[0] * v.shape[1] for v in self.views)


def tiny(keep_rgb=False) -> Workload:
    (s,) = seed_ints(1, 1)
    tex = make_textures([(s, 256, 256, 75, 420, 1)], keep_rgb=keep_rgb)
    y, x = np.mgrid[0:256, 0:256]
    g = np.zeros((256, 256), GPIXEL_DTYPE)
    g["u"] = ((x + 0.5) / 256).astype(np.float32)
    g["v"] = ((y + 0.5) / 256).astype(np.float32)
    g["tex"] = 0
    g["lod"] = 0.0
    return Workload("tiny 256x256 q75 4:2:0 nearest", tex, [g], FILTER_NEAREST)


def quad_scene(seed, n_tex, tex_side, q_lo, q_hi, n_levels, W, H, n_quads, sampling=420,
               filt=FILTER_BILINEAR, keep_rgb=False, name=None) -> Workload:
    ss = np.random.SeedSequence(seed)
    tex_seq, q_seq, scene_seq = ss.spawn(3)
    tex_seeds = [int(s.generate_state(1, np.uint64)[0]) for s in tex_seq.spawn(n_tex)]
    qs = np.random.default_rng(q_seq).integers(q_lo, q_hi + 1, n_tex)
    specs = [(tex_seeds[i], tex_side, tex_side, int(qs[i]), sampling, n_levels) for i in range(n_tex)]
    textures = make_textures(specs, keep_rgb=keep_rgb)
    rng = np.random.default_rng(scene_seq)
    sizes = {i: (float(tex_side), float(tex_side)) for i in range(n_tex)}
    quads = random_quads(rng, W, H, n_quads, list(range(n_tex)), sizes)
    g = rasterise(W, H, quads)
    return Workload(name or "quads", textures, [g], filt, dict(quads=quads, qualities=qs.tolist()))


def frame1080(keep_rgb=False) -> Workload:
    return quad_scene(2, 32, 2048, 50, 90, 8, 1920, 1080, 200, keep_rgb=keep_rgb,
                      name="1080p: 32 x 2048^2 q50-90 4:2:0 8 levels, 200 quads, bilinear")


def reduced(seed=7, n_tex=4, side=256, W=320, H=200, n_quads=24, n_levels=5, filt=FILTER_BILINEAR,
            keep_rgb=False) -> Workload:
    return quad_scene(seed, n_tex, side, 50, 90, n_levels, W, H, n_quads, filt=filt, keep_rgb=keep_rgb,
                      name="reduced %dx%d^2, %dx%d" % (n_tex, side, W, H))
