"""Seeded workloads.  They stand in for the paper's Sponza / Graffiti scenes
(evaluation section, test-scene table), which are not available: same frame
sizes (1920x1080 desktop), textures of 1k-8k texels per side, mip chains,
and repeated as well as non-repeating uv mappings.

  tiny      one 256x256 texture, q75, 4:2:0, single level; a 256x256 frame
            that maps pixel centres 1:1 onto texel centres, nearest filter.
  1080p     32 textures of 2048x2048, q ~ U{50..90}, 4:2:0, 8 levels each
            (2048 .. 16); 1920x1080 frame from 200 random quads, bilinear.
  diff1080  the differentiable-form scene: as 1080p with every texture at q75.
  reduced   the 1080p recipe at a size the CPU checker finishes quickly
            (used by tests only).
"""
from __future__ import annotations

import numpy as np

from . import GPIXEL_DTYPE, make_textures, random_quads, rasterise, seed_ints

FILTER_NEAREST, FILTER_BILINEAR, FILTER_TRILINEAR, FILTER_BILINEAR_CLAMPED = 0, 1, 2, 3
FILTER_MIP_OFF = 0x100


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


def diff1080(keep_rgb=False) -> Workload:
    """Differentiable-form scene: 32 textures of 2048x2048 at q75, 4:2:0,
    8 levels; 1920x1080 frame from 200 quads, bilinear."""
    return quad_scene(5, 32, 2048, 75, 75, 8, 1920, 1080, 200, keep_rgb=keep_rgb,
                      name="diff 1080p: 32 x 2048^2 q75 4:2:0 8 levels, 200 quads, bilinear")


def reduced(seed=7, n_tex=4, side=256, W=320, H=200, n_quads=24, n_levels=5, filt=FILTER_BILINEAR,
            keep_rgb=False) -> Workload:
    return quad_scene(seed, n_tex, side, 50, 90, n_levels, W, H, n_quads, filt=filt, keep_rgb=keep_rgb,
                      name="reduced %dx%d^2, %dx%d" % (n_tex, side, W, H))


def drift_transforms(rng: np.random.Generator, W: int, H: int, n_frames: int):
    """Seeded camera drift: per frame a random-walk step of translation
    ~ N(0, 1% of W), rotation ~ N(0, 0.5 deg), zoom ~ exp N(0, 0.02)."""
    from . import similarity
    tx = ty = rot = 0.0
    zoom = 1.0
    out = []
    for f in range(n_frames):
        if f:
            tx += rng.normal(0, 0.01 * W); ty += rng.normal(0, 0.01 * W)
            rot += rng.normal(0, 0.5); zoom *= float(np.exp(rng.normal(0, 0.02)))
        out.append(similarity(tx, ty, rot, zoom, W, H))
    return out


def heavy(seed=3, n_tex=256, sides=(512, 1024, 2048, 4096, 8192), q_lo=40, q_hi=95, W=3840, H=2160, n_quads=2000,
          n_frames=8, keep_rgb=False, name=None, log=None) -> Workload:
    """Heavy recipe: textures of random power-of-two sides, q ~ U{q_lo..q_hi},
    4:2:0 / 4:4:4 half and half, full mip chains; a quad scene seen over
    n_frames frames of seeded camera drift; trilinear.  Views = frames."""
    from . import make_textures, random_quads, rasterise
    ss = np.random.SeedSequence(seed)
    tex_seq, prm_seq, scene_seq, cam_seq = ss.spawn(4)
    tex_seeds = [int(s.generate_state(1, np.uint64)[0]) for s in tex_seq.spawn(n_tex)]
    prm = np.random.default_rng(prm_seq)
    side = prm.choice(np.array(sides), n_tex)
    qs = prm.integers(q_lo, q_hi + 1, n_tex)
    smp = np.where(prm.random(n_tex) < 0.5, 420, 444)
    specs = [(tex_seeds[i], int(side[i]), int(side[i]), int(qs[i]), int(smp[i]), None) for i in range(n_tex)]
    textures = make_textures(specs, keep_rgb=keep_rgb, log=log)
    rng = np.random.default_rng(scene_seq)
    sizes = {i: (float(side[i]), float(side[i])) for i in range(n_tex)}
    quads = random_quads(rng, W, H, n_quads, list(range(n_tex)), sizes)
    xf = drift_transforms(np.random.default_rng(cam_seq), W, H, n_frames)
    frames = [rasterise(W, H, quads, x) for x in xf]
    return Workload(name or "heavy %d tex, %dx%d, %d frames" % (n_tex, W, H, n_frames), textures, frames,
                    FILTER_TRILINEAR, dict(quads=quads, qualities=qs.tolist(), sides=side.tolist(),
                                           sampling=smp.tolist()))


def batched(seed=4, n_pool=128, sides=(512, 1024, 2048, 4096), q_lo=50, q_hi=90, n_pairs=2,
            eye=(2064, 2208), n_mono=12, mono_w=(1280, 2560), tex_per_scene=(8, 64), quads_per_mpx=96,
            filt=FILTER_BILINEAR, name=None, log=None) -> Workload:
    """Batched recipe: a pool of n_pool 4:2:0 textures (side uniform over
    `sides`, q ~ U{q_lo..q_hi}, full mip chains) seen by n_pairs stereo
    pairs of eye[0] x eye[1] pixels per eye and n_mono mono views of width
    ~ U[mono_w] at 16:9.  Each scene (a stereo pair shares one) draws its
    own subset of tex_per_scene textures and quads_per_mpx quads per
    megapixel; the second eye sees the first eye's quads shifted by a
    horizontal disparity of 3% of its width.  Views: pairs first, then mono."""
    ss = np.random.SeedSequence(seed)
    tex_seq, prm_seq, scene_seq = ss.spawn(3)
    tex_seeds = [int(s.generate_state(1, np.uint64)[0]) for s in tex_seq.spawn(n_pool)]
    prm = np.random.default_rng(prm_seq)
    side = prm.choice(np.array(sides), n_pool)
    qs = prm.integers(q_lo, q_hi + 1, n_pool)
    specs = [(tex_seeds[i], int(side[i]), int(side[i]), int(qs[i]), 420, None) for i in range(n_pool)]
    textures = make_textures(specs, log=log)
    sizes = {i: (float(side[i]), float(side[i])) for i in range(n_pool)}
    rng = np.random.default_rng(scene_seq)
    from . import similarity
    views, shapes = [], []

    def scene(W, H):
        k = int(rng.integers(tex_per_scene[0], tex_per_scene[1] + 1))
        ids = sorted(rng.choice(n_pool, min(k, n_pool), replace=False).tolist())
        nq = max(1, int(round(quads_per_mpx * W * H / 1e6)))
        return random_quads(rng, W, H, nq, ids, sizes)

    for _ in range(n_pairs):
        W, H = eye
        quads = scene(W, H)
        views.append(rasterise(W, H, quads))
        views.append(rasterise(W, H, quads, similarity(-0.03 * W, 0.0, 0.0, 1.0, W, H)))
        shapes += [(W, H)] * 2
    for _ in range(n_mono):
        W = int(rng.integers(mono_w[0] // 16, mono_w[1] // 16 + 1)) * 16
        H = W * 9 // 16
        views.append(rasterise(W, H, scene(W, H)))
        shapes.append((W, H))
    return Workload(name or "batched %d views (%d stereo pairs %dx%d + %d mono), %d-texture pool"
                    % (len(views), n_pairs, eye[0], eye[1], n_mono, n_pool), textures, views, filt,
                    dict(shapes=shapes, sides=side.tolist(), qualities=qs.tolist()))


def batched16(log=None) -> Workload:
    """The 16-view batch: 2 stereo pairs of 2064x2208 + 12 mono views from
    1280x720 to 2560x1440 over a 128-texture pool of sides 512..4096."""
    return batched(log=log)


def batched_small(seed=6, filt=FILTER_BILINEAR) -> Workload:
    """The batched recipe at a size the CPU checker finishes quickly."""
    return batched(seed=seed, n_pool=10, sides=(64, 128, 256), n_pairs=1, eye=(96, 104), n_mono=3,
                   mono_w=(64, 160), tex_per_scene=(2, 6), quads_per_mpx=2000, filt=filt,
                   name="batched small")
