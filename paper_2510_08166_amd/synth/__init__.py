"""Seeded synthetic inputs for the on-demand JPEG texture path.

Stand-ins for the paper's test scenes and texture sets (Sponza, Graffiti,
evaluation section), which are not available here: procedural RGB8 textures
(value noise plus hard-edged rectangles), box-filtered mip chains, baseline
JPEG files made by our own encoder, and deferred-shading G-buffers rasterised
from seeded random textured quads.

Nothing in this module decodes JPEG or samples textures; it only produces
inputs, which both the GPU path and the CPU checker consume.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_SO = os.path.join(_HERE, "libsynth.so")
_lock = threading.Lock()
_lib = None

GPIXEL_DTYPE = np.dtype([("u", "<f4"), ("v", "<f4"), ("tex", "<u4"), ("lod", "<f4")])
BACKGROUND = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (host code only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build()
            L = ctypes.CDLL(_SO)
            L.synth_texture.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
            L.synth_mip.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
            L.synth_encode.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.c_void_p]
            L.synth_quant_tables.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
            L.synth_raster.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------- textures
def texture(seed: int, w: int, h: int) -> np.ndarray:
    out = np.empty((h, w, 3), np.uint8)
    rc = lib().synth_texture(ctypes.c_uint64(seed & (2**64 - 1)), w, h, _ptr(out))
    if rc != 0:
        raise RuntimeError("synth_texture failed: %d" % rc)
    return out


def mip(rgb: np.ndarray) -> np.ndarray:
    h, w = rgb.shape[:2]
    rgb = np.ascontiguousarray(rgb)
    out = np.empty((max(1, h // 2), max(1, w // 2), 3), np.uint8)
    lib().synth_mip(_ptr(rgb), w, h, _ptr(out))
    return out


def mip_chain(rgb: np.ndarray, n_levels: int | None = None) -> list[np.ndarray]:
    """Level 0 plus successive 2x2 box reductions; n_levels=None -> down to 1x1."""
    levels = [rgb]
    while True:
        h, w = levels[-1].shape[:2]
        if n_levels is not None and len(levels) >= n_levels:
            break
        if n_levels is None and w == 1 and h == 1:
            break
        levels.append(mip(levels[-1]))
    return levels


def full_chain_length(w: int, h: int) -> int:
    return int(max(w, h)).bit_length()


def quant_tables(quality: int) -> tuple[np.ndarray, np.ndarray]:
    """IJG-scaled Annex K tables (natural order) the encoder uses at this quality."""
    l = np.empty(64, np.uint16); c = np.empty(64, np.uint16)
    lib().synth_quant_tables(int(quality), _ptr(l), _ptr(c))
    return l, c


def encode(rgb: np.ndarray, quality: int, sampling: int = 420, want_coef: bool = False):
    """Baseline JPEG bytes (and optionally the quantised coefficients,
    natural order, shape [n_mcu, n_du, 64])."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    h, w = rgb.shape[:2]
    ms = 16 if sampling == 420 else 8
    n_mcu = ((w + ms - 1) // ms) * ((h + ms - 1) // ms)
    ndu = 6 if sampling == 420 else 3
    coef = np.zeros((n_mcu, ndu, 64), np.int16) if want_coef else None
    cap = 4096 + w * h * 4
    out = np.empty(cap, np.uint8)
    n = ctypes.c_size_t(0)
    rc = lib().synth_encode(_ptr(rgb), w, h, int(quality), int(sampling), _ptr(out), cap, ctypes.byref(n),
                            _ptr(coef) if want_coef else None)
    if rc != 0:
        raise RuntimeError("synth_encode failed: %d" % rc)
    data = out[: n.value].tobytes()
    return (data, coef) if want_coef else data


# --------------------------------------------------------------- G-buffer
def _homography(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """3x3 H with dst ~ H src for four point pairs (direct linear solve, h33 = 1)."""
    A = np.zeros((8, 8)); b = np.zeros(8)
    for i in range(4):
        x, y = src[i]; X, Y = dst[i]
        A[2 * i] = [x, y, 1, 0, 0, 0, -X * x, -X * y]; b[2 * i] = X
        A[2 * i + 1] = [0, 0, 0, x, y, 1, -Y * x, -Y * y]; b[2 * i + 1] = Y
    h = np.linalg.solve(A, b)
    return np.append(h, 1.0).reshape(3, 3)


UNIT_SQUARE = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])


def random_quads(rng: np.random.Generator, W: int, H: int, n_quads: int, tex_ids, tex_sizes):
    """Seeded quad soup: screen centre uniform over the frame +-10%, half
    extents log-uniform in [0.05, 0.5]*H, uniform rotation, a random
    projective tilt, uniform depth, texture id uniform over tex_ids, uv scale
    log-uniform in [0.25, 4] repeats, uniform uv offset.  Returns a list of
    dicts holding the screen corners of each quad."""
    quads = []
    tex_ids = np.asarray(tex_ids)
    for _ in range(n_quads):
        cx = rng.uniform(-0.1 * W, 1.1 * W); cy = rng.uniform(-0.1 * H, 1.1 * H)
        a = H * np.exp(rng.uniform(np.log(0.05), np.log(0.5)))
        b = H * np.exp(rng.uniform(np.log(0.05), np.log(0.5)))
        th = rng.uniform(0, 2 * np.pi)
        c, s = np.cos(th), np.sin(th)
        local = np.array([[-a, -b], [a, -b], [a, b], [-a, b]])
        tilt_dir = rng.uniform(0, 2 * np.pi); k = rng.uniform(0.0, 0.6)
        d = np.array([np.cos(tilt_dir), np.sin(tilt_dir)])
        ext = max(a, b)
        corners = []
        for p in local:
            f = 1.0 + k * (p @ d) / ext          # far side shrinks, near side grows
            p = p * f
            corners.append([cx + c * p[0] - s * p[1], cy + s * p[0] + c * p[1]])
        t = int(tex_ids[rng.integers(len(tex_ids))])
        quads.append(dict(corners=np.array(corners), depth=rng.uniform(0, 1), tex=t,
                          scale=float(np.exp(rng.uniform(np.log(0.25), np.log(4.0)))),
                          off=(rng.uniform(), rng.uniform()), texwh=tex_sizes[t]))
    return quads


def rasterise(W: int, H: int, quads, screen_xform: np.ndarray | None = None) -> np.ndarray:
    """G-buffer (H, W) of GPIXEL_DTYPE from quads drawn far to near.
    screen_xform (3x3, optional) moves every quad on screen (camera drift,
    second eye of a stereo pair, ...)."""
    order = sorted(range(len(quads)), key=lambda i: -quads[i]["depth"])
    Gs, boxes, texs, uvp, twh = [], [], [], [], []
    for i in order:
        q = quads[i]
        Hm = _homography(UNIT_SQUARE, q["corners"])
        if screen_xform is not None:
            Hm = screen_xform @ Hm
        pts = (Hm @ np.c_[UNIT_SQUARE, np.ones(4)].T).T
        if np.any(pts[:, 2] <= 0):
            continue
        pts = pts[:, :2] / pts[:, 2:3]
        x0, y0 = np.floor(pts.min(0)).astype(int); x1, y1 = np.ceil(pts.max(0)).astype(int) + 1
        x0, y0 = max(x0, 0), max(y0, 0); x1, y1 = min(x1, W), min(y1, H)
        if x0 >= x1 or y0 >= y1:
            continue
        Gs.append(np.linalg.inv(Hm).ravel()); boxes.append([x0, y0, x1, y1]); texs.append(q["tex"])
        uvp.append([q["scale"], q["scale"], q["off"][0], q["off"][1]]); twh.append(q["texwh"])
    g = np.zeros((H, W), GPIXEL_DTYPE)
    g["tex"] = BACKGROUND
    if Gs:
        G = np.ascontiguousarray(np.array(Gs, np.float64)); B = np.ascontiguousarray(np.array(boxes, np.int32))
        T = np.ascontiguousarray(np.array(texs, np.uint32)); U = np.ascontiguousarray(np.array(uvp, np.float64))
        S = np.ascontiguousarray(np.array(twh, np.float64))
        lib().synth_raster(W, H, len(Gs), _ptr(G), _ptr(B), _ptr(T), _ptr(U), _ptr(S), _ptr(g))
    return g


def similarity(tx: float, ty: float, rot_deg: float, zoom: float, W: int, H: int) -> np.ndarray:
    """Screen-space camera move about the frame centre."""
    c, s = np.cos(np.radians(rot_deg)) * zoom, np.sin(np.radians(rot_deg)) * zoom
    cx, cy = W / 2.0, H / 2.0
    return np.array([[c, -s, cx - c * cx + s * cy + tx], [s, c, cy - s * cx - c * cy + ty], [0, 0, 1.0]])


# ------------------------------------------------------------ texture sets
class EncodedTexture:
    """One texture: its levels as JPEG files (and the RGB levels when kept)."""

    def __init__(self, tex_id, width, height, quality, sampling, jpegs, rgb_levels=None):
        self.tex_id = tex_id; self.width = width; self.height = height
        self.quality = quality; self.sampling = sampling
        self.jpegs = jpegs; self.rgb_levels = rgb_levels


def make_texture(seed: int, w: int, h: int, quality: int, sampling: int, n_levels, keep_rgb=False, tex_id=0):
    base = texture(seed, w, h)
    levels = mip_chain(base, n_levels)
    jpegs = [encode(l, quality, sampling) for l in levels]
    return EncodedTexture(tex_id, w, h, quality, sampling, jpegs, levels if keep_rgb else None)


def make_textures(specs, keep_rgb=False, threads: int | None = None, log=None):
    """specs: list of (seed, w, h, quality, sampling, n_levels).  Runs the C
    generators on a thread pool (ctypes releases the GIL).  `log` (optional)
    is called with a progress line every 16 textures."""
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        futs = [ex.submit(make_texture, s, w, h, q, smp, nl, keep_rgb, i)
                for i, (s, w, h, q, smp, nl) in enumerate(specs)]
        out = []
        for i, f in enumerate(futs):
            out.append(f.result())
            if log and (i + 1) % 16 == 0:
                log("textures %d / %d" % (i + 1, len(futs)))
        return out


def seed_ints(seed: int, n: int) -> list[int]:
    return [int(s.generate_state(1, np.uint64)[0]) for s in np.random.SeedSequence(seed).spawn(n)]


def target_frame(seed: int, H: int, W: int) -> np.ndarray:
    """Seeded target image for an L2 loss: [H, W, 3] float32, uniform in [0, 255]."""
    return np.random.default_rng(seed).uniform(0.0, 255.0, (H, W, 3)).astype(np.float32)
