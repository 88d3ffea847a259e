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
            L.synth_bc1_encode.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
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

    def __init__(self, tex_id, width, height, quality, sampling, jpegs, rgb_levels=None, seed=None):
        self.tex_id = tex_id; self.width = width; self.height = height
        self.quality = quality; self.sampling = sampling
        self.jpegs = jpegs; self.rgb_levels = rgb_levels
        self.seed = seed   # of the procedural base image (synth texture), when generated here


def make_texture(seed: int, w: int, h: int, quality: int, sampling: int, n_levels, keep_rgb=False, tex_id=0):
    base = texture(seed, w, h)
    levels = mip_chain(base, n_levels)
    jpegs = [encode(l, quality, sampling) for l in levels]
    return EncodedTexture(tex_id, w, h, quality, sampling, jpegs, levels if keep_rgb else None, seed=seed)


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


# ------------------------------------------------------------- 3-D scenes
# Triangles and cameras for the geometry pass (the pass before Mark): the
# layouts of jpt_triangle (80 bytes) and jpt_camera (64 bytes).
TRIANGLE_DTYPE = np.dtype([("p0", "<f4", 3), ("p1", "<f4", 3), ("p2", "<f4", 3), ("uv0", "<f4", 2),
                           ("uv1", "<f4", 2), ("uv2", "<f4", 2), ("tex", "<u4"), ("reserved", "<u4", 4)])
CAMERA_DTYPE = np.dtype([("eye", "<f4", 3), ("fwd", "<f4", 3), ("right", "<f4", 3), ("up", "<f4", 3),
                         ("tan_half_x", "<f4"), ("tan_half_y", "<f4"), ("reserved", "<f4", 2)])
assert TRIANGLE_DTYPE.itemsize == 80 and CAMERA_DTYPE.itemsize == 64


def quad_triangles(corner, e1, e2, uv_scale, tex):
    """Two triangles covering corner + a e1 + b e2 (a, b in [0, 1]) with
    uv = (a su, b sv)."""
    c = np.asarray(corner, np.float64); e1 = np.asarray(e1, np.float64); e2 = np.asarray(e2, np.float64)
    su, sv = uv_scale
    t = np.zeros(2, TRIANGLE_DTYPE)
    t[0]["p0"], t[0]["p1"], t[0]["p2"] = c, c + e1, c + e1 + e2
    t[0]["uv0"], t[0]["uv1"], t[0]["uv2"] = (0, 0), (su, 0), (su, sv)
    t[1]["p0"], t[1]["p1"], t[1]["p2"] = c, c + e1 + e2, c + e2
    t[1]["uv0"], t[1]["uv1"], t[1]["uv2"] = (0, 0), (su, sv), (0, sv)
    t["tex"] = tex
    return t


def room_scene(seed: int, n_tex: int, size=24.0, height=8.0, panels=6, n_boxes=24, texels_per_unit=256.0,
               tex_side=2048):
    """An atrium-like room (a stand-in for the paper's Sponza): floor,
    ceiling and four walls cut into panels, and boxes (pillars and crates)
    inside, every face a textured quad with a seeded texture id; uv
    scales give about `texels_per_unit` texels per world unit.  Returns the
    triangles (TRIANGLE_DTYPE)."""
    rng = np.random.default_rng(seed)
    tris = []
    s = size / 2.0
    rep = texels_per_unit / tex_side

    def add(corner, e1, e2):
        l1, l2 = np.linalg.norm(e1), np.linalg.norm(e2)
        tris.append(quad_triangles(corner, e1, e2, (l1 * rep, l2 * rep), int(rng.integers(0, n_tex))))

    step = size / panels
    for i in range(panels):
        for j in range(panels):
            add((-s + i * step, 0.0, -s + j * step), (step, 0, 0), (0, 0, step))        # floor
            add((-s + i * step, height, -s + j * step), (0, 0, step), (step, 0, 0))     # ceiling
    hs = height / 2
    for i in range(panels):
        for j in range(2):
            a = -s + i * step
            add((a, j * hs, -s), (step, 0, 0), (0, hs, 0))                # wall z = -s
            add((a + step, j * hs, s), (-step, 0, 0), (0, hs, 0))         # wall z = +s
            add((-s, j * hs, a + step), (0, 0, -step), (0, hs, 0))        # wall x = -s
            add((s, j * hs, a), (0, 0, step), (0, hs, 0))                 # wall x = +s
    for _ in range(n_boxes):
        cx, cz = rng.uniform(-s * 0.8, s * 0.8, 2)
        if abs(cx) < 2.0 and abs(cz) < 2.0:
            cx += 3.0 * np.sign(cx or 1.0)
        w, d = rng.uniform(0.4, 1.6, 2)
        h = rng.uniform(0.5, height) if rng.random() < 0.5 else height
        x0, x1, z0, z1 = cx - w / 2, cx + w / 2, cz - d / 2, cz + d / 2
        add((x0, 0, z0), (w, 0, 0), (0, h, 0))
        add((x1, 0, z1), (-w, 0, 0), (0, h, 0))
        add((x0, 0, z1), (0, 0, -d), (0, h, 0))
        add((x1, 0, z0), (0, 0, d), (0, h, 0))
        add((x0, h, z0), (0, 0, d), (w, 0, 0))
    return np.concatenate(tris)


def camera(eye, yaw_deg: float, pitch_deg: float, fov_x_deg: float, W: int, H: int) -> np.ndarray:
    """A pinhole camera at `eye` turned by yaw (about the vertical axis, from
    looking along -z) and pitch; square pixels."""
    yaw, pitch = np.radians(yaw_deg), np.radians(pitch_deg)
    fwd = np.array([np.sin(yaw) * np.cos(pitch), np.sin(pitch), -np.cos(yaw) * np.cos(pitch)])
    right = np.array([np.cos(yaw), 0.0, np.sin(yaw)])
    up = np.cross(right, fwd)
    c = np.zeros(1, CAMERA_DTYPE)
    c["eye"], c["fwd"], c["right"], c["up"] = eye, fwd, right, up
    tx = np.tan(np.radians(fov_x_deg) / 2)
    c["tan_half_x"], c["tan_half_y"] = tx, tx * H / W
    return c


# ---------------------------------------------------------------- BC1 input
def bc1_encode(rgb: np.ndarray) -> bytes:
    """A simple BC1 encoder for the fixed-rate baseline (the paper's
    Background: BC1), in C (synth_bc1_encode): per 4x4 block (edges
    replicated) the endpoints are the block's darkest and brightest texels
    by luma, rounded to RGB565, ordered so that colour 0 > colour 1
    (four-colour mode; equal endpoints give an all-zero index block), and
    every texel takes the palette entry nearest in RGB.  8 bytes per block,
    row-major blocks."""
    rgb = np.ascontiguousarray(rgb, np.uint8)
    h, w = rgb.shape[:2]
    out = np.zeros(((h + 3) // 4) * ((w + 3) // 4) * 8, np.uint8)
    if lib().synth_bc1_encode(_ptr(rgb), w, h, _ptr(out)) != 0:
        raise RuntimeError("synth_bc1_encode failed")
    return out.tobytes()
