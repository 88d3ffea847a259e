"""CPU oracle for the on-demand JPEG texture path.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the GPU library.  It shares no
code with the GPU library; the only thing both sides use is the seeded input
generator module (paper_2510_08166_amd.synth), which holds none of the
decode path's arithmetic.

The C part (oracle.c) is a plain sequential baseline-JPEG decoder
(ITU-T T.81 Annex C / F.2 procedures), an fp64 IDCT by definition, colour
conversion with a single rounding, and footprint mark / resolve from fully
decoded levels.  This Python part adds the scene bookkeeping and the
frame-granular LRU simulator of the cache update.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

NEAREST, BILINEAR, TRILINEAR, BILINEAR_CLAMPED = 0, 1, 2, 3
NO_MIP = 0x100   # OR'd into a filter: every pixel samples level 0
BACKGROUND = 0xFFFFFFFF
INVALID_TEXEL = 0xFFFF00FF
# zigzag scan position -> natural index (T.81 Figure A.6), for tests that
# compare coefficient buffers kept in scan order
ZIGZAG = np.array([0, 1, 8, 16, 9, 2, 3, 10, 17, 24, 32, 25, 18, 11, 4, 5, 12, 19, 26, 33, 40, 48, 41, 34, 27,
                   20, 13, 6, 7, 14, 21, 28, 35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23, 30, 37, 44, 51, 58,
                   59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63], np.int64)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "ondemand.c"),
                               os.path.join(_HERE, "geometry.c"), os.path.join(_HERE, "bc1.c"),
                               "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build()
            L = ctypes.CDLL(_SO)
            vp, i64, u64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
            L.orc_open.restype = vp
            L.orc_open.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int)]
            L.orc_close.argtypes = [vp]
            L.orc_info.argtypes = [vp, vp]
            L.orc_quant.argtypes = [vp, vp]
            L.orc_decode_seq.argtypes = [vp, vp, vp, vp, vp]
            L.orc_decode_mcu_at.argtypes = [vp, u64, vp, vp, vp]
            L.orc_decode_stripped_mcu.argtypes = [vp, vp, u64, u64, vp, u64, ctypes.c_uint32, vp, vp]
            L.orc_decode_predicted_mcu.argtypes = [vp, vp, u64, u64, vp, u64, ctypes.c_uint32, vp, vp]
            L.orc_idct.argtypes = [vp, vp]
            L.orc_pixels.argtypes = [vp, vp, vp, vp]
            L.orc_mcu_pixels.argtypes = [vp, vp, vp, vp]
            L.orc_mcu_reduced.argtypes = [vp, vp, i32, vp, vp]
            L.orc_scene_layout.restype = u64
            L.orc_scene_layout.argtypes = [i32, vp, vp, vp]
            L.orc_mark.restype = i64
            L.orc_mark.argtypes = [i32, vp, vp, vp, vp, vp, vp, i64, i32, vp]
            L.orc_resolve.restype = i64
            L.orc_resolve.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, i64, i32, vp, vp]
            L.orc_taps.restype = i64
            L.orc_taps.argtypes = [i32, vp, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp]
            L.orc_geometry.argtypes = [vp, i64, vp, i32, i32, vp, vp, i32, vp, vp]
            L.orc_bc1_decode.argtypes = [vp, i32, i32, vp]
            L.orc_ondemand_frame.restype = i64
            L.orc_ondemand_frame.argtypes = [i32, vp, vp, i32, vp, vp, vp, u64, vp, vp, vp, vp, vp, i64, i32, vp,
                                             vp, vp, i32, vp, vp]
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


class Jpeg:
    """A parsed baseline JPEG (owns the C handle)."""

    def __init__(self, data: bytes):
        self._buf = np.frombuffer(data, np.uint8).copy()
        err = ctypes.c_int(0)
        self.h = lib().orc_open(_p(self._buf), len(self._buf), ctypes.byref(err))
        if not self.h:
            raise OracleError("orc_open failed: %d" % err.value)
        info = np.zeros(10, np.int64)
        lib().orc_info(self.h, _p(info))
        (self.width, self.height, self.sampling, self.mcu_cols, self.mcu_rows, self.n_mcu, self.n_du,
         self.ecs_bits) = (int(x) for x in info[:8])
        q = np.zeros(128, np.uint16)
        lib().orc_quant(self.h, _p(q))
        self.quant = q.reshape(2, 64)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_close(self.h)
            self.h = None

    def decode(self):
        """Sequential decode: (coef [n_mcu, n_du, 64] natural order, mcu_bit [n_mcu+1],
        pred [n_mcu, 3], dc_bits [n_mcu])."""
        coef = np.zeros((self.n_mcu, self.n_du, 64), np.int16)
        mb = np.zeros(self.n_mcu + 1, np.uint64)
        pred = np.zeros((self.n_mcu, 3), np.int32)
        dcb = np.zeros(self.n_mcu, np.uint32)
        rc = lib().orc_decode_seq(self.h, _p(coef), _p(mb), _p(pred), _p(dcb))
        if rc:
            raise OracleError("orc_decode_seq: %d" % rc)
        return coef, mb, pred, dcb

    def decode_mcu_at(self, bitpos: int, pred):
        out = np.zeros((self.n_du, 64), np.int16)
        end = ctypes.c_uint64(0)
        p = np.asarray(pred, np.int32)
        rc = lib().orc_decode_mcu_at(self.h, int(bitpos), _p(p), _p(out), ctypes.byref(end))
        return rc, out, end.value

    def decode_stripped_mcu(self, words: np.ndarray, stream_bits: int, records: np.ndarray, m: int):
        out = np.zeros((self.n_du, 64), np.int16)
        end = ctypes.c_uint64(0)
        words = np.ascontiguousarray(words, np.uint32)
        records = np.ascontiguousarray(records, np.uint8)
        rc = lib().orc_decode_stripped_mcu(self.h, _p(words), len(words), int(stream_bits), _p(records),
                                           len(records) // 64, int(m), _p(out), ctypes.byref(end))
        return rc, out, end.value

    def decode_predicted_mcu(self, words: np.ndarray, stream_bits: int, records: np.ndarray, m: int):
        out = np.zeros((self.n_du, 64), np.int16)
        end = ctypes.c_uint64(0)
        words = np.ascontiguousarray(words, np.uint32)
        records = np.ascontiguousarray(records, np.uint8)
        rc = lib().orc_decode_predicted_mcu(self.h, _p(words), len(words), int(stream_bits), _p(records),
                                            len(records) // 64, int(m), _p(out), ctypes.byref(end))
        return rc, out, end.value

    def pixels(self, coef, want_f64=False):
        coef = np.ascontiguousarray(coef, np.int16)
        rgb = np.zeros((self.height, self.width, 3), np.uint8)
        f = np.zeros((self.height, self.width, 3), np.float64) if want_f64 else None
        lib().orc_pixels(self.h, _p(coef), _p(rgb), _p(f))
        return (rgb, f) if want_f64 else rgb

    def mcu_pixels(self, coef_mcu, want_f64=False):
        ms = 16 if self.sampling == 420 else 8
        c = np.ascontiguousarray(coef_mcu, np.int16)
        rgb = np.zeros((ms, ms, 3), np.uint8)
        f = np.zeros((ms, ms, 3), np.float64) if want_f64 else None
        lib().orc_mcu_pixels(self.h, _p(c), _p(rgb), _p(f))
        return (rgb, f) if want_f64 else rgb


def mcu_reduced(j: "Jpeg", coef_mcu, scale_log2: int, want_f64=False):
    """orc_mcu_reduced: an MCU's texel tile at 1/2^scale_log2 resolution."""
    ms = (16 if j.sampling == 420 else 8) >> scale_log2
    c = np.ascontiguousarray(coef_mcu, np.int16)
    rgb = np.zeros((ms, ms, 3), np.uint8)
    f = np.zeros((ms, ms, 3), np.float64) if want_f64 else None
    if lib().orc_mcu_reduced(j.h, _p(c), int(scale_log2), _p(rgb), _p(f)) != 0:
        raise OracleError("orc_mcu_reduced: bad arguments")
    return (rgb, f) if want_f64 else rgb


def idct(F: np.ndarray) -> np.ndarray:
    F = np.ascontiguousarray(F, np.float64).reshape(64)
    out = np.zeros(64, np.float64)
    lib().orc_idct(_p(F), _p(out))
    return out.reshape(8, 8)


class Scene:
    """Textures as chains of levels, each level a JPEG; block-id layout of
    the scene (levels texture by texture, then level by level, each level's
    block range starting at a multiple of 32)."""

    def __init__(self, textures):
        self.textures = textures
        self.jpegs = []
        tex_first, tex_count, lw, lh = [], [], [], []
        for t in textures:
            tex_first.append(len(self.jpegs)); tex_count.append(len(t.jpegs))
            for data in t.jpegs:
                j = Jpeg(data)
                self.jpegs.append(j); lw.append(j.width); lh.append(j.height)
        self.tex_first = np.array(tex_first, np.int32); self.tex_count = np.array(tex_count, np.int32)
        self.lev_w = np.array(lw, np.int32); self.lev_h = np.array(lh, np.int32)
        self.blk_base = np.zeros(len(lw), np.uint32)
        self.n_blocks = int(lib().orc_scene_layout(len(lw), _p(self.lev_w), _p(self.lev_h), _p(self.blk_base)))
        self.blk_cols = (self.lev_w + 15) // 16
        self.blk_rows = (self.lev_h + 15) // 16
        self._levels = {}

    def level_of_block(self, b: int) -> int:
        return int(np.searchsorted(self.blk_base, b, side="right") - 1)

    def block_coords(self, b: int):
        L = self.level_of_block(b)
        r = b - int(self.blk_base[L])
        return L, r % int(self.blk_cols[L]), r // int(self.blk_cols[L])

    def decode_level(self, L: int, want_f64=False):
        key = (L, want_f64)
        if key not in self._levels:
            j = self.jpegs[L]
            coef, _, _, _ = j.decode()
            self._levels[key] = j.pixels(coef, want_f64)
        return self._levels[key]

    def mark(self, g: np.ndarray, filt: int):
        vis = np.zeros(self.n_blocks, np.uint8)
        g = np.ascontiguousarray(g)
        bad = lib().orc_mark(len(self.textures), _p(self.tex_first), _p(self.tex_count), _p(self.lev_w),
                             _p(self.lev_h), _p(self.blk_base), _p(g), g.size, filt, _p(vis))
        return np.nonzero(vis)[0].astype(np.uint32), int(bad)

    def taps(self, g: np.ndarray, filt: int):
        """Per pixel up to 8 taps: (level, x, y, weight) arrays of shape g.shape + (8,)."""
        g = np.ascontiguousarray(g)
        lv = np.zeros(g.shape + (8,), np.int32); x = np.zeros_like(lv); y = np.zeros_like(lv)
        w = np.zeros(g.shape + (8,), np.float64)
        bad = lib().orc_taps(len(self.textures), _p(self.tex_first), _p(self.tex_count), _p(self.lev_w),
                             _p(self.lev_h), _p(g), g.size, filt, _p(lv), _p(x), _p(y), _p(w))
        return lv, x, y, w, int(bad)

    def levels_of_blocks(self, blocks) -> set:
        return {self.level_of_block(int(b)) for b in blocks}

    def resolve(self, g: np.ndarray, filt: int, level_rgb: dict, level_f64: dict | None = None,
                want_f64=False):
        """level_rgb: {level index: (h, w, 3) uint8}; missing levels read as absent."""
        n = len(self.jpegs)
        keep = []
        ptrs = (ctypes.c_void_p * n)()
        fptrs = (ctypes.c_void_p * n)()
        for L, img in level_rgb.items():
            img = np.ascontiguousarray(img, np.uint8); keep.append(img); ptrs[L] = img.ctypes.data
        if level_f64:
            for L, img in level_f64.items():
                img = np.ascontiguousarray(img, np.float64); keep.append(img); fptrs[L] = img.ctypes.data
        g = np.ascontiguousarray(g)
        frame = np.zeros(g.shape, np.uint32)
        ff = np.zeros(g.shape + (3,), np.float64) if want_f64 else None
        bad = lib().orc_resolve(len(self.textures), _p(self.tex_first), _p(self.tex_count), _p(self.lev_w),
                                _p(self.lev_h), ctypes.cast(ptrs, ctypes.c_void_p),
                                ctypes.cast(fptrs, ctypes.c_void_p) if level_f64 else None, _p(g), g.size,
                                filt, _p(frame), _p(ff))
        return (frame, ff, int(bad)) if want_f64 else (frame, int(bad))

    def render(self, g: np.ndarray, filt: int):
        """The plain definition: the visible set, every touched level decoded
        sequentially and in full, then the filtered lookup."""
        vis, _ = self.mark(g, filt)
        levels = {L: self.decode_level(L) for L in self.levels_of_blocks(vis)}
        frame, bad = self.resolve(g, filt, levels)
        return frame, vis, bad


class OnDemand:
    """The CPU on-demand baseline over a Scene (orc_ondemand_frame): the
    per-MCU index (start bit and DC predictors of every MCU of every level)
    is recorded once by a sequential decode, outside any timing; each frame
    then marks, decodes only the MCUs of the marked blocks by random access,
    and resolves, on n threads."""

    def __init__(self, scene: Scene):
        self.s = scene
        n = len(scene.jpegs)
        self._bits, self._pred, self._img = [], [], []
        for j in scene.jpegs:
            _, mb, pred, _ = j.decode()
            self._bits.append(mb)
            self._pred.append(np.ascontiguousarray(pred.reshape(-1)))
            self._img.append(np.zeros((j.height, j.width, 3), np.uint8))
        self._jp = (ctypes.c_void_p * n)(*[j.h for j in scene.jpegs])
        self._bp = (ctypes.c_void_p * n)(*[a.ctypes.data for a in self._bits])
        self._pp = (ctypes.c_void_p * n)(*[a.ctypes.data for a in self._pred])
        self._ip = (ctypes.c_void_p * n)(*[a.ctypes.data for a in self._img])
        self._vis = np.zeros(scene.n_blocks, np.uint8)
        self._list = np.zeros(max(1, scene.n_blocks), np.uint32)

    def frame(self, g: np.ndarray, filt: int, threads: int = 1):
        """(frame u32, seconds of mark / listing / decode / resolve, blocks decoded, bad count)."""
        s = self.s
        g = np.ascontiguousarray(g)
        out = np.zeros(g.shape, np.uint32)
        times = np.zeros(4, np.float64)
        nd = ctypes.c_uint64(0)
        bad = lib().orc_ondemand_frame(len(s.textures), _p(s.tex_first), _p(s.tex_count), len(s.jpegs),
                                       _p(s.lev_w), _p(s.lev_h), _p(s.blk_base), s.n_blocks,
                                       ctypes.cast(self._jp, ctypes.c_void_p), ctypes.cast(self._bp, ctypes.c_void_p),
                                       ctypes.cast(self._pp, ctypes.c_void_p), ctypes.cast(self._ip, ctypes.c_void_p),
                                       _p(g), g.size, filt, _p(out), _p(self._vis), _p(self._list), int(threads),
                                       _p(times), ctypes.byref(nd))
        if bad < 0:
            raise OracleError("orc_ondemand_frame: bad arguments")
        return out, times, int(nd.value), int(bad)


def geometry(tris: np.ndarray, cam: np.ndarray, W: int, H: int, tex_w, tex_h, want_tri=False):
    """The geometry pass by definition (orc_geometry): tris a structured
    array of the triangle layout, cam one camera record; returns the
    G-buffer (H, W) (and the hit triangle per pixel)."""
    from paper_2510_08166_amd.synth import GPIXEL_DTYPE
    tris = np.ascontiguousarray(tris)
    cam = np.ascontiguousarray(cam)
    tw = np.ascontiguousarray(tex_w, np.int32); th = np.ascontiguousarray(tex_h, np.int32)
    g = np.zeros((H, W), GPIXEL_DTYPE)
    hit = np.zeros((H, W), np.int32)
    lib().orc_geometry(_p(tris), len(tris), _p(cam), W, H, _p(tw), _p(th), len(tw), _p(g), _p(hit))
    return (g, hit) if want_tri else g


def bc1_decode(blocks: bytes, w: int, h: int) -> np.ndarray:
    """A BC1 image by definition (orc_bc1_decode): (h, w, 3) uint8."""
    b = np.frombuffer(blocks, np.uint8)
    assert len(b) >= ((w + 3) // 4) * ((h + 3) // 4) * 8
    out = np.zeros((h, w, 3), np.uint8)
    lib().orc_bc1_decode(_p(np.ascontiguousarray(b)), w, h, _p(out))
    return out


def unpack_frame(frame: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(frame, np.uint32)
    return f.view(np.uint8).reshape(f.shape + (4,))


class LruSim:
    """Frame-granular LRU cache of decoded blocks (the paper's Update Cache
    pass, with a capacity and least-recently-used eviction instead of
    evicting every invisible block).  Per frame f with visible set V (frame
    numbers never decrease):
        new   = V - R                      (to decode)
        touch = V & R                      (last_used := f)
        if |new| > free: evict the |new| - free resident blocks not in V with
        the smallest (last_used, block id);
        R := (R - evicted) | new,  last_used[new] := f."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.last_used: dict[int, int] = {}

    def step(self, frame_no: int, visible) -> tuple[list, list]:
        V = set(int(b) for b in visible)
        R = set(self.last_used)
        new = sorted(V - R)
        for b in V & R:
            self.last_used[b] = frame_no
        free = self.capacity - len(R)
        evicted = []
        if len(new) > free:
            cand = sorted((self.last_used[b], b) for b in R - V)
            need = len(new) - free
            if need > len(cand):
                raise OracleError("visible set exceeds the cache capacity")
            evicted = sorted(b for _, b in cand[:need])
            for b in evicted:
                del self.last_used[b]
        for b in new:
            self.last_used[b] = frame_no
        return new, evicted


class EvictInvisibleSim:
    """The paper's cache update (Method: Update Cache): after each frame every
    cached block that the frame did not read is evicted; blocks read in
    consecutive frames stay and are not decoded again.  Per frame with
    visible set V: new = V - R, evicted = R - V, R := V."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.resident: set[int] = set()

    def step(self, visible) -> tuple[list, list]:
        V = set(int(b) for b in visible)
        if len(V) > self.capacity:
            raise OracleError("visible set exceeds the cache capacity")
        new = sorted(V - self.resident)
        evicted = sorted(self.resident - V)
        self.resident = V
        return new, evicted

