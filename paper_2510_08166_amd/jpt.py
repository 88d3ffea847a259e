"""Python binding of libjpt (include/jpt.h): argument marshalling only.

Every step of the per-frame path runs in the HIP kernels of libjpt.so; this
module builds the host-side descriptors, owns device memory through torch
tensors, and passes raw pointers and the current HIP stream to the C ABI.
If libjpt.so is missing the import of the library fails loudly (there is no
fallback path).
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libjpt.so")

u8, u16, u32, u64, f64, vp = (ctypes.c_uint8, ctypes.c_uint16, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                              ctypes.c_void_p)

JPT_OK, JPT_E_ARG, JPT_E_UNSUPPORTED, JPT_E_CORRUPT, JPT_E_RANGE, JPT_E_BUFSIZE, JPT_E_HIP, JPT_E_CAPACITY = \
    0, -1, -2, -3, -4, -5, -6, -7
FILTER_NEAREST, FILTER_BILINEAR, FILTER_TRILINEAR, FILTER_BILINEAR_CLAMPED = 0, 1, 2, 3
SAMPLING_420, SAMPLING_444 = 420, 444
FILTER_MIP_OFF = 0x100
CACHE_NONE, CACHE_LRU, CACHE_EVICT_INVISIBLE, CACHE_HASH = 0, 1, 2, 3
INDEX_SPLICED, INDEX_PREDICTORS = 0, 1
SCENE_PREDICTOR_INDEX = 1
IDCT_MFMA_F16, IDCT_SCALAR_F32, IDCT_FUSED_F32, IDCT_MFMA_BF16 = 0, 1, 2, 3
FRAME_AUTO = 0xFFFFFFFF
TUNE_XCD_TILES, TUNE_RESOLVE_PAIRED, TUNE_RESOLVE_SINGLE = 1, 2, 4
CTR_ITEMS, CTR_NEW, CTR_VISIBLE, CTR_ERROR, CTR_ERROR_ITEM, CTR_EVICTED, CTR_RESIDENT, CTR_GRAD_MAX = range(8)
N_COUNTERS = 16
ERR_CORRUPT, ERR_CAPACITY, ERR_PIXEL, ERR_INTERNAL, ERR_GRAD = 1, 2, 4, 8, 16
SLOT_NONE = 0xFFFFFFFF
TEXEL_INVALID = 0xFFFF00FF
ITEMS_DU = 6
ITEM_COEFS = ITEMS_DU * 64
RECORD_BYTES = 64
TABLESET_WORDS = 6656


class LevelInfo(ctypes.Structure):
    _fields_ = [("width", u32), ("height", u32), ("sampling", u32), ("mcu_cols", u32), ("mcu_rows", u32),
                ("n_mcu", u32), ("blk_cols", u32), ("blk_rows", u32), ("n_records", u32), ("stream_words", u32),
                ("stream_bits", u64), ("scan_bits", u64), ("removed_dc_bits", u64),
                ("quant", (u16 * 64) * 2), ("huff_bits", (u8 * 16) * 4), ("huff_vals", (u8 * 256) * 4),
                ("huff_nvals", u16 * 4), ("index_kind", u16), ("reserved0", u16),
                ("index_bits_per_mcu", f64), ("dc_bits_per_mcu", f64), ("overhead_bpp_bound", f64),
                ("overhead_bpp_effective", f64), ("stored_bpp", f64)]


class LevelDesc(ctypes.Structure):
    _fields_ = [("stream", u64), ("records", u64), ("stream_bits", u32), ("index_kind", u32), ("width", u32),
                ("height", u32),
                ("blk_cols", u32), ("blk_rows", u32), ("mcu_cols", u32), ("n_mcu", u32), ("blk_base", u32),
                ("sampling", u32), ("table_set", u32), ("quant", u32)]


class TextureDesc(ctypes.Structure):
    _fields_ = [("first_level", u32), ("n_levels", u32), ("width", u32), ("height", u32)]


class SceneC(ctypes.Structure):
    _fields_ = [("levels", vp), ("textures", vp), ("word_level", vp), ("tables", vp), ("quant", vp),
                ("n_levels", u32), ("n_textures", u32), ("n_tablesets", u32), ("n_quant", u32),
                ("n_blocks", u32), ("flags", u32)]


class ViewC(ctypes.Structure):
    _fields_ = [("gbuf", vp), ("frame", vp), ("width", u32), ("height", u32), ("pitch", u32),
                ("frame_pitch", u32)]


class FrameC(ctypes.Structure):
    _fields_ = [("vis", vp), ("work", vp), ("counters", vp), ("scan", vp), ("coef", vp), ("max_items", u32),
                ("frame_no", u32)]


class CacheC(ctypes.Structure):
    _fields_ = [("texels", vp), ("slot_of", vp), ("owner", vp), ("last_used", vp), ("resident", vp),
                ("free_stack", vp), ("meta", vp), ("tie_mask", vp), ("n_slots", u32), ("policy", u32),
                ("hash", vp), ("n_buckets", u32), ("reserved", u32)]


class SizesC(ctypes.Structure):
    _fields_ = [("n_blocks", u32), ("vis_words", u32), ("scan_entries", u32), ("max_items", u32),
                ("coef_entries", u64), ("max_blocks", u32), ("items_total", u32), ("texel_words", u64),
                ("pixels", u64)]


LRU_MAX_AGE = 1023
CACHE_META_WORDS = 16 + LRU_MAX_AGE + 1 + 2048 + 2048 + 1024
STATIC_SCAN_ENTRIES = 65536


class TuningC(ctypes.Structure):
    _fields_ = [("decode_groups", u32), ("idct_groups", u32), ("mark_groups", u32), ("resolve_groups", u32),
                ("flags", u32), ("wide_bits", u32), ("reserved", u32 * 2)]


assert ctypes.sizeof(LevelDesc) == 64 and ctypes.sizeof(TextureDesc) == 16
assert ctypes.sizeof(SceneC) == 64 and ctypes.sizeof(ViewC) == 32 and ctypes.sizeof(FrameC) == 48
assert ctypes.sizeof(CacheC) == 88 and ctypes.sizeof(LevelInfo) == 1464 and ctypes.sizeof(SizesC) == 48

# name -> (restype, argtypes) of every function the header declares
SIGNATURES = {
    "jpt_build_index": (ctypes.c_int32, [vp, ctypes.c_size_t, vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t]),
    "jpt_build_index_ex": (ctypes.c_int32, [vp, ctypes.c_size_t, u32, vp, vp, ctypes.c_size_t, vp,
                                            ctypes.c_size_t]),
    "jpt_build_tables": (ctypes.c_int32, [vp, vp, ctypes.c_size_t, vp]),
    "jpt_layout": (ctypes.c_int32, [vp, u32, vp, vp, ctypes.c_size_t, vp]),
    "jpt_make_level_desc": (ctypes.c_int32, [vp, u64, u64, u32, u32, u32, vp]),
    "jpt_scan_entries": (u32, [u32]),
    "jpt_query_sizes": (ctypes.c_int32, [vp, u32, vp, u32, u32, vp]),
    "jpt_mark_blocks": (ctypes.c_int32, [vp, vp, u32, u32, vp, vp, vp, vp]),
    "jpt_mark_blocks_static": (ctypes.c_int32, [vp, vp, u32, u32, vp, vp, vp, vp]),
    "jpt_decode_blocks": (ctypes.c_int32, [vp, vp, vp, u32, vp, vp]),
    "jpt_entropy_decode": (ctypes.c_int32, [vp, vp, vp, vp]),
    "jpt_decode_reduced": (ctypes.c_int32, [vp, vp, u32, vp, vp, vp]),
    "jpt_idct_color": (ctypes.c_int32, [vp, vp, vp, u32, vp, vp]),
    "jpt_resolve": (ctypes.c_int32, [vp, vp, u32, u32, vp, vp, vp, vp]),
    "jpt_cache_reset": (ctypes.c_int32, [vp, vp, vp]),
    "jpt_graph_capture": (ctypes.c_int32, [vp, vp, u32, u32, vp, vp, u32, vp, vp, ctypes.POINTER(vp)]),
    "jpt_graph_launch": (ctypes.c_int32, [vp, vp]),
    "jpt_graph_destroy": (ctypes.c_int32, [vp]),
    "jpt_dequantize": (ctypes.c_int32, [vp, vp, vp, u32, vp]),
    "jpt_fwd_float": (ctypes.c_int32, [vp, vp, u32, u32, vp, vp, vp, u32, vp, vp, vp]),
    "jpt_backward": (ctypes.c_int32, [vp, vp, u32, u32, vp, vp, vp, vp, vp, u32, vp]),
    "jpt_geometry_pass": (ctypes.c_int32, [vp, vp, u32, vp, u32, u32, u32, vp, vp]),
    "jpt_bc1_resolve": (ctypes.c_int32, [vp, vp, u32, u32, vp]),
    "jpt_version": (u32, []),
    "jpt_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
}

_lib = None


class JptError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__("%s failed: %d (%s)" % (fn, status, lib().jpt_status_string(status).decode()))


def lib():
    """Load libjpt.so (built in-tree by __graft_entry__.build()).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libjpt.so not built at %s: run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(fn, st):
    if st != JPT_OK:
        raise JptError(fn, st)


def _np_ptr(a):
    return a.ctypes.data_as(vp)


# ------------------------------------------------------------- host side
class LevelIndex:
    """Result of jpt_build_index for one level (host arrays)."""

    def __init__(self, info: LevelInfo, stream: np.ndarray, records: np.ndarray):
        self.info, self.stream, self.records = info, stream, records


def build_index(jpeg: bytes, kind: int = INDEX_SPLICED) -> LevelIndex:
    buf = np.frombuffer(jpeg, np.uint8)
    info = LevelInfo()
    L = lib()
    _check("jpt_build_index_ex", L.jpt_build_index_ex(_np_ptr(buf), len(buf), kind, ctypes.byref(info), None, 0,
                                                      None, 0))
    stream = np.zeros(info.stream_words, np.uint32)
    records = np.zeros(info.n_records * RECORD_BYTES, np.uint8)
    _check("jpt_build_index_ex", L.jpt_build_index_ex(_np_ptr(buf), len(buf), kind, ctypes.byref(info),
                                                      _np_ptr(stream), len(stream), _np_ptr(records), len(records)))
    return LevelIndex(info, stream, records)


def build_tables(info: LevelInfo) -> np.ndarray:
    out = np.zeros(TABLESET_WORDS, np.uint32)
    n = ctypes.c_size_t(0)
    _check("jpt_build_tables", lib().jpt_build_tables(ctypes.byref(info), _np_ptr(out), len(out), ctypes.byref(n)))
    return out


def layout(infos: list[LevelInfo]):
    arr = (LevelInfo * len(infos))(*infos)
    base = np.zeros(len(infos), np.uint32)
    nb = u32(0)
    L = lib()
    _check("jpt_layout", L.jpt_layout(arr, len(infos), _np_ptr(base), None, 0, ctypes.byref(nb)))
    wl = np.zeros(max(1, nb.value // 32), np.uint32)
    _check("jpt_layout", L.jpt_layout(arr, len(infos), _np_ptr(base), _np_ptr(wl), len(wl), ctypes.byref(nb)))
    return base, wl, nb.value


def query_sizes(infos: list[LevelInfo], view_sizes, filt: int) -> SizesC:
    """jpt_query_sizes for a scene's level infos and views given as
    (width, height) pairs."""
    arr = (LevelInfo * len(infos))(*infos)
    vs = (ViewC * max(1, len(view_sizes)))()
    for i, (w, h) in enumerate(view_sizes):
        vs[i] = ViewC(None, None, w, h, w, w)
    out = SizesC()
    _check("jpt_query_sizes", lib().jpt_query_sizes(arr, len(infos), vs, len(view_sizes), filt, ctypes.byref(out)))
    return out


def _table_key(info: LevelInfo) -> bytes:
    return bytes(info.huff_bits) + bytes(info.huff_vals) + bytes(info.huff_nvals)


class HostScene:
    """Index build and descriptors of a texture set (no device memory)."""

    def __init__(self, textures, threads: int | None = None, index_kind: int = INDEX_SPLICED):
        self.textures = textures
        self.index_kind = index_kind
        jpegs, tex_first, tex_count = [], [], []
        for t in textures:
            tex_first.append(len(jpegs)); tex_count.append(len(t.jpegs))
            jpegs.extend(t.jpegs)
        threads = threads or min(16, os.cpu_count() or 1)
        with ThreadPoolExecutor(threads) as ex:
            self.levels = list(ex.map(lambda j: build_index(j, index_kind), jpegs))
        self.tex_first = tex_first; self.tex_count = tex_count
        infos = [l.info for l in self.levels]
        self.blk_base, self.word_level, self.n_blocks = layout(infos)
        # deduplicate Huffman table sets and quant tables by content
        self.tablesets, ts_index, self.level_ts = [], {}, []
        self.quants, q_index, self.level_q = [], {}, []
        for inf in infos:
            k = _table_key(inf)
            if k not in ts_index:
                ts_index[k] = len(self.tablesets); self.tablesets.append(build_tables(inf))
            self.level_ts.append(ts_index[k])
            qk = bytes(inf.quant)
            if qk not in q_index:
                q_index[qk] = len(self.quants)
                self.quants.append(np.frombuffer(qk, np.uint16).copy())
            self.level_q.append(q_index[qk])
        # stream / record pools (offsets in bytes, 256-byte aligned)
        self.stream_off, self.record_off = [], []
        so = ro = 0
        for l in self.levels:
            self.stream_off.append(so); so += (l.stream.nbytes + 255) // 256 * 256
            self.record_off.append(ro); ro += (l.records.nbytes + 255) // 256 * 256
        self.stream_bytes, self.record_bytes = max(so, 256), max(ro, 256)
        self.n_items_total = int(sum(l.info.blk_cols * l.info.blk_rows * (4 if l.info.sampling == 444 else 1)
                                     for l in self.levels))

    def stream_pool(self) -> np.ndarray:
        pool = np.zeros(self.stream_bytes, np.uint8)
        for l, o in zip(self.levels, self.stream_off):
            pool[o:o + l.stream.nbytes] = l.stream.view(np.uint8)
        return pool

    def record_pool(self) -> np.ndarray:
        pool = np.zeros(self.record_bytes, np.uint8)
        for l, o in zip(self.levels, self.record_off):
            pool[o:o + l.records.nbytes] = l.records
        return pool

    def level_descs(self, stream_base: int, record_base: int) -> bytes:
        arr = (LevelDesc * len(self.levels))()
        L = lib()
        for i, l in enumerate(self.levels):
            _check("jpt_make_level_desc", L.jpt_make_level_desc(
                ctypes.byref(l.info), stream_base + self.stream_off[i], record_base + self.record_off[i],
                int(self.blk_base[i]), self.level_ts[i], self.level_q[i], ctypes.byref(arr[i])))
        return bytes(arr)

    def texture_descs(self) -> bytes:
        arr = (TextureDesc * len(self.textures))()
        for i in range(len(self.textures)):
            f = self.tex_first[i]
            arr[i] = TextureDesc(f, self.tex_count[i], self.levels[f].info.width, self.levels[f].info.height)
        return bytes(arr)

    def overhead(self):
        """(paper-accounting bpp bound, effective bpp, stored bpp) over all
        levels: the library's per-level figures (jpt_level_info), weighted by
        the texels they are per (MCU texels for the first two, image texels
        for the stored size)."""
        mcu_px = [l.info.n_mcu * (256 if l.info.sampling == SAMPLING_420 else 64) for l in self.levels]
        px = [l.info.width * l.info.height for l in self.levels]
        bound = sum(l.info.overhead_bpp_bound * m for l, m in zip(self.levels, mcu_px)) / sum(mcu_px)
        eff = sum(l.info.overhead_bpp_effective * m for l, m in zip(self.levels, mcu_px)) / sum(mcu_px)
        stored = sum(l.info.stored_bpp * p for l, p in zip(self.levels, px)) / sum(px)
        return bound, eff, stored


# ----------------------------------------------------------- device side
def _torch():
    import torch
    return torch


def _dev_bytes(data: bytes | np.ndarray, device):
    torch = _torch()
    a = np.frombuffer(data, np.uint8) if isinstance(data, (bytes, bytearray)) else data.view(np.uint8).ravel()
    t = torch.empty(max(len(a), 1), dtype=torch.uint8, device=device)
    if len(a):
        t[: len(a)].copy_(torch.from_numpy(a.copy()))
    return t


class DeviceScene:
    """Compressed textures resident in HBM plus their descriptors."""

    def __init__(self, host: HostScene, device="cuda"):
        torch = _torch()
        self.host = host
        self.device = torch.device(device)
        self.streams = _dev_bytes(host.stream_pool(), device)
        self.records = _dev_bytes(host.record_pool(), device)
        self.levels_t = _dev_bytes(host.level_descs(self.streams.data_ptr(), self.records.data_ptr()), device)
        self.textures_t = _dev_bytes(host.texture_descs(), device)
        self.word_level_t = _dev_bytes(host.word_level, device)
        self.tables_t = _dev_bytes(np.concatenate(host.tablesets), device)
        self.quant_t = _dev_bytes(np.concatenate(host.quants), device)
        self.c = SceneC(self.levels_t.data_ptr(), self.textures_t.data_ptr(), self.word_level_t.data_ptr(),
                        self.tables_t.data_ptr(), self.quant_t.data_ptr(), len(host.levels), len(host.textures),
                        len(host.tablesets), len(host.quants), host.n_blocks,
                        SCENE_PREDICTOR_INDEX if any(l.info.index_kind == INDEX_PREDICTORS for l in host.levels)
                        else 0)
        self.n_blocks = host.n_blocks

    def compressed_bytes(self) -> int:
        return sum(l.stream.nbytes + l.records.nbytes for l in self.host.levels)


class Frame:
    """Per-frame device scratch: visibility bitmask, work list, counters, scan, coefficients."""

    def __init__(self, scene: DeviceScene, max_items: int):
        torch = _torch()
        d = scene.device
        n_words = scene.n_blocks // 32
        self.vis = torch.zeros(n_words, dtype=torch.int32, device=d)
        self.work = torch.zeros(max(1, max_items), dtype=torch.int32, device=d)
        self.counters = torch.zeros(N_COUNTERS, dtype=torch.int32, device=d)
        self.scan = torch.zeros(int(lib().jpt_scan_entries(scene.n_blocks)), dtype=torch.int64, device=d)
        self.coef = torch.zeros(max(1, max_items) * ITEM_COEFS, dtype=torch.int16, device=d)
        self.c = FrameC(self.vis.data_ptr(), self.work.data_ptr(), self.counters.data_ptr(), self.scan.data_ptr(),
                        self.coef.data_ptr(), max_items, 0)

    def counters_host(self) -> np.ndarray:
        return self.counters.cpu().numpy().view(np.uint32)

    def work_items(self) -> np.ndarray:
        n = int(self.counters_host()[CTR_ITEMS])
        return self.work[:n].cpu().numpy().view(np.uint32)


class Cache:
    """Decoded-block cache: slots of 16x16 RGBA8 texels and the block -> slot table."""

    def __init__(self, scene: DeviceScene, n_slots: int, policy: int = CACHE_NONE, stream=None):
        torch = _torch()
        d = scene.device
        self.texels = torch.zeros(max(1, n_slots) * 256, dtype=torch.int32, device=d)
        self.slot_of = torch.full((scene.n_blocks,), -1, dtype=torch.int32, device=d)
        self.n_slots = n_slots
        self.policy = policy
        if policy in (CACHE_LRU, CACHE_EVICT_INVISIBLE):
            n_words = scene.n_blocks // 32
            self.owner = torch.empty(n_slots, dtype=torch.int32, device=d)
            self.last_used = torch.empty(n_slots, dtype=torch.int32, device=d)
            self.free_stack = torch.empty(n_slots, dtype=torch.int32, device=d)
            self.resident = torch.empty(n_words, dtype=torch.int32, device=d)
            self.tie_mask = torch.empty(n_words, dtype=torch.int32, device=d)
            self.meta = torch.empty(CACHE_META_WORDS, dtype=torch.int32, device=d)
            self.c = CacheC(self.texels.data_ptr(), self.slot_of.data_ptr(), self.owner.data_ptr(),
                            self.last_used.data_ptr(), self.resident.data_ptr(), self.free_stack.data_ptr(),
                            self.meta.data_ptr(), self.tie_mask.data_ptr(), n_slots, policy, None, 0, 0)
            self.reset(scene, stream)
        elif policy == CACHE_HASH:
            nb = 1 << max(4, (2 * n_slots - 1).bit_length())
            self.owner = torch.empty(n_slots, dtype=torch.int32, device=d)
            self.free_stack = torch.empty(n_slots, dtype=torch.int32, device=d)
            self.meta = torch.empty(CACHE_META_WORDS, dtype=torch.int32, device=d)
            self.hash = torch.empty(2 * nb, dtype=torch.int32, device=d)
            self.c = CacheC(self.texels.data_ptr(), self.slot_of.data_ptr(), self.owner.data_ptr(), None, None,
                            self.free_stack.data_ptr(), self.meta.data_ptr(), None, n_slots, policy,
                            self.hash.data_ptr(), nb, 0)
            self.reset(scene, stream)
        else:
            self.c = CacheC(self.texels.data_ptr(), self.slot_of.data_ptr(), None, None, None, None, None, None,
                            n_slots, policy, None, 0, 0)

    def reset(self, scene: DeviceScene, stream=None):
        _check("jpt_cache_reset", lib().jpt_cache_reset(ctypes.byref(scene.c), ctypes.byref(self.c),
                                                        stream if stream is not None else current_stream()))

    def hash_entries(self) -> dict:
        """JPT_CACHE_HASH: {key: slot} of the map's entries (host copy)."""
        h = self.hash.cpu().numpy().view(np.uint32).reshape(-1, 2)
        live = h[:, 0] != 0xFFFFFFFF
        return {int(k): int(v) & 0x7FFFFFFF for k, v in h[live]}

    def resident_blocks(self) -> np.ndarray:
        m = self.resident.cpu().numpy().view(np.uint32)
        return np.nonzero(np.unpackbits(m.view(np.uint8), bitorder="little"))[0].astype(np.uint32)


class Views:
    """G-buffers and framebuffers of one or more views."""

    def __init__(self, gbufs, device="cuda"):
        torch = _torch()
        self.gbufs, self.frames = [], []
        arr = (ViewC * len(gbufs))()
        for i, g in enumerate(gbufs):
            H, W = g.shape
            gt = torch.from_numpy(np.ascontiguousarray(g).view(np.int32).reshape(H, W, 4).copy()).to(device)
            ft = torch.zeros((H, W), dtype=torch.int32, device=device)
            self.gbufs.append(gt); self.frames.append(ft)
            arr[i] = ViewC(gt.data_ptr(), ft.data_ptr(), W, H, W, W)
        self.c = arr
        self.n = len(gbufs)
        self.n_pixels = sum(g.shape[0] * g.shape[1] for g in gbufs)

    def frame_host(self, i=0) -> np.ndarray:
        return self.frames[i].cpu().numpy().view(np.uint32)

    def view(self, i) -> "Views":
        """View i alone, sharing its device buffers."""
        v = Views.__new__(Views)
        v.gbufs, v.frames = [self.gbufs[i]], [self.frames[i]]
        v.c = (ViewC * 1)(self.c[i])
        v.n = 1
        H, W = self.frames[i].shape
        v.n_pixels = H * W
        return v


def current_stream():
    return vp(_torch().cuda.current_stream().cuda_stream)


def mark_blocks(scene: DeviceScene, views: Views, filt: int, frame: Frame, cache: Cache | None, tuning=None,
                stream=None):
    _check("jpt_mark_blocks", lib().jpt_mark_blocks(
        ctypes.byref(scene.c), views.c, views.n, filt, ctypes.byref(frame.c),
        ctypes.byref(cache.c) if cache is not None else None, ctypes.byref(tuning) if tuning else None,
        stream if stream is not None else current_stream()))


def mark_blocks_static(scene: DeviceScene, views: Views, filt: int, frame: Frame, cache: Cache | None, tuning=None,
                       stream=None):
    """jpt_mark_blocks_static: mark_blocks with the library's own scan scratch (frame.scan unused)."""
    _check("jpt_mark_blocks_static", lib().jpt_mark_blocks_static(
        ctypes.byref(scene.c), views.c, views.n, filt, ctypes.byref(frame.c),
        ctypes.byref(cache.c) if cache is not None else None, ctypes.byref(tuning) if tuning else None,
        stream if stream is not None else current_stream()))


def entropy_decode(scene: DeviceScene, frame: Frame, tuning=None, stream=None):
    _check("jpt_entropy_decode", lib().jpt_entropy_decode(
        ctypes.byref(scene.c), ctypes.byref(frame.c), ctypes.byref(tuning) if tuning else None,
        stream if stream is not None else current_stream()))


def decode_blocks(scene: DeviceScene, frame: Frame, cache: Cache, idct_mode: int = IDCT_MFMA_F16, tuning=None,
                  stream=None):
    _check("jpt_decode_blocks", lib().jpt_decode_blocks(
        ctypes.byref(scene.c), ctypes.byref(frame.c), ctypes.byref(cache.c), idct_mode,
        ctypes.byref(tuning) if tuning else None, stream if stream is not None else current_stream()))


def decode_reduced(scene: DeviceScene, frame: Frame, scale_log2: int, out, tuning=None, stream=None):
    """jpt_decode_reduced into `out` (a device tensor of at least
    items x (16 >> scale_log2)^2 int32)."""
    _check("jpt_decode_reduced", lib().jpt_decode_reduced(
        ctypes.byref(scene.c), ctypes.byref(frame.c), scale_log2, vp(out.data_ptr()),
        ctypes.byref(tuning) if tuning else None, stream if stream is not None else current_stream()))


def idct_color(scene: DeviceScene, frame: Frame, cache: Cache, idct_mode: int = IDCT_MFMA_F16, tuning=None,
               stream=None):
    _check("jpt_idct_color", lib().jpt_idct_color(
        ctypes.byref(scene.c), ctypes.byref(frame.c), ctypes.byref(cache.c), idct_mode,
        ctypes.byref(tuning) if tuning else None, stream if stream is not None else current_stream()))


def resolve(scene: DeviceScene, views: Views, filt: int, frame: Frame, cache: Cache, tuning=None, stream=None):
    _check("jpt_resolve", lib().jpt_resolve(
        ctypes.byref(scene.c), views.c, views.n, filt, ctypes.byref(frame.c), ctypes.byref(cache.c),
        ctypes.byref(tuning) if tuning else None, stream if stream is not None else current_stream()))


def geometry_pass(scene: DeviceScene, tris, cam, views: "Views", i: int = 0, stream=None):
    """jpt_geometry_pass into view i's G-buffer.  tris: a device tensor
    holding the triangles (synth.TRIANGLE_DTYPE records); cam: one camera
    record (synth.CAMERA_DTYPE)."""
    H, W = views.frames[i].shape
    cam = np.ascontiguousarray(cam)
    n = tris.numel() // 80
    _check("jpt_geometry_pass", lib().jpt_geometry_pass(
        ctypes.byref(scene.c), vp(tris.data_ptr()) if n else None, n, cam.ctypes.data_as(vp), W, H, W,
        vp(views.gbufs[i].data_ptr()), stream if stream is not None else current_stream()))


class Bc1Level(ctypes.Structure):
    _fields_ = [("blocks", vp), ("width", u32), ("height", u32), ("blocks_per_row", u32), ("reserved", u32)]


class Bc1SceneC(ctypes.Structure):
    _fields_ = [("levels", vp), ("textures", vp), ("n_levels", u32), ("n_textures", u32)]


assert ctypes.sizeof(Bc1Level) == 24 and ctypes.sizeof(Bc1SceneC) == 24


class Bc1Scene:
    """BC1 textures resident in HBM (the fixed-rate baseline).  textures:
    per texture a list of levels (level 0 first), each (blocks, width,
    height) with `blocks` the level's BC1 bytes."""

    def __init__(self, textures, device="cuda"):
        blobs, dims, tex = [], [], []
        for levels in textures:
            tex.append((len(dims), len(levels), levels[0][1], levels[0][2]))
            for blk, w, h in levels:
                assert len(blk) >= ((w + 3) // 4) * ((h + 3) // 4) * 8
                blobs.append(blk)
                dims.append((w, h))
        offs, o = [], 0
        for b in blobs:
            offs.append(o)
            o += (len(b) + 255) // 256 * 256
        pool = np.zeros(max(o, 256), np.uint8)
        for b, off in zip(blobs, offs):
            pool[off:off + len(b)] = np.frombuffer(b, np.uint8)
        self.pool = _dev_bytes(pool, device)
        lv = (Bc1Level * len(dims))()
        for i, ((w, h), off) in enumerate(zip(dims, offs)):
            lv[i] = Bc1Level(self.pool.data_ptr() + off, w, h, (w + 3) // 4, 0)
        self.levels_t = _dev_bytes(bytes(lv), device)
        td = (TextureDesc * len(tex))(*[TextureDesc(*t) for t in tex])
        self.textures_t = _dev_bytes(bytes(td), device)
        self.c = Bc1SceneC(self.levels_t.data_ptr(), self.textures_t.data_ptr(), len(dims), len(tex))
        self.bytes = sum(len(b) for b in blobs)


def bc1_resolve(scene: Bc1Scene, views: "Views", filt: int, stream=None):
    _check("jpt_bc1_resolve", lib().jpt_bc1_resolve(ctypes.byref(scene.c), views.c, views.n, filt,
                                                    stream if stream is not None else current_stream()))


class Renderer:
    """One frame of the plain form: mark -> decode -> resolve on the current
    stream, over one or more views.  `tuning` (TuningC or None) holds launch
    knobs; `frame_no = FRAME_AUTO` lets an LRU cache count frames itself."""

    def __init__(self, textures, gbufs, filt, device="cuda", max_items=None, n_slots=None, host=None,
                 policy=CACHE_NONE, tuning=None, idct_mode=IDCT_MFMA_F16):
        self.host = host or HostScene(textures)
        self.scene = DeviceScene(self.host, device)
        self.views = Views(gbufs, device)
        self.filter = filt
        self.sizes = query_sizes([l.info for l in self.host.levels], [(g.shape[1], g.shape[0]) for g in gbufs],
                                 filt)
        self.max_items = int(max_items or max(1, self.sizes.max_items))
        self.frame = Frame(self.scene, self.max_items)
        self.cache = Cache(self.scene, int(n_slots or max(1, self.sizes.max_blocks)), policy)
        self.frame_no = 0
        self.tuning = tuning
        self.idct_mode = idct_mode

    def set_views(self, gbufs):
        """Load new G-buffers (same sizes) into the existing view buffers."""
        torch = _torch()
        for gt, g in zip(self.views.gbufs, gbufs):
            H, W = g.shape
            gt.copy_(torch.from_numpy(np.ascontiguousarray(g).view(np.int32).reshape(H, W, 4).copy()))

    def mark(self, stream=None):
        self.frame.c.frame_no = self.frame_no
        mark_blocks(self.scene, self.views, self.filter, self.frame, self.cache, self.tuning, stream=stream)
        if self.frame_no != FRAME_AUTO:
            self.frame_no += 1

    def decode(self, stream=None, idct_mode=None):
        decode_blocks(self.scene, self.frame, self.cache, self.idct_mode if idct_mode is None else idct_mode,
                      self.tuning, stream=stream)

    def resolve(self, stream=None):
        resolve(self.scene, self.views, self.filter, self.frame, self.cache, self.tuning, stream=stream)

    def render(self, stream=None):
        self.mark(stream)
        self.decode(stream)
        self.resolve(stream)

    def capture(self, stream, views: "Views | None" = None):
        """The batched form: capture one frame of every view (the renderer's,
        or `views`) into a HIP graph (jpt_graph_capture) on `stream`, a
        torch.cuda.Stream other than the default one.  With an LRU cache the
        renderer switches to FRAME_AUTO."""
        if self.cache.policy in (CACHE_LRU, CACHE_EVICT_INVISIBLE):
            self.frame_no = FRAME_AUTO
        self.frame.c.frame_no = self.frame_no
        return Graph(self, stream, views or self.views)


class Graph:
    """A captured frame (jpt_graph); launch() replays it on its stream."""

    def __init__(self, r: Renderer, stream, views: Views):
        self.r = r
        self.views = views
        self.stream = stream
        h = vp()
        _check("jpt_graph_capture", lib().jpt_graph_capture(
            ctypes.byref(r.scene.c), views.c, views.n, r.filter, ctypes.byref(r.frame.c), ctypes.byref(r.cache.c),
            r.idct_mode, ctypes.byref(r.tuning) if r.tuning else None, vp(stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def launch(self):
        _check("jpt_graph_launch", lib().jpt_graph_launch(self.h, vp(self.stream.cuda_stream)))

    def close(self):
        if self.h:
            lib().jpt_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DiffFrame:
    """Differentiable form over a Renderer's current frame.

    After mark + decode, the leaf is F = the dequantised coefficients of this
    frame's work items ([n_items, 6, 64] float32, natural order); forward()
    maps F to the float frame ([n_pixels of all views, 3]) with the rounding
    and clamping of the 8-bit path removed, backward() applies the
    hand-written adjoint.  Needs JPT_CACHE_NONE, so that every block the
    views read is a work item of the frame."""

    def __init__(self, r: "Renderer"):
        if r.cache.policy != CACHE_NONE:
            raise ValueError("the differentiable form needs a frame-local cache (JPT_CACHE_NONE)")
        self.r = r
        self.texel_f = self.dtexel = None
        self.n_pixels = r.views.n_pixels

    def _scratch(self):
        """Float texels and texel adjoints for the frame's new blocks (their
        slots are 0 .. counters[CTR_NEW] - 1 in a frame-local cache)."""
        torch = _torch()
        n = max(1, min(int(self.r.frame.counters_host()[CTR_NEW]), self.r.cache.n_slots))
        if self.texel_f is None or self.texel_f.numel() < n * 768:
            d = self.r.scene.device
            self.texel_f = torch.empty(n * 768, dtype=torch.float32, device=d)
            self.dtexel = torch.empty(n * 768, dtype=torch.int64, device=d)

    def n_items(self) -> int:
        return int(self.r.frame.counters_host()[CTR_ITEMS])

    def dequantize(self, stream=None):
        torch = _torch()
        self._scratch()
        F = torch.empty((self.n_items(), ITEMS_DU, 64), dtype=torch.float32, device=self.r.scene.device)
        if F.numel():
            _check("jpt_dequantize", lib().jpt_dequantize(ctypes.byref(self.r.scene.c), ctypes.byref(self.r.frame.c),
                                                          vp(F.data_ptr()), F.shape[0], stream or current_stream()))
        return F

    def forward(self, F, stream=None):
        torch = _torch()
        if self.texel_f is None:
            self._scratch()
        F = F.contiguous()
        self._check_F(F)
        frame_f = torch.empty((self.n_pixels, 3), dtype=torch.float32, device=F.device)
        r = self.r
        _check("jpt_fwd_float", lib().jpt_fwd_float(
            ctypes.byref(r.scene.c), r.views.c, r.views.n, r.filter, ctypes.byref(r.frame.c), ctypes.byref(r.cache.c),
            vp(F.data_ptr()), F.shape[0], vp(self.texel_f.data_ptr()), vp(frame_f.data_ptr()),
            stream or current_stream()))
        return frame_f

    def backward(self, dframe, F_shape, stream=None):
        torch = _torch()
        if self.dtexel is None:
            self._scratch()
        dframe = dframe.contiguous().float()
        if tuple(dframe.shape) != (self.n_pixels, 3):
            raise ValueError("dframe shape %s" % (tuple(dframe.shape),))
        dF = torch.empty(F_shape, dtype=torch.float32, device=dframe.device)
        r = self.r
        _check("jpt_backward", lib().jpt_backward(
            ctypes.byref(r.scene.c), r.views.c, r.views.n, r.filter, ctypes.byref(r.frame.c), ctypes.byref(r.cache.c),
            vp(dframe.data_ptr()), vp(self.dtexel.data_ptr()), vp(dF.data_ptr()), F_shape[0],
            stream or current_stream()))
        return dF

    def _check_F(self, F):
        torch = _torch()
        if F.dtype != torch.float32 or F.dim() != 3 or F.shape[1:] != (ITEMS_DU, 64):
            raise ValueError("F must be float32 [n_items, 6, 64]")
        if F.shape[0] > self.r.max_items:
            raise ValueError("more items than the frame holds")

    def __call__(self, F):
        return _diff_fn().apply(F, self)


_DIFF_FN = None


def _diff_fn():
    """torch.autograd.Function whose forward and backward are jpt_fwd_float
    and jpt_backward."""
    global _DIFF_FN
    if _DIFF_FN is None:
        torch = _torch()

        class DiffResolve(torch.autograd.Function):
            @staticmethod
            def forward(ctx, F, diff):
                ctx.diff = diff
                ctx.F_shape = tuple(F.shape)
                return diff.forward(F.detach())

            @staticmethod
            def backward(ctx, dframe):
                return ctx.diff.backward(dframe, ctx.F_shape), None

        _DIFF_FN = DiffResolve
    return _DIFF_FN
