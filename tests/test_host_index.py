"""Host side of libjpt (no GPU): the per-level index of the paper's
Implementation details ("Indexing Table", "Memory Overhead") checked
against the independent oracle, its overhead accounting against the
paper's closed forms, and its error paths."""
import ctypes
import io
import re

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st
from PIL import Image

import oracle
from paper_2510_08166_amd import jpt, synth
from paper_2510_08166_amd.synth import configs


def stripped_equals_sequential(data):
    li = jpt.build_index(data)
    j = oracle.Jpeg(data)
    coef, mb, pred, dcb = j.decode()
    inf = li.info
    assert (inf.width, inf.height, inf.n_mcu) == (j.width, j.height, j.n_mcu)
    assert inf.scan_bits == mb[-1]
    assert inf.removed_dc_bits == int(dcb.sum())
    assert inf.stream_bits == mb[-1] - dcb.sum()
    ends = []
    for m in range(j.n_mcu):
        rc, out, end = j.decode_stripped_mcu(li.stream, inf.stream_bits, li.records, m)
        assert rc == 0 and np.array_equal(out, coef[m]), m
        ends.append(end)
    # MCU spans tile the spliced stream exactly
    assert ends[-1] == inf.stream_bits
    return li


@pytest.mark.parametrize("smp", [420, 444])
@pytest.mark.parametrize("q", [5, 40, 75, 95, 100])
def test_index_random_access_matches_sequential(smp, q):
    rgb = synth.texture(q * 7 + smp, 136, 88)
    stripped_equals_sequential(synth.encode(rgb, q, smp))


@pytest.mark.parametrize("sub", [0, 2])
def test_index_on_pil_files(sub):
    rgb = synth.texture(77, 120, 72)
    b = io.BytesIO()
    Image.fromarray(rgb).save(b, format="JPEG", quality=85, subsampling=sub, optimize=False)
    stripped_equals_sequential(b.getvalue())
    b = io.BytesIO()
    Image.fromarray(rgb).save(b, format="JPEG", quality=85, subsampling=sub, optimize=True)  # custom Huffman tables
    stripped_equals_sequential(b.getvalue())


@settings(max_examples=30, deadline=None)
@given(st.integers(1, 70), st.integers(1, 70), st.integers(1, 100), st.sampled_from([420, 444]),
       st.integers(0, 2**32))
def test_index_property_random_images(w, h, q, smp, seed):
    stripped_equals_sequential(synth.encode(synth.texture(seed, w, h), q, smp))


def test_tiny_config_index():
    wl = configs.tiny()
    li = stripped_equals_sequential(wl.textures[0].jpegs[0])
    assert li.info.n_mcu == 256 and li.info.n_records == 29


def test_overhead_closed_forms():
    """(32 + 16*8)/9 = 17.78 bit index + 3*12 = 36 bit DCs = 53.78 bit per MCU = 0.21 bpp."""
    li = jpt.build_index(synth.encode(synth.texture(1, 64, 64), 75, 420))
    inf = li.info
    assert abs(inf.index_bits_per_mcu - 17.7777777) < 1e-6
    assert inf.dc_bits_per_mcu == 36.0
    assert abs(inf.overhead_bpp_bound - 53.7777777 / 256) < 1e-9
    assert round(inf.overhead_bpp_bound, 2) == 0.21
    assert inf.overhead_bpp_effective < inf.overhead_bpp_bound


def test_effective_overhead_falls_with_quality():
    """Higher quality spends more bits on the removed DC codes, so the
    effective overhead drops (memory-overhead results of the evaluation)."""
    rgb = synth.texture(4, 256, 256)
    eff = [jpt.build_index(synth.encode(rgb, q, 420)).info.overhead_bpp_effective for q in (30, 50, 70, 90)]
    assert all(a > b for a, b in zip(eff, eff[1:]))
    assert all(0.0 < e < 0.2101 for e in eff)


def test_layout_and_tables():
    tex = synth.make_textures([(1, 100, 60, 75, 420, 3), (2, 64, 64, 50, 444, 2)])
    hs = jpt.HostScene(tex)
    assert np.all(hs.blk_base % 32 == 0) and hs.n_blocks % 32 == 0
    for L, l in enumerate(hs.levels):
        w0, w1 = hs.blk_base[L] // 32, (hs.blk_base[L] + l.info.blk_cols * l.info.blk_rows + 31) // 32
        assert np.all(hs.word_level[w0:w1] == L)
    osc = oracle.Scene(tex)
    assert np.array_equal(osc.blk_base, hs.blk_base) and osc.n_blocks == hs.n_blocks
    assert len(hs.tablesets) == 1          # both textures use the Annex K Huffman tables
    assert len(hs.quants) == 2


def test_build_tables_cover_the_short_codes():
    """Kraft count: the 10-bit prefixes resolved by the fast table are exactly
    sum over lengths l <= 10 of (codes of length l) * 2^(10-l), for the
    standard tables and for PIL's optimised ones."""
    b = io.BytesIO()
    Image.fromarray(synth.texture(5, 64, 64)).save(b, format="JPEG", quality=90, optimize=True)
    for data in (synth.encode(synth.texture(3, 32, 32), 75, 420), b.getvalue()):
        inf = jpt.build_index(data).info
        tab = jpt.build_tables(inf)
        for t in range(4):
            bits = np.frombuffer(bytes(inf.huff_bits[t]), np.uint8).astype(int)
            want = sum(bits[l - 1] << (10 - l) for l in range(1, 11))
            fast = tab[t * 1024:(t + 1) * 1024]
            assert int(((fast & 31) > 0).sum() + ((fast & (1 << 15)) > 0).sum()) == want


# ------------------------------------------------------- marker layout
def _segments(data):
    """(marker, whole segment bytes) of the header up to and including SOS,
    and the entropy-coded rest (split by segment lengths, not by the
    library's or the oracle's parser)."""
    assert data[:2] == b"\xff\xd8"
    segs, p = [], 2
    while True:
        assert data[p] == 0xFF
        m = data[p + 1]
        n = (data[p + 2] << 8) | data[p + 3]
        segs.append((m, data[p:p + 2 + n]))
        p += 2 + n
        if m == 0xDA:
            return segs, data[p:]


def _assemble(segs, rest):
    return b"\xff\xd8" + b"".join(seg for _, seg in segs) + rest


def _merged(segs, marker):
    """The segments of one kind (DQT or DHT) merged into one, where the first was."""
    body = b"".join(seg[4:] for m, seg in segs if m == marker)
    one = bytes([0xFF, marker, (len(body) + 2) >> 8, (len(body) + 2) & 255]) + body
    out, done = [], False
    for m, seg in segs:
        if m != marker:
            out.append((m, seg))
        elif not done:
            out.append((m, one))
            done = True
    return out


def _layouts(data):
    segs, rest = _segments(data)
    app = lambda n, payload: (0xE0 + n, bytes([0xFF, 0xE0 + n, 0, len(payload) + 2]) + payload)
    com = (0xFE, b"\xff\xfe\x00\x08layout")
    yield "app and comment segments", [app(1, b"Exif\x00\x00"), com] + segs[:-1] + [app(15, b"x" * 9)] + segs[-1:]
    yield "fill bytes before markers", [(m, b"\xff\xff" + seg) for m, seg in segs]
    yield "one DQT segment", _merged(segs, 0xDB)
    # the same with its tables in the other order (each names its slot)
    merged = _merged(segs, 0xDB)
    m, one = next(x for x in merged if x[0] == 0xDB)
    flipped = one[:4] + one[4 + 65:] + one[4:4 + 65]
    yield "one DQT segment, tables reversed", [(mm, flipped if mm == 0xDB else ss) for mm, ss in merged]
    yield "one DHT segment", _merged(segs, 0xC4)
    sof = [x for x in segs if x[0] == 0xC0]
    tables = [x for x in segs if x[0] in (0xDB, 0xC4)]
    others = [x for x in segs if x[0] not in (0xC0, 0xDB, 0xC4, 0xDA)]
    yield "tables between SOF and SOS", others + sof + tables + segs[-1:]


@pytest.mark.parametrize("src", ["synth 420", "synth 444", "pil optimised 420"])
def test_index_is_invariant_to_marker_layout(src):
    """Re-laid-out markers (APPn and COM segments, fill bytes, tables merged
    into one segment or moved between SOF and SOS: all legal T.81 layouts)
    leave the index byte-identical to the canonical file's: the library's
    marker handling pinned without the oracle's parser."""
    rgb = synth.texture(91, 72, 56)
    if src.startswith("synth"):
        data = synth.encode(rgb, 80, int(src[-3:]))
    else:
        b = io.BytesIO()
        Image.fromarray(rgb).save(b, format="JPEG", quality=80, subsampling=2, optimize=True)
        data = b.getvalue()
    ref = jpt.build_index(data)
    segs, rest = _segments(data)
    assert _assemble(segs, rest) == data
    for name, layout in _layouts(data):
        li = jpt.build_index(_assemble(layout, rest))
        # every field: sizes, quantisers, Huffman specifications, overheads
        assert bytes(li.info) == bytes(ref.info), name
        assert np.array_equal(li.stream, ref.stream) and np.array_equal(li.records, ref.records), name
        assert np.array_equal(jpt.build_tables(li.info), jpt.build_tables(ref.info)), name


# ------------------------------------------------------------ error paths
def test_errors():
    data = synth.encode(synth.texture(1, 64, 64), 75, 420)
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(b"\x00\x01garbage")
    assert e.value.status == jpt.JPT_E_CORRUPT
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(data[: len(data) // 2])
    assert e.value.status == jpt.JPT_E_CORRUPT
    b = io.BytesIO()
    Image.fromarray(synth.texture(2, 32, 32)).save(b, format="JPEG", quality=75, progressive=True)
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(b.getvalue())
    assert e.value.status == jpt.JPT_E_UNSUPPORTED
    # a restart interval (DRI) is not supported
    i = data.index(b"\xff\xda")
    dri = data[:i] + b"\xff\xdd\x00\x04\x00\x10" + data[i:]
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(dri)
    assert e.value.status == jpt.JPT_E_UNSUPPORTED
    # grayscale (one component) is not supported
    b = io.BytesIO()
    Image.fromarray(synth.texture(2, 32, 32)[..., 0]).save(b, format="JPEG", quality=75)
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(b.getvalue())
    assert e.value.status == jpt.JPT_E_UNSUPPORTED
    # too-small buffers
    info = jpt.LevelInfo()
    buf = np.frombuffer(data, np.uint8)
    st_ = jpt.lib().jpt_build_index(buf.ctypes.data_as(ctypes.c_void_p), len(buf), ctypes.byref(info),
                                    np.zeros(4, np.uint32).ctypes.data_as(ctypes.c_void_p), 4, None, 0)
    assert st_ == jpt.JPT_E_BUFSIZE
    assert jpt.lib().jpt_build_index(None, 0, None, None, 0, None, 0) == jpt.JPT_E_ARG


# ------------------------------------------------------------------- ABI
def test_library_exports_every_declared_function():
    hdr = open(jpt.os.path.join(jpt.os.path.dirname(jpt._PKG), "include", "jpt.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(jpt_[a-z0-9_]+)\s*\(", hdr))
    assert names, "no declarations found"
    L = ctypes.CDLL(jpt.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert set(jpt.SIGNATURES) == names
    assert jpt.lib().jpt_version() == 1


def test_device_calls_reject_bad_arguments_without_gpu():
    L = jpt.lib()
    sc = jpt.SceneC(); fr = jpt.FrameC()
    assert L.jpt_mark_blocks(None, None, 0, 0, None, None, None, None) == jpt.JPT_E_ARG
    assert L.jpt_mark_blocks(ctypes.byref(sc), None, 0, 7, ctypes.byref(fr), None, None, None) == jpt.JPT_E_ARG
    assert L.jpt_decode_blocks(ctypes.byref(sc), ctypes.byref(fr), None, 0, None, None) == jpt.JPT_E_ARG
    assert L.jpt_resolve(ctypes.byref(sc), None, 0, 0, None, None, None, None) == jpt.JPT_E_ARG
    assert L.jpt_mark_blocks_static(None, None, 0, 0, None, None, None, None) == jpt.JPT_E_ARG
    assert L.jpt_mark_blocks_static(ctypes.byref(sc), None, 0, 7, ctypes.byref(fr), None, None, None) == jpt.JPT_E_ARG
    # a scene of fewer than 32 block ids, with or without textures (jpt_layout
    # never makes one; resolve reads the slot table in pairs, and at block 0
    # for the pixels of a scene without textures)
    fake = 0x1000  # never dereferenced: the checks fail first
    for n_tex, n_blocks in ((1, 0), (1, 31), (0, 0)):
        sc2 = jpt.SceneC(fake, fake, fake, fake, fake, 1, n_tex, 1, 1, n_blocks, 0)
        ca = jpt.CacheC(fake, fake, None, None, None, None, None, None, 1, 0, None, 0, 0)
        assert L.jpt_resolve(ctypes.byref(sc2), None, 0, 1, None, ctypes.byref(ca), None, None) == jpt.JPT_E_ARG
    # both forms of the slot lookups forced at once
    sc2 = jpt.SceneC(fake, fake, fake, fake, fake, 1, 1, 1, 1, 32, 0)
    t = jpt.TuningC()
    t.flags = jpt.TUNE_RESOLVE_PAIRED | jpt.TUNE_RESOLVE_SINGLE
    assert L.jpt_resolve(ctypes.byref(sc2), None, 0, 1, None, ctypes.byref(ca), ctypes.byref(t), None) == \
        jpt.JPT_E_ARG


def test_static_mark_rejects_scenes_beyond_its_scratch():
    """jpt_mark_blocks_static checks the scene against its fixed scratch
    before any device work: the largest scene (2^29 block ids) needs more
    than JPT_STATIC_SCAN_ENTRIES scan entries."""
    L = jpt.lib()
    fake = 0x1000  # never dereferenced: the checks fail first
    sc = jpt.SceneC(fake, fake, fake, fake, fake, 1, 1, 1, 1, 1 << 29, 0)
    fr = jpt.FrameC(fake, fake, fake, 0, fake, 1, 0)
    assert L.jpt_scan_entries(1 << 29) > jpt.STATIC_SCAN_ENTRIES
    assert L.jpt_mark_blocks_static(ctypes.byref(sc), None, 0, 0, ctypes.byref(fr), None, None, None) == \
        jpt.JPT_E_CAPACITY
    # the largest scene it takes: 3 per-tile entries and 16 per 256 tiles, plus one
    tiles = (1 << 29) // 32 // 256
    while L.jpt_scan_entries(tiles * 256 * 32) > jpt.STATIC_SCAN_ENTRIES:
        tiles -= 1
    assert tiles * 256 * 32 >= 100_000_000  # over 25 G texels of block ids


# ------------------------------------------- the predictor index reading
def predicted_equals_sequential(data):
    li = jpt.build_index(data, jpt.INDEX_PREDICTORS)
    j = oracle.Jpeg(data)
    coef, mb, pred, dcb = j.decode()
    inf = li.info
    assert inf.index_kind == jpt.INDEX_PREDICTORS
    assert inf.removed_dc_bits == 0 and inf.stream_bits == inf.scan_bits == mb[-1]
    assert abs(inf.overhead_bpp_effective - inf.overhead_bpp_bound) < 1e-12
    rec = li.records.reshape(-1, 64)
    for m in range(j.n_mcu):
        # the record's offset is the MCU's start in the original segment and
        # its fields are the predictors the sequential decode had there
        g, r = divmod(m, 9)
        bits = np.unpackbits(rec[g], bitorder="little")
        anchor = int(np.packbits(bits[0:32], bitorder="little").view(np.uint32)[0])
        rel = 0 if r == 0 else int(np.packbits(bits[32 + 16 * (r - 1):48 + 16 * (r - 1)],
                                                bitorder="little").view(np.uint16)[0])
        assert anchor + rel == mb[m]
        for c in range(3):
            f = bits[160 + 12 * (3 * r + c):172 + 12 * (3 * r + c)]
            v = int(sum(int(x) << i for i, x in enumerate(f)))
            assert (v - 4096 if v >= 2048 else v) == pred[m, c]
        rc, out, end = j.decode_predicted_mcu(li.stream, inf.stream_bits, li.records, m)
        assert rc == 0 and np.array_equal(out, coef[m]) and end == mb[m + 1], m
    return li


@pytest.mark.parametrize("smp", [420, 444])
@pytest.mark.parametrize("q", [5, 50, 95])
def test_predictor_index_matches_sequential(smp, q):
    rgb = synth.texture(q * 11 + smp, 136, 88)
    data = synth.encode(rgb, q, smp)
    li = predicted_equals_sequential(data)
    # the stream is the untouched segment: the spliced one is shorter by the removed DC codes
    sp = jpt.build_index(data)
    assert li.info.stream_bits == sp.info.stream_bits + sp.info.removed_dc_bits
    # the paper's bound, nothing removed: (32 + 8 * 16) / 9 + 36 bits per MCU
    ms = 16 if smp == 420 else 8
    assert abs(li.info.overhead_bpp_bound - ((32 + 16 * 8) / 9 + 36) / (ms * ms)) < 1e-12


def test_predictor_index_on_pil_files_with_optimised_tables():
    rgb = synth.texture(78, 120, 72)
    b = io.BytesIO()
    Image.fromarray(rgb).save(b, format="JPEG", quality=85, subsampling=2, optimize=True)
    predicted_equals_sequential(b.getvalue())


# ---------------------------------------------------------- size queries
def _info(w, h, smp):
    inf = jpt.LevelInfo()
    inf.width, inf.height, inf.sampling = w, h, smp
    inf.blk_cols, inf.blk_rows = (w + 15) // 16, (h + 15) // 16
    return inf


def test_query_sizes_closed_forms():
    """jpt_query_sizes against counts worked out by hand: a 256^2 4:2:0
    texture (256 blocks, one item each), a 40x24 4:4:4 level (3x2 blocks of
    up to four MCUs each) and block ids padded to multiples of 32."""
    infos = [_info(256, 256, 420), _info(40, 24, 444)]
    s = jpt.query_sizes(infos, [(256, 256)], jpt.FILTER_NEAREST)
    assert s.n_blocks == 256 + 32 and s.vis_words == 9 and s.scan_entries == jpt.lib().jpt_scan_entries(288)
    assert s.items_total == 256 + 6 * 4 and s.pixels == 65536
    assert s.max_items == 280 and s.max_blocks == 262 and s.texel_words == 262 * 256
    assert s.coef_entries == 280 * 6 * 64
    # few pixels bound the frame instead: 3 pixels, trilinear (8 blocks a pixel, 4 items a 4:4:4 block)
    s = jpt.query_sizes(infos, [(3, 1)], jpt.FILTER_TRILINEAR)
    assert s.max_blocks == 24 and s.max_items == 96
    s = jpt.query_sizes(infos[:1], [(2, 1), (1, 1)], jpt.FILTER_BILINEAR | jpt.FILTER_MIP_OFF)
    assert s.max_blocks == 12 and s.max_items == 12 and s.pixels == 3
    s = jpt.query_sizes(infos[:1], [(5, 1)], jpt.FILTER_BILINEAR_CLAMPED)
    assert s.max_blocks == 5
    with pytest.raises(jpt.JptError):
        jpt.query_sizes(infos, [(4, 4)], 9)
    assert jpt.lib().jpt_query_sizes(None, 0, None, 0, 0, None) == jpt.JPT_E_ARG
