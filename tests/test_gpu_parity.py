"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: visible blocks, work items and coefficients bit-exact; texels within
1 LSB of the fp64 oracle with every mismatch at a rounding near-tie; frames
bit-exact against the oracle's resolve of the GPU texels and within 1 LSB of
the oracle's full render.
"""
import numpy as np
import pytest

import oracle
from oracle import parity
from paper_2510_08166_amd.synth import configs

from gpu_common import full_parity, run

pytestmark = pytest.mark.gpu


def test_tiny_all_blocks(gpu):
    wl = configs.tiny()
    r, osc, blocks = full_parity(wl)
    assert len(blocks) == 256                      # all 1024 luma 8x8 blocks of the 256^2 texture
    assert len(r.frame.work_items()) * 6 == 1536   # 1536 data units
    # nearest at texel centres: the frame is the decoded texture itself
    lvl = osc.decode_level(0)
    f = oracle.unpack_frame(r.views.frame_host())
    assert np.abs(f[:, :, :3].astype(int) - lvl.astype(int)).max() <= 1


@pytest.mark.parametrize("filt", [configs.FILTER_NEAREST, configs.FILTER_BILINEAR, configs.FILTER_TRILINEAR])
def test_reduced_filters(gpu, filt):
    wl = configs.reduced(seed=11, filt=filt)
    full_parity(wl)


@pytest.mark.parametrize("n_tex", [300, 600])
def test_descriptors_beyond_the_lds_cache(gpu, n_tex):
    """Scenes with more levels (300 x 5 = 1500) or more textures (600) than the
    mark and resolve kernels keep in LDS: texture records in LDS and level
    records from HBM, or every record from HBM."""
    wl = configs.quad_scene(31, n_tex, 16, 50, 90, 5, 160, 120, 40, filt=configs.FILTER_TRILINEAR,
                            name="%d textures of 16^2" % n_tex)
    full_parity(wl)


def test_reduced_444_and_ragged(gpu):
    # 4:4:4 textures with a side that is not a multiple of 16 -> partial blocks and MCUs
    wl = configs.quad_scene(21, 3, 200, 50, 95, 4, 160, 120, 12, sampling=444,
                            filt=configs.FILTER_BILINEAR, name="444 ragged")
    full_parity(wl)


@pytest.mark.parametrize("case", ["420 trilinear", "444 ragged"])
def test_scalar_f32_idct(gpu, case):
    """The separable fp32 IDCT (JPT_IDCT_SCALAR_F32) to the same bar as the MFMA one."""
    from paper_2510_08166_amd import jpt
    if case == "444 ragged":
        wl = configs.quad_scene(22, 3, 200, 50, 95, 4, 160, 120, 12, sampling=444, filt=configs.FILTER_BILINEAR)
    else:
        wl = configs.reduced(seed=12, filt=configs.FILTER_TRILINEAR)
    full_parity(wl, idct_mode=jpt.IDCT_SCALAR_F32)


@pytest.mark.parametrize("case", ["420 trilinear", "444 ragged"])
def test_mfma_bf16_idct(gpu, case):
    """The bf16 MFMA IDCT (JPT_IDCT_MFMA_BF16) to the same bar as the fp16 one."""
    from paper_2510_08166_amd import jpt
    if case == "444 ragged":
        wl = configs.quad_scene(23, 3, 200, 50, 95, 4, 160, 120, 12, sampling=444, filt=configs.FILTER_BILINEAR)
    else:
        wl = configs.reduced(seed=13, filt=configs.FILTER_TRILINEAR)
    full_parity(wl, idct_mode=jpt.IDCT_MFMA_BF16)


@pytest.mark.parametrize("case", ["420 trilinear", "444 ragged", "corrupt", "8 decode groups", "16 decode groups"])
def test_fused_decode_matches_scalar(gpu, case):
    """JPT_IDCT_FUSED_F32 (entropy decode, IDCT and colour in one kernel) stores
    exactly the texels of the two-kernel scalar fp32 path (also on small
    decode grids, where each wave takes many MCUs and a grid of a multiple of
    8 workgroups deals them XCD by XCD)."""
    from paper_2510_08166_amd import jpt
    if case == "444 ragged":
        wl = configs.quad_scene(23, 3, 200, 50, 95, 4, 160, 120, 12, sampling=444, filt=configs.FILTER_BILINEAR)
    else:
        wl = configs.reduced(seed=13, filt=configs.FILTER_TRILINEAR)
    tuning = None
    if case.endswith("decode groups"):
        tuning = jpt.TuningC()
        tuning.decode_groups = int(case.split()[0])
    res = []
    for mode in (jpt.IDCT_SCALAR_F32, jpt.IDCT_FUSED_F32):
        import torch
        r = jpt.Renderer(wl.textures, wl.views, wl.filter, tuning=tuning if mode == jpt.IDCT_FUSED_F32 else None)
        if case == "corrupt":
            r.scene.streams.fill_(0xFF)
        r.mark()
        r.decode(idct_mode=mode)
        r.resolve()
        torch.cuda.synchronize()
        ctr = r.frame.counters_host().copy()
        n_new = min(int(ctr[jpt.CTR_NEW]), r.cache.n_slots)
        res.append((ctr, r.frame.work_items(), r.cache.texels[: n_new * 256].cpu().numpy(), r.views.frame_host()))
    (c0, i0, t0, f0), (c1, i1, t1, f1) = res
    assert np.array_equal(c0[:7], c1[:7]) and np.array_equal(i0, i1)
    assert np.array_equal(t0, t1) and np.array_equal(f0, f1)
    if case == "corrupt":
        fg = wl.views[0]["tex"] != oracle.BACKGROUND
        assert c1[jpt.CTR_ERROR] & jpt.ERR_CORRUPT and (f1[fg] == jpt.TEXEL_INVALID).all()


@pytest.mark.parametrize("wide_bits", [1, 0xFFFFFFFF])
def test_entropy_step_width(gpu, wide_bits):
    """Every MCU through the decoder's 128-offset steps (wide_bits 1) or
    none (64-offset steps only): coefficients bit-exact against the oracle
    for 4:2:0 and ragged 4:4:4, and corrupt streams still flagged."""
    import torch
    from paper_2510_08166_amd import jpt
    t = jpt.TuningC()
    t.wide_bits = wide_bits
    wl = configs.reduced(seed=14, filt=configs.FILTER_TRILINEAR)
    full_parity(wl, tuning=t)
    full_parity(configs.quad_scene(24, 3, 200, 50, 97, 4, 160, 120, 12, sampling=444,
                                   filt=configs.FILTER_BILINEAR), tuning=t)
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, tuning=t)
    r.scene.streams.fill_(0xFF)
    r.render()
    torch.cuda.synchronize()
    assert r.frame.counters_host()[jpt.CTR_ERROR] & jpt.ERR_CORRUPT
    assert (r.frame.work_items() >> 31).all()


def test_many_tiles(gpu):
    # more work items than one decode wave and several scan tiles of bitmask words
    wl = configs.quad_scene(5, 12, 512, 40, 95, 6, 640, 360, 40, filt=configs.FILTER_BILINEAR, name="many tiles")
    full_parity(wl, full_render=False)


def test_background_only(gpu):
    from paper_2510_08166_amd import jpt
    wl = configs.tiny()
    wl.views[0]["tex"] = 0xFFFFFFFF
    r, ctr, items, coef, tiles, frames = run(wl)
    assert ctr[jpt.CTR_ITEMS] == 0 and ctr[jpt.CTR_ERROR] == 0
    assert not frames[0].any()


def test_invalid_pixels_flagged(gpu):
    from paper_2510_08166_amd import jpt
    wl = configs.tiny()
    g = wl.views[0]
    g["u"][0, 0] = np.nan
    g["tex"][0, 1] = 7            # no such texture
    g["v"][0, 2] = np.float32(1e12)
    r, ctr, items, coef, tiles, frames = run(wl)
    assert ctr[jpt.CTR_ERROR] & jpt.ERR_PIXEL
    assert frames[0][0, 0] == jpt.TEXEL_INVALID and frames[0][0, 1] == jpt.TEXEL_INVALID
    assert frames[0][0, 2] == jpt.TEXEL_INVALID
    osc = oracle.Scene(wl.textures)
    ref, _, bad = osc.render(g, wl.filter)
    assert bad == 3
    assert parity.frame_diff(frames[0], ref) <= 1


def test_capacity_overflow_is_flagged(gpu):
    from paper_2510_08166_amd import jpt
    wl = configs.tiny()
    r, ctr, items, coef, tiles, frames = run(wl, max_items=100, n_slots=100)
    assert ctr[jpt.CTR_ERROR] & jpt.ERR_CAPACITY
    assert ctr[jpt.CTR_ITEMS] == 100
    f = frames[0]
    assert (f == jpt.TEXEL_INVALID).sum() > 0


def test_corrupt_stream_flagged(gpu):
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.tiny()
    r = jpt.Renderer(wl.textures, wl.views, wl.filter)
    # all-ones bits are no code of the Annex K tables: every MCU must fail
    r.scene.streams.fill_(0xFF)
    r.render()
    torch.cuda.synchronize()
    ctr = r.frame.counters_host()
    assert ctr[jpt.CTR_ERROR] & jpt.ERR_CORRUPT
    assert ctr[jpt.CTR_ERROR_ITEM] == 0
    items = r.frame.work_items()
    assert (items >> 31).all()
    assert (r.views.frame_host() == jpt.TEXEL_INVALID).all()


def test_pil_files_with_optimised_tables(gpu):
    """Files written by libjpeg (through PIL) with per-image optimised Huffman
    tables: several table sets (decode tables read from HBM) and codes longer
    than the fast-table index."""
    import io
    from PIL import Image
    from paper_2510_08166_amd import synth
    texs = []
    for i, (q, sub) in enumerate([(92, 2), (60, 2), (85, 0), (97, 2)]):
        rgb = synth.texture(300 + i, 192, 160)
        levels = synth.mip_chain(rgb, 3)
        jp = []
        for l in levels:
            b = io.BytesIO()
            Image.fromarray(l).save(b, format="JPEG", quality=q, subsampling=sub, optimize=True)
            jp.append(b.getvalue())
        texs.append(synth.EncodedTexture(i, 192, 160, q, 420 if sub == 2 else 444, jp))
    rng = np.random.default_rng(8)
    quads = synth.random_quads(rng, 240, 180, 20, list(range(4)), {i: (192.0, 160.0) for i in range(4)})
    g = synth.rasterise(240, 180, quads)
    wl = configs.Workload("pil optimised", texs, [g], configs.FILTER_TRILINEAR)
    from paper_2510_08166_amd import jpt
    assert len(jpt.HostScene(texs).tablesets) > 1
    full_parity(wl)


def test_lru_cache_over_drifting_frames(gpu):
    """LRU cache under camera drift (mixed 4:2:0 / 4:4:4, full mip chains,
    trilinear): per frame, the decoded set, the number of evictions and the
    resident set equal the oracle's simulator; frames match the oracle."""
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.heavy(seed=31, n_tex=12, sides=(64, 128, 256), W=320, H=200, n_quads=40, n_frames=6)
    osc = oracle.Scene(wl.textures)
    vis_sets = [parity.visible_blocks(osc, [g], wl.filter) for g in wl.views]
    cap = max(len(v) for v in vis_sets) + 24          # small: forces evictions every frame
    r = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, n_slots=cap, policy=jpt.CACHE_LRU)
    sim = oracle.LruSim(cap)
    lc = parity.LevelCache(osc)
    evictions = 0
    for f, g in enumerate(wl.views):
        r.set_views([g])
        r.render()
        torch.cuda.synchronize()
        ctr = r.frame.counters_host()
        new, ev = sim.step(f, vis_sets[f])
        evictions += len(ev)
        items = r.frame.work_items()
        print("frame %d: visible %d new %d evicted %d err %x" % (f, ctr[jpt.CTR_VISIBLE], ctr[jpt.CTR_NEW],
                                                                ctr[jpt.CTR_EVICTED], ctr[jpt.CTR_ERROR]), flush=True)
        assert ctr[jpt.CTR_ERROR] == 0
        assert ctr[jpt.CTR_VISIBLE] == len(vis_sets[f])
        assert np.array_equal(items, parity.expected_items(osc, np.array(new, np.uint32)))
        assert ctr[jpt.CTR_EVICTED] == len(ev)
        assert np.array_equal(r.cache.resident_blocks(), np.array(sorted(sim.last_used), np.uint32))
        assert ctr[jpt.CTR_RESIDENT] == len(sim.last_used)
        # texels of every visible block, fetched through slot_of
        slot_of = r.cache.slot_of.cpu().numpy().view(np.uint32)
        tex = r.cache.texels.cpu().numpy().view(np.uint32).reshape(-1, 256)
        blocks = vis_sets[f]
        assert (slot_of[blocks] != jpt.SLOT_NONE).all()
        tiles = tex[slot_of[blocks]]
        maxd, nmis, tie, dist, n = parity.check_texels(lc, blocks, tiles)
        assert maxd <= 1 and tie <= 1.0
        ref, bad = osc.resolve(g, wl.filter, parity.levels_from_tiles(osc, blocks, tiles))
        assert np.array_equal(r.views.frame_host(), ref)
    assert evictions > 0


def lru_gap_workload():
    """Twelve small textures (mixed 4:2:0 / 4:4:4, full chains) and four
    independent quad scenes over them, shown in the order A B C D A C B D A
    at frame numbers far apart."""
    from paper_2510_08166_amd import synth
    base = configs.heavy(seed=32, n_tex=12, sides=(64, 128, 256), W=320, H=200, n_quads=40, n_frames=1)
    sizes = {i: (float(s), float(s)) for i, s in enumerate(base.extra["sides"])}
    rng = np.random.default_rng(77)
    scenes = [synth.rasterise(320, 200, synth.random_quads(rng, 320, 200, 40, list(range(12)), sizes))
              for _ in range(4)]
    order = [0, 1, 2, 3, 0, 2, 1, 3, 0]
    frame_nos = [0, 1, 1500, 1501, 2_100_000, 2_100_001, 2_100_900, 4_000_000_000, 4_000_000_001]
    return configs.Workload("lru gaps", base.textures, [scenes[i] for i in order], configs.FILTER_TRILINEAR), \
        frame_nos


def test_lru_exact_ages_past_the_histogram_cap(gpu):
    """Frame numbers set explicitly, far apart (0, 1, 1500, ... 4e9), so that
    eviction candidates are more than JPT_LRU_MAX_AGE frames old and differ
    in every digit of their 32-bit age: decoded, evicted and resident sets
    still equal the plain LRU simulator (smallest last use first, then the
    smaller block id), and frames match the oracle."""
    import torch
    from paper_2510_08166_amd import jpt
    wl, frame_nos = lru_gap_workload()
    osc = oracle.Scene(wl.textures)
    vis_sets = [parity.visible_blocks(osc, [g], wl.filter) for g in wl.views]
    cap = max(len(v) for v in vis_sets) + 40
    r = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, n_slots=cap, policy=jpt.CACHE_LRU)
    sim = oracle.LruSim(cap)
    lc = parity.LevelCache(osc)
    deep_frames = 0
    for fno, g, V in zip(frame_nos, wl.views, vis_sets):
        r.set_views([g])
        r.frame_no = fno
        r.render()
        torch.cuda.synchronize()
        ctr = r.frame.counters_host()
        new, ev = sim.step(fno, V)
        deep = int(r.cache.meta[7].item())   # set when the evictions ended among blocks past the age cap
        deep_frames += deep
        print("frame %d: visible %d new %d evicted %d (oracle %d) deep %d err %x" % (
            fno, ctr[jpt.CTR_VISIBLE], ctr[jpt.CTR_NEW], ctr[jpt.CTR_EVICTED], len(ev), deep, ctr[jpt.CTR_ERROR]),
            flush=True)
        assert ctr[jpt.CTR_ERROR] == 0
        assert np.array_equal(r.frame.work_items(), parity.expected_items(osc, np.array(new, np.uint32)))
        assert ctr[jpt.CTR_EVICTED] == len(ev)
        assert np.array_equal(r.cache.resident_blocks(), np.array(sorted(sim.last_used), np.uint32))
        slot_of = r.cache.slot_of.cpu().numpy().view(np.uint32)
        tex = r.cache.texels.cpu().numpy().view(np.uint32).reshape(-1, 256)
        tiles = tex[slot_of[V]]
        maxd, nmis, tie, dist, n = parity.check_texels(lc, V, tiles)
        assert maxd <= 1 and tie <= 1.0
        ref, bad = osc.resolve(g, wl.filter, parity.levels_from_tiles(osc, V, tiles))
        assert np.array_equal(r.views.frame_host(), ref)
    assert deep_frames >= 3


@pytest.mark.parametrize("sampling", [420, 444])
@pytest.mark.parametrize("q,dc_max,density", [(8, 255, 0.05), (255, 2047, 0.1)])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_wide_coefficients(gpu, sampling, q, dc_max, density, mode):
    """Crafted streams at the limits the index admits (ACs up to 1023, DCs
    up to 2047, quantisers up to 255, so |F| up to 521985): coefficients
    bit-exact and texels within 1 LSB in every IDCT mode; the MFMA path
    takes its three-digit split of F for these units (fp16 and bf16)."""
    from paper_2510_08166_amd.synth import EncodedTexture, GPIXEL_DTYPE
    from jpeg_writer import mcu_count, mcus_from_coefs, random_coefs, write_jpeg
    w, h = (40, 24) if sampling == 420 else (24, 40)
    rng = np.random.default_rng(q * 7 + sampling)
    coef = random_coefs(rng, mcu_count(w, h, sampling), sampling, dc_max=dc_max, density=density)
    qt = np.full(64, q)
    data = write_jpeg(w, h, sampling, qt, qt, mcus_from_coefs(coef, sampling))
    tex = [EncodedTexture(0, w, h, 0, sampling, [data])]
    y, x = np.mgrid[0:h, 0:w]
    g = np.zeros((h, w), GPIXEL_DTYPE)
    g["u"] = ((x + 0.5) / w).astype(np.float32)
    g["v"] = ((y + 0.5) / h).astype(np.float32)
    wl = configs.Workload("wide q%d %d" % (q, sampling), tex, [g], configs.FILTER_NEAREST)
    r, osc, blocks = full_parity(wl, idct_mode=mode)
    assert len(blocks) == ((w + 15) // 16) * ((h + 15) // 16)


@pytest.mark.parametrize("filt", [configs.FILTER_BILINEAR_CLAMPED,
                                  configs.FILTER_BILINEAR_CLAMPED | configs.FILTER_MIP_OFF,
                                  configs.FILTER_NEAREST | configs.FILTER_MIP_OFF,
                                  configs.FILTER_TRILINEAR | configs.FILTER_MIP_OFF])
def test_paper_variants_clamped_and_mip_off(gpu, filt):
    """The paper's single-MCU clamped bilinear (centre-only marking) and its
    rows without mip mapping, against the oracle's definitions."""
    wl = configs.reduced(seed=12, filt=filt)
    r, osc, blocks = full_parity(wl)
    if filt & 0xFF == configs.FILTER_BILINEAR_CLAMPED:
        near, _ = osc.mark(wl.views[0], configs.FILTER_NEAREST | (filt & configs.FILTER_MIP_OFF))
        assert np.array_equal(blocks, near)


def test_evict_invisible_policy(gpu):
    """The paper's Update Cache: after each frame every block the frame did
    not read leaves the cache; decoded and evicted sets equal the oracle's
    simulator, frames match the oracle."""
    import torch
    from paper_2510_08166_amd import jpt
    wl, _ = lru_gap_workload()
    osc = oracle.Scene(wl.textures)
    vis_sets = [parity.visible_blocks(osc, [g], wl.filter) for g in wl.views]
    cap = max(len(v) for v in vis_sets) + 8
    r = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, n_slots=cap, policy=jpt.CACHE_EVICT_INVISIBLE)
    sim = oracle.EvictInvisibleSim(cap)
    lc = parity.LevelCache(osc)
    for f, (g, V) in enumerate(zip(wl.views, vis_sets)):
        r.set_views([g])
        r.render()
        torch.cuda.synchronize()
        ctr = r.frame.counters_host()
        new, ev = sim.step(V)
        print("frame %d: visible %d new %d evicted %d (oracle %d) err %x" % (
            f, ctr[jpt.CTR_VISIBLE], ctr[jpt.CTR_NEW], ctr[jpt.CTR_EVICTED], len(ev), ctr[jpt.CTR_ERROR]), flush=True)
        assert ctr[jpt.CTR_ERROR] == 0
        assert np.array_equal(r.frame.work_items(), parity.expected_items(osc, np.array(new, np.uint32)))
        assert ctr[jpt.CTR_EVICTED] == len(ev)
        assert np.array_equal(r.cache.resident_blocks(), np.array(sorted(sim.resident), np.uint32))
        slot_of = r.cache.slot_of.cpu().numpy().view(np.uint32)
        tiles = r.cache.texels.cpu().numpy().view(np.uint32).reshape(-1, 256)[slot_of[V]]
        maxd, nmis, tie, dist, n = parity.check_texels(lc, V, tiles)
        assert maxd <= 1 and tie <= 1.0
        ref, bad = osc.resolve(g, wl.filter, parity.levels_from_tiles(osc, V, tiles))
        assert np.array_equal(r.views.frame_host(), ref)


def test_hash_map_cache(gpu):
    """The paper's hash-map block cache (16/13/3-bit keys, atomicCAS in mark,
    a probe per tap in resolve, invisible blocks evicted): per frame the
    decoded set (in insertion order, so compared as a set) and the evicted
    count equal the evict-invisible simulator, every visible block's key maps
    to a slot holding its texels, and frames equal the oracle's resolve of
    those texels."""
    import torch
    from paper_2510_08166_amd import jpt, synth
    wl0 = configs.quad_scene(71, 5, 256, 50, 90, 5, 320, 200, 30, filt=configs.FILTER_BILINEAR)
    sizes = {i: (256.0, 256.0) for i in range(5)}
    rng = np.random.default_rng(72)
    scenes = [wl0.views[0]] + [synth.rasterise(320, 200, synth.random_quads(rng, 320, 200, 30, list(range(5)), sizes))
                               for _ in range(3)]
    order = [0, 1, 1, 2, 0, 3, 3, 1]
    osc = oracle.Scene(wl0.textures)
    vis_sets = [parity.visible_blocks(osc, [scenes[i]], wl0.filter) for i in order]
    cap = max(len(v) for v in vis_sets) + 16
    r = jpt.Renderer(wl0.textures, [scenes[0]], wl0.filter, n_slots=cap, policy=jpt.CACHE_HASH)
    sim = oracle.EvictInvisibleSim(cap)
    lc = parity.LevelCache(osc)
    for f, (i, V) in enumerate(zip(order, vis_sets)):
        g = scenes[i]
        r.set_views([g])
        r.render()
        torch.cuda.synchronize()
        ctr = r.frame.counters_host()
        new, ev = sim.step(V)
        items = r.frame.work_items()
        print("frame %d: visible %d new %d evicted %d (oracle %d) err %x" % (
            f, ctr[jpt.CTR_VISIBLE], ctr[jpt.CTR_NEW], ctr[jpt.CTR_EVICTED], len(ev), ctr[jpt.CTR_ERROR]), flush=True)
        assert ctr[jpt.CTR_ERROR] == 0
        assert ctr[jpt.CTR_VISIBLE] == len(V)
        assert np.array_equal(np.sort(items), parity.expected_items(osc, np.array(new, np.uint32)))
        assert ctr[jpt.CTR_EVICTED] == len(ev)
        # the map: every visible block's key -> its slot
        ent = r.cache.hash_entries()
        slots = []
        for b in V:
            L, bx, by = osc.block_coords(int(b))
            t = int(np.searchsorted(osc.tex_first, L, side="right") - 1)
            key = ((by * int(osc.blk_cols[L]) + bx) << 16) | (t << 3) | (L - int(osc.tex_first[t]))
            assert key in ent
            slots.append(ent[key])
        tex = r.cache.texels.cpu().numpy().view(np.uint32).reshape(-1, 256)
        tiles = tex[np.array(slots)]
        maxd, nmis, tie, dist, n = parity.check_texels(lc, V, tiles)
        assert maxd <= 1 and tie <= 1.0
        ref, bad = osc.resolve(g, wl0.filter, parity.levels_from_tiles(osc, V, tiles))
        assert np.array_equal(r.views.frame_host(), ref)


@pytest.mark.parametrize("filt", [configs.FILTER_NEAREST, configs.FILTER_BILINEAR, configs.FILTER_TRILINEAR])
def test_resolve_beyond_4_gib_of_texels(gpu, filt):
    """A cache of more than 2^22 slots (over 4 GiB of texels) takes resolve's
    64-bit texel addressing; its frame equals the 32-bit path's bit for bit
    (the frame's blocks sit in the first slots either way)."""
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.reduced(seed=14, filt=filt)
    frames = []
    for n_slots in (None, (1 << 22) + 1):
        r = jpt.Renderer(wl.textures, wl.views, wl.filter, n_slots=n_slots)
        r.render()
        torch.cuda.synchronize()
        assert r.frame.counters_host()[jpt.CTR_ERROR] == 0
        frames.append(r.views.frame_host().copy())
        del r
        torch.cuda.empty_cache()
    assert np.array_equal(frames[0], frames[1])


@pytest.mark.parametrize("form", ["paired", "single"])
@pytest.mark.parametrize("filt", [configs.FILTER_BILINEAR, configs.FILTER_BILINEAR_CLAMPED])
def test_taps_in_the_last_block_id(gpu, filt, form):
    """Bilinear taps in the scene's last block id and across both wraps of a
    level, with each form of resolve's slot lookups.  The paired form reads
    the slot table in 8-byte pairs (a tap's block and the next id); a pair
    that would start at the last id starts one earlier, and a tap the pair
    does not hold (a wrap) is read on its own.  The last texture is 128 x 64
    with one level: 32 blocks, so its bottom-right block is the scene's last
    id."""
    from paper_2510_08166_amd import jpt
    from paper_2510_08166_amd.synth import GPIXEL_DTYPE, make_textures, seed_ints
    s0, s1 = seed_ints(91, 2)
    tex = make_textures([(s0, 64, 64, 70, 420, 3), (s1, 128, 64, 80, 420, 1)])
    H, W = 56, 96
    y, x = np.mgrid[0:H, 0:W]
    g = np.zeros((H, W), GPIXEL_DTYPE)
    # steps of 1.35 texels from near the level's origin past its right edge
    # (u > 1 wraps) and down to its last texel row (whose y1 wraps to row 0)
    g["u"] = ((x * 1.35 + 0.4) / 128).astype(np.float32)
    g["v"] = (((y - 8) * 1.35 + 0.4) / 64).astype(np.float32)
    g["tex"] = 1
    g["lod"] = 0.0
    g["tex"][:8] = 0           # a band of the other texture, between its levels
    g["v"][:8] = ((y[:8] + 0.5) / 16).astype(np.float32)
    g["lod"][:8] = 1.3
    wl = configs.Workload("last block id", tex, [g], filt)
    t = jpt.TuningC()
    t.flags = jpt.TUNE_RESOLVE_PAIRED if form == "paired" else jpt.TUNE_RESOLVE_SINGLE
    r, _, _ = full_parity(wl, tuning=t)
    assert r.host.n_blocks % 32 == 0
    assert int(r.cache.slot_of[r.host.n_blocks - 1]) != -1   # the last id was read


@pytest.mark.parametrize("filt", [configs.FILTER_BILINEAR, configs.FILTER_BILINEAR_CLAMPED])
def test_resolve_slot_lookup_forms_agree(gpu, filt):
    """The paired and the single slot lookups of the bilinear resolves give
    the same frame bit for bit, on a scene of many textures, levels and
    block boundaries (the default picks by the launch's rounds of
    workgroups)."""
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.quad_scene(5, 12, 512, 40, 95, 6, 640, 360, 40, filt=filt, name="many tiles")
    frames = []
    for flags in (jpt.TUNE_RESOLVE_PAIRED, jpt.TUNE_RESOLVE_SINGLE, 0):
        t = jpt.TuningC()
        t.flags = flags
        r = jpt.Renderer(wl.textures, wl.views, wl.filter, tuning=t)
        r.render()
        torch.cuda.synchronize()
        assert r.frame.counters_host()[jpt.CTR_ERROR] == 0
        frames.append(r.views.frame_host().copy())
    assert np.array_equal(frames[0], frames[1]) and np.array_equal(frames[0], frames[2])
