"""Pins of the oracle's mark / resolve / cache simulator (paper: Method,
Mark, Resolve, Update Cache; Texture Block Cache).

Mark is pinned to resolve by perturbation (a block is marked exactly when
the unrounded frame depends on its texels), resolve to closed forms (texel
centres reproduce the texture, half-texel offsets average four texels,
constant textures give constant frames, uv repeats, trilinear at integer
lod equals bilinear), the LRU simulator to its invariants and to a
brute-force oldest-first check."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_2510_08166_amd.synth import GPIXEL_DTYPE, configs, make_textures, EncodedTexture, encode

NEAREST, BILINEAR, TRILINEAR = oracle.NEAREST, oracle.BILINEAR, oracle.TRILINEAR


def gb(u, v, tex=0, lod=0.0):
    u = np.atleast_2d(np.asarray(u, np.float32)); v = np.atleast_2d(np.asarray(v, np.float32))
    g = np.zeros(u.shape, GPIXEL_DTYPE)
    g["u"], g["v"], g["tex"], g["lod"] = u, v, tex, lod
    return g


@pytest.fixture(scope="module")
def small_scene():
    tex = make_textures([(11, 64, 64, 80, 420, 4), (12, 48, 32, 60, 444, 3)], keep_rgb=True)
    return oracle.Scene(tex)


def test_layout_is_32_aligned(small_scene):
    s = small_scene
    assert np.all(s.blk_base % 32 == 0)
    assert s.n_blocks % 32 == 0
    ends = s.blk_base + s.blk_cols * s.blk_rows
    assert np.all(ends[:-1] <= s.blk_base[1:])


def test_tiny_marks_every_block_and_reproduces_texture():
    wl = configs.tiny()
    s = oracle.Scene(wl.textures)
    frame, vis, bad = s.render(wl.views[0], NEAREST)
    assert bad == 0 and len(vis) == 256 and s.n_blocks == 256
    lvl = s.decode_level(0)
    assert np.array_equal(oracle.unpack_frame(frame)[:, :, :3], lvl)
    assert (oracle.unpack_frame(frame)[:, :, 3] == 255).all()


def test_bilinear_at_texel_centres_is_nearest(small_scene):
    s = small_scene
    x, y = np.meshgrid(np.arange(64), np.arange(64))
    g = gb((x + 0.5) / 64, (y + 0.5) / 64, tex=0, lod=0.0)
    lv = {0: s.decode_level(0)}
    fb, _ = s.resolve(g, BILINEAR, lv)
    fn, _ = s.resolve(g, NEAREST, lv)
    assert np.array_equal(fb, fn)
    assert np.array_equal(oracle.unpack_frame(fn)[:, :, :3], lv[0])


def test_bilinear_half_texel_is_rounded_average(small_scene):
    s = small_scene
    img = s.decode_level(0).astype(np.int64)
    x, y = np.meshgrid(np.arange(63), np.arange(63))
    g = gb((x + 1.0) / 64, (y + 1.0) / 64)          # s = x + 0.5: weights 128/128
    fb, _ = s.resolve(g, BILINEAR, {0: s.decode_level(0)})
    want = (img[:-1, :-1] + img[:-1, 1:] + img[1:, :-1] + img[1:, 1:]) * 128 * 128
    want = (want + 32768) >> 16
    assert np.array_equal(oracle.unpack_frame(fb)[:, :, :3].astype(np.int64), want)


def test_repeat_addressing(small_scene):
    s = small_scene
    rng = np.random.default_rng(3)
    u = rng.random((16, 16)).astype(np.float32); v = rng.random((16, 16)).astype(np.float32)
    lv = {L: s.decode_level(L) for L in range(len(s.jpegs))}
    for f in (NEAREST, BILINEAR):
        a, _ = s.resolve(gb(u, v), f, lv)
        b, _ = s.resolve(gb(u + 3.0, v - 2.0), f, lv)
        assert np.array_equal(a, b)


def test_constant_texture_constant_frame():
    rgb = np.zeros((64, 64, 3), np.uint8); rgb[...] = (200, 30, 90)
    jp = [encode(rgb, 100, 420)]
    s = oracle.Scene([EncodedTexture(0, 64, 64, 100, 420, jp)])
    col = s.decode_level(0)[0, 0]
    rng = np.random.default_rng(4)
    g = gb(rng.normal(0, 3, (20, 20)), rng.normal(0, 3, (20, 20)), lod=0.0)
    for f in (NEAREST, BILINEAR, TRILINEAR):
        fr, bad = s.resolve(g, f, {0: s.decode_level(0)})
        assert bad == 0 and (oracle.unpack_frame(fr)[:, :, :3] == col).all()


def test_level_selection_and_trilinear_at_integer_lod(small_scene):
    s = small_scene
    lv = {L: s.decode_level(L) for L in range(4)}
    rng = np.random.default_rng(5)
    u = rng.random((8, 8)).astype(np.float32); v = rng.random((8, 8)).astype(np.float32)
    for lod, level in ((-3.0, 0), (0.49, 0), (0.5, 1), (1.2, 1), (2.6, 3), (9.0, 3)):
        a, _ = s.resolve(gb(u, v, lod=lod), BILINEAR, lv)
        # the same level sampled through a one-level texture
        one = oracle.Scene([EncodedTexture(0, 0, 0, 0, 0, [s.textures[0].jpegs[level]])])
        b, _ = one.resolve(gb(u, v), BILINEAR, {0: lv[level]})
        assert np.array_equal(a, b)
    for lod in (0.0, 1.0, 2.0):
        t, _ = s.resolve(gb(u, v, lod=lod), TRILINEAR, lv)
        b, _ = s.resolve(gb(u, v, lod=lod), BILINEAR, lv)
        assert np.array_equal(t, b)


def test_trilinear_blends_rounded_levels(small_scene):
    s = small_scene
    lv = {L: s.decode_level(L) for L in range(4)}
    rng = np.random.default_rng(6)
    u = rng.random((6, 6)).astype(np.float32); v = rng.random((6, 6)).astype(np.float32)
    t, _ = s.resolve(gb(u, v, lod=1.25), TRILINEAR, lv)
    a, _ = s.resolve(gb(u, v, lod=1.0), TRILINEAR, lv)
    b, _ = s.resolve(gb(u, v, lod=2.0), TRILINEAR, lv)
    A = oracle.unpack_frame(a)[..., :3].astype(int); B = oracle.unpack_frame(b)[..., :3].astype(int)
    assert np.array_equal(oracle.unpack_frame(t)[..., :3], (A * 192 + B * 64 + 128) >> 8)


@settings(max_examples=25, deadline=None)
@given(st.integers(0, 2**31 - 1), st.sampled_from([NEAREST, BILINEAR, TRILINEAR]))
def test_mark_is_exactly_the_dependency_set(seed, filt):
    """A block is marked iff the unrounded frame changes when its texels change."""
    tex = make_textures([(seed, 48, 40, 70, 420, 3)], keep_rgb=False)
    s = oracle.Scene(tex)
    rng = np.random.default_rng(seed)
    g = gb(rng.normal(0.5, 0.7, (4, 4)), rng.normal(0.5, 0.7, (4, 4)), lod=rng.uniform(-0.5, 2.5, (4, 4)))
    g["lod"] = np.where(rng.random((4, 4)) < 0.3, np.round(g["lod"]), g["lod"])
    vis, bad = s.mark(g, filt)
    assert bad == 0
    base_f = {L: s.decode_level(L, want_f64=True)[1] for L in range(3)}
    base_b = {L: s.decode_level(L) for L in range(3)}
    _, f0, _ = s.resolve(g, filt, base_b, base_f, want_f64=True)
    marked = set(int(b) for b in vis)
    for b in range(s.n_blocks):
        L = s.level_of_block(b)
        r = b - int(s.blk_base[L])
        if r >= int(s.blk_cols[L] * s.blk_rows[L]):
            continue
        bx, by = r % int(s.blk_cols[L]), r // int(s.blk_cols[L])
        pf = dict(base_f); pf[L] = base_f[L].copy()
        pf[L][16 * by:16 * by + 16, 16 * bx:16 * bx + 16] += 1000.0
        _, f1, _ = s.resolve(g, filt, base_b, pf, want_f64=True)
        assert (np.abs(f1 - f0).max() > 0) == (b in marked), (b, filt)


def test_invalid_pixels(small_scene):
    s = small_scene
    g = gb([[0.1, np.nan, 0.3, 0.2]], [[0.1, 0.2, np.float32(1e12), 0.2]])
    g["tex"][0, 3] = 9
    vis, bad = s.mark(g, BILINEAR)
    assert bad == 3
    fr, bad = s.resolve(g, BILINEAR, {L: s.decode_level(L) for L in range(4)})
    assert bad == 3 and list(fr[0, 1:]) == [oracle.INVALID_TEXEL] * 3
    g["tex"][0, 0] = oracle.BACKGROUND
    fr, _ = s.resolve(g, BILINEAR, {})
    assert fr[0, 0] == 0


# ------------------------------------------------------------------ LRU
@settings(max_examples=60, deadline=None)
@given(st.lists(st.sets(st.integers(0, 40), max_size=12), min_size=1, max_size=12), st.integers(12, 30))
def test_lru_invariants(frames, cap):
    sim = oracle.LruSim(cap)
    resident_prev = set()
    seen = set()
    unbounded = oracle.LruSim(10**9)
    for f, V in enumerate(frames):
        last_before = dict(sim.last_used)
        new, ev = sim.step(f, V)
        R = set(sim.last_used)
        assert len(R) <= cap
        assert V <= R
        assert set(new) == V - resident_prev
        assert not (set(ev) & V) and set(ev) <= resident_prev
        kept = (resident_prev - set(ev)) - V
        for e in ev:                                  # the evicted are the oldest
            for k in kept:
                assert (last_before[e], e) < (last_before[k], k)
        unew, _ = unbounded.step(f, V)
        assert set(unew) == V - seen
        seen |= V
        resident_prev = R


def test_lru_hand_example_with_frame_gaps():
    """Hand-worked trace (Update Cache with a capacity): frames far apart, so
    that ages exceed any small age cap; eviction must follow last use, not
    block id.  Capacity 3."""
    sim = oracle.LruSim(3)
    assert sim.step(0, {10}) == ([10], [])
    assert sim.step(500, {3}) == ([3], [])
    assert sim.step(600, {7}) == ([7], [])
    # f = 3000: resident 10 (used at 0), 3 (500), 7 (600); 10 is the oldest
    # although its id is the largest
    assert sim.step(3000, {5}) == ([5], [10])
    # f = 10**6: two new blocks, 5 stays visible; 3 then 7 are the oldest
    assert sim.step(10**6, {5, 1, 2}) == ([1, 2], [3, 7])
    # equal last use: the smaller block id goes first
    assert sim.step(10**6 + 1, {8}) == ([8], [1])
    assert sim.step(4_000_000_000, {9}) == ([9], [2])


@settings(max_examples=60, deadline=None)
@given(st.lists(st.tuples(st.integers(1, 3_000_000), st.sets(st.integers(0, 40), max_size=12)), min_size=1,
                max_size=10), st.integers(12, 30))
def test_lru_oldest_first_with_large_gaps(steps, cap):
    """Brute force per frame: the evicted blocks are the |new| - free
    non-visible resident blocks of smallest (last use, id), for frame
    numbers far apart."""
    sim = oracle.LruSim(cap)
    f = 0
    last = {}
    for gap, V in steps:
        f += gap
        R = set(last)
        new = sorted(V - R)
        free = cap - len(R)
        need = max(0, len(new) - free)
        keys = sorted((last[b], b) for b in R - V)
        want_ev = sorted(b for _, b in keys[:need])
        got_new, got_ev = sim.step(f, V)
        assert got_new == new and got_ev == want_ev
        for b in want_ev:
            del last[b]
        for b in V:
            last[b] = f
        assert dict(sim.last_used) == last


def _level_image(rng, s, L):
    return rng.integers(0, 256, (int(s.lev_h[L]), int(s.lev_w[L]), 3)).astype(np.uint8)


@pytest.mark.parametrize("frac,fx", [(0.25, 64), (0.75, 192), (1 / 512 - 2 ** -16, 0), (1 / 512, 1),
                                     (1 / 512 + 2 ** -16, 1), (3 / 512 - 2 ** -16, 1), (3 / 512, 2),
                                     (3 / 512 + 2 ** -16, 2), (1 - 2 ** -10, 256)])
def test_bilinear_weights_at_general_fractions(small_scene, frac, fx):
    """Closed form of the 8-bit horizontal weight f = floor(frac * 256 + 0.5)
    (values written out by hand, ties at odd multiples of 1/512 rounding up):
    with v at texel centres the pixel is (t0 (256 - f) + t1 f + 128) >> 8 per
    channel, t0 = texel floor(s), t1 the next one (repeat-wrapped)."""
    s = small_scene
    rng = np.random.default_rng(8)
    img = _level_image(rng, s, 0)
    x, y = np.meshgrid(np.arange(64), np.arange(64))
    u = ((x + 0.5 + frac) / 64).astype(np.float32)    # s = u*64 - 0.5 = x + frac, exact in fp32
    assert np.all(u * np.float32(64) - np.float32(0.5) == (x + frac).astype(np.float32))
    fb, bad = s.resolve(gb(u, (y + 0.5) / 64), BILINEAR, {0: img})
    assert bad == 0
    t0 = img.astype(np.int64)
    t1 = np.roll(t0, -1, axis=1)
    want = (t0 * (256 - fx) + t1 * fx + 128) >> 8
    assert np.array_equal(oracle.unpack_frame(fb)[:, :, :3].astype(np.int64), want)


def test_bilinear_weights_in_both_axes(small_scene):
    """s = x + 1/4 and t = y + 3/4: weights 192/64 across, 64/192 down."""
    s = small_scene
    img = _level_image(np.random.default_rng(9), s, 0).astype(np.int64)
    x, y = np.meshgrid(np.arange(64), np.arange(64))
    fb, _ = s.resolve(gb((x + 0.75) / 64, (y + 1.25) / 64), BILINEAR, {0: img.astype(np.uint8)})
    r = lambda a, dy, dx: np.roll(np.roll(a, -dy, axis=0), -dx, axis=1)
    acc = (img * 192 * 64 + r(img, 0, 1) * 64 * 64 + r(img, 1, 0) * 192 * 192 + r(img, 1, 1) * 64 * 192)
    assert np.array_equal(oracle.unpack_frame(fb)[:, :, :3].astype(np.int64), (acc + 32768) >> 16)


@pytest.mark.parametrize("lod,t", [(1.3, 77), (1.7, 179), (2.0 + 1 / 512, 1), (1.0 + 1 / 1024, 0)])
def test_trilinear_weight_at_non_dyadic_lod(small_scene, lod, t):
    """t = floor(frac(lod) * 256 + 0.5) in fp32: lod 1.3 -> 76.8 -> 77, lod
    1.7 -> 179.2 -> 179, a tie at 1/512 rounds up, 1/1024 rounds down; the
    pixel is (a (256 - t) + b t + 128) >> 8 of the two levels' bilinear
    results."""
    s = small_scene
    rng = np.random.default_rng(10)
    lv = {L: _level_image(rng, s, L) for L in range(4)}
    u = rng.random((8, 8)).astype(np.float32); v = rng.random((8, 8)).astype(np.float32)
    lo = int(np.floor(lod))
    tr, _ = s.resolve(gb(u, v, lod=np.float32(lod)), TRILINEAR, lv)
    a, _ = s.resolve(gb(u, v, lod=float(lo)), BILINEAR, lv)
    b, _ = s.resolve(gb(u, v, lod=float(lo + 1)), BILINEAR, lv)
    A = oracle.unpack_frame(a)[..., :3].astype(int); B = oracle.unpack_frame(b)[..., :3].astype(int)
    assert np.array_equal(oracle.unpack_frame(tr)[..., :3], (A * (256 - t) + B * t + 128) >> 8)


@pytest.mark.parametrize("threads", [1, 3])
def test_cpu_ondemand_baseline_equals_full_render(threads):
    """The CPU on-demand baseline (decode only the marked blocks through the
    oracle's per-MCU index, then resolve) gives the plain definition's
    frame bit for bit, with 4:2:0 and 4:4:4 levels and trilinear taps."""
    wl = configs.heavy(seed=34, n_tex=6, sides=(64, 128), W=160, H=100, n_quads=16, n_frames=1)
    s = oracle.Scene(wl.textures)
    od = oracle.OnDemand(s)
    ref, vis, _ = s.render(wl.views[0], wl.filter)
    f, t, n, bad = od.frame(wl.views[0], wl.filter, threads)
    assert bad == 0 and n == len(vis)
    assert np.array_equal(f, ref)


BILINEAR_CLAMPED, NO_MIP = oracle.BILINEAR_CLAMPED, oracle.NO_MIP


def test_clamped_bilinear_marks_the_centre_block_only(small_scene):
    """Centre-only marking: the clamped filter's footprint is the block of
    the nearest filter's texel, so it marks exactly what nearest marks."""
    s = small_scene
    rng = np.random.default_rng(12)
    g = gb(rng.normal(0.5, 1.5, (24, 24)), rng.normal(0.5, 1.5, (24, 24)), tex=rng.integers(0, 2, (24, 24)),
           lod=rng.uniform(-1, 4, (24, 24)))
    a, _ = s.mark(g, BILINEAR_CLAMPED)
    b, _ = s.mark(g, NEAREST)
    assert np.array_equal(a, b)


def test_clamped_bilinear_closed_forms(small_scene):
    """Inside a block the clamped filter is bilinear; across a block border
    the tap in the other block reads the centre texel's column (or row):
    s = 15.75 has taps 15 and 16 with weights 64/192 and centre texel 16
    (block 1), so the pixel is texel 16; s = 15.25 (centre 15, block 0)
    gives texel 15; s = 16.25 is inside block 1 and stays bilinear."""
    s = small_scene
    rng = np.random.default_rng(13)
    img = _level_image(rng, s, 0)
    t = img.astype(np.int64)
    y = np.arange(64)
    lv = {0: img}

    def px(sx):
        g = gb(np.full(64, (sx + 0.5) / 64), (y + 0.5) / 64)
        f, bad = s.resolve(g, BILINEAR_CLAMPED, lv)
        assert bad == 0
        return oracle.unpack_frame(f)[0, :, :3].astype(np.int64)

    assert np.array_equal(px(15.75), t[:, 16])
    assert np.array_equal(px(15.25), t[:, 15])
    assert np.array_equal(px(16.25), (t[:, 16] * 192 + t[:, 17] * 64 + 128) >> 8)
    # and across the wrap at the last column: s = 63.75 -> centre 0 (block 0), tap 63 clamps to 0
    assert np.array_equal(px(63.75), t[:, 0])
    # interior pixels of random G-buffers equal plain bilinear
    u = rng.uniform(0, 1, (16, 16)).astype(np.float32); v = rng.uniform(0, 1, (16, 16)).astype(np.float32)
    sx = u * np.float32(64) - np.float32(0.5); sy = v * np.float32(64) - np.float32(0.5)
    inside = ((np.floor(sx) % 64) // 16 == ((np.floor(sx) + 1) % 64) // 16) & \
             ((np.floor(sy) % 64) // 16 == ((np.floor(sy) + 1) % 64) // 16)
    a, _ = s.resolve(gb(u, v), BILINEAR_CLAMPED, lv)
    b, _ = s.resolve(gb(u, v), BILINEAR, lv)
    assert inside.sum() > 100 and np.array_equal(a[inside], b[inside])


@pytest.mark.parametrize("filt", [NEAREST, BILINEAR, TRILINEAR, BILINEAR_CLAMPED])
def test_no_mip_samples_level_zero(small_scene, filt):
    """Mip mapping off: the same as every pixel at lod 0 (level 0 only)."""
    s = small_scene
    rng = np.random.default_rng(14)
    g = gb(rng.normal(0.5, 1.5, (20, 20)), rng.normal(0.5, 1.5, (20, 20)), tex=rng.integers(0, 2, (20, 20)),
           lod=rng.uniform(-1, 6, (20, 20)))
    g0 = g.copy()
    g0["lod"] = 0.0
    lv = {L: s.decode_level(L) for L in range(len(s.jpegs))}
    a, _ = s.resolve(g, filt | NO_MIP, lv)
    b, _ = s.resolve(g0, filt, lv)
    assert np.array_equal(a, b)
    va, _ = s.mark(g, filt | NO_MIP)
    vb, _ = s.mark(g0, filt)
    assert np.array_equal(va, vb)


def test_evict_invisible_hand_trace():
    """The paper's policy: whatever a frame does not read leaves the cache."""
    sim = oracle.EvictInvisibleSim(10)
    assert sim.step({1, 2, 3}) == ([1, 2, 3], [])
    assert sim.step({2, 3, 4}) == ([4], [1])
    assert sim.step({5}) == ([5], [2, 3, 4])
    assert sim.step({5}) == ([], [])
    assert sim.step({1, 5}) == ([1], [])        # 1 was evicted two frames ago: decoded again
    with pytest.raises(oracle.OracleError):
        sim.step(set(range(11)))
