"""GPU parity of the batched form: many views per launch (one shared block
bitmask, so blocks are deduplicated across views), launch knobs that must
not change any result, and the frame captured into a HIP graph and
replayed (plain and with the LRU cache counting its own frames)."""
import numpy as np
import pytest

import oracle
from oracle import parity
from paper_2510_08166_amd.synth import configs

from gpu_common import full_parity, run

pytestmark = pytest.mark.gpu


def test_batched_small_views_parity(gpu):
    wl = configs.batched_small()
    assert len(wl.views) == 5
    full_parity(wl)


def test_more_views_than_one_launch_holds(gpu):
    """18 views: the view table of one launch holds 16, so mark and resolve
    take two launches; the shared bitmask still dedupes across them."""
    wl = configs.batched(seed=17, n_pool=6, sides=(64, 128), n_pairs=1, eye=(40, 24), n_mono=16, mono_w=(32, 96),
                         tex_per_scene=(1, 4), quads_per_mpx=4000, filt=configs.FILTER_TRILINEAR, name="18 views")
    assert len(wl.views) == 18
    full_parity(wl)


@pytest.mark.parametrize("knobs", [dict(mark_groups=7, resolve_groups=5),
                                   dict(mark_groups=16, resolve_groups=24, flags=1),
                                   dict(flags=1),
                                   dict(decode_groups=3, idct_groups=2),
                                   dict(decode_groups=16, idct_groups=8),
                                   dict(wide_bits=1), dict(wide_bits=0xFFFFFFFF)])
def test_launch_knobs_do_not_change_results(gpu, knobs):
    from paper_2510_08166_amd import jpt
    wl = configs.batched_small(seed=8, filt=configs.FILTER_TRILINEAR)
    _, ctr0, items0, coef0, tiles0, frames0 = run(wl)
    t = jpt.TuningC()
    for k, v in knobs.items():
        setattr(t, k, v)
    for mode in (jpt.IDCT_MFMA_F16, jpt.IDCT_SCALAR_F32):
        _, ctr, items, coef, tiles, frames = run(wl, mode, tuning=t)
        assert np.array_equal(ctr[:7], ctr0[:7]) and np.array_equal(items, items0)
        assert np.array_equal(coef, coef0)
        if mode == jpt.IDCT_MFMA_F16:
            assert np.array_equal(tiles, tiles0)
            for f, f0 in zip(frames, frames0):
                assert np.array_equal(f, f0)


def test_graph_replay_matches_eager(gpu):
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.batched_small(seed=9)
    r = jpt.Renderer(wl.textures, wl.views, wl.filter)
    r.render()
    torch.cuda.synchronize()
    ref = [r.views.frame_host(i) for i in range(r.views.n)]
    ref_items = r.frame.work_items()
    s = torch.cuda.Stream()
    g = r.capture(s)
    for rep in range(3):
        # eager work between replays: wipe the outputs
        for f in r.views.frames:
            f.zero_()
        r.frame.work.zero_()
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        assert np.array_equal(r.frame.work_items(), ref_items), "replay %d" % rep
        for i in range(r.views.n):
            assert np.array_equal(r.views.frame_host(i), ref[i]), "replay %d view %d" % (rep, i)
    g.close()
    # the captured frame agrees with the oracle too
    osc = oracle.Scene(wl.textures)
    for gb, f in zip(wl.views, ref):
        full, _, bad = osc.render(gb, wl.filter)
        assert bad == 0 and parity.frame_diff(f, full) <= 1


def _graph_vs_eager(r, n_rep=3):
    """Replay r's captured frame n_rep times (wiping outputs eagerly between
    replays) and compare everything it produced with the eager frame."""
    import torch
    from paper_2510_08166_amd import jpt
    r.render()
    torch.cuda.synchronize()
    ctr0 = r.frame.counters_host().copy()
    items0 = r.frame.work_items()
    n_new = min(int(ctr0[jpt.CTR_NEW]), r.cache.n_slots)
    tex0 = r.cache.texels[: n_new * 256].cpu().numpy()
    slots0 = r.cache.slot_of.cpu().numpy()
    frames0 = [r.views.frame_host(i) for i in range(r.views.n)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = r.capture(s)
    for rep in range(n_rep):
        for f in r.views.frames:
            f.zero_()
        r.frame.work.zero_()
        r.frame.counters.zero_()
        r.cache.texels.zero_()
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        ctr = r.frame.counters_host()
        assert np.array_equal(ctr[:7], ctr0[:7]), "replay %d counters %s vs %s" % (rep, ctr[:7], ctr0[:7])
        assert np.array_equal(r.frame.work_items(), items0), "replay %d" % rep
        assert np.array_equal(r.cache.texels[: n_new * 256].cpu().numpy(), tex0), "replay %d" % rep
        used = items0 & 0x7FFFFFFF
        assert np.array_equal(r.cache.slot_of.cpu().numpy()[used >> 2], slots0[used >> 2])
        for i in range(r.views.n):
            assert np.array_equal(r.views.frame_host(i), frames0[i]), "replay %d view %d" % (rep, i)
    g.close()
    return ctr0, frames0


@pytest.mark.parametrize("case", ["420 trilinear", "444 bilinear", "corrupt", "capacity", "background"])
def test_fused_graph_matches_eager(gpu, case):
    """The captured frame with the fused decode (the benchmark's path)
    produces exactly the eager frame: work list, counters, slots, texels and
    framebuffers, also for corrupt streams, exhausted capacity and a
    background-only frame."""
    import torch
    from paper_2510_08166_amd import jpt
    kw = {}
    if case == "444 bilinear":
        wl = configs.quad_scene(25, 3, 200, 50, 95, 4, 160, 120, 12, sampling=444, filt=configs.FILTER_BILINEAR)
    else:
        wl = configs.batched_small(seed=11, filt=configs.FILTER_TRILINEAR)
    if case == "capacity":
        kw = dict(max_items=100, n_slots=60)
    if case == "background":
        for g in wl.views:
            g["tex"] = 0xFFFFFFFF
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, idct_mode=jpt.IDCT_FUSED_F32, **kw)
    if case == "corrupt":
        r.scene.streams.fill_(0xFF)
    ctr, frames = _graph_vs_eager(r)
    if case == "corrupt":
        assert ctr[jpt.CTR_ERROR] & jpt.ERR_CORRUPT and ctr[jpt.CTR_ERROR_ITEM] == 0
    elif case == "capacity":
        assert ctr[jpt.CTR_ERROR] & jpt.ERR_CAPACITY and ctr[jpt.CTR_ITEMS] == 100
    elif case == "background":
        assert ctr[jpt.CTR_ITEMS] == 0 and ctr[jpt.CTR_ERROR] == 0
    else:
        assert ctr[jpt.CTR_ERROR] == 0
        osc = oracle.Scene(wl.textures)
        for gb, f in zip(wl.views, frames):
            full, _, bad = osc.render(gb, wl.filter)
            assert bad == 0 and parity.frame_diff(f, full) <= 1


def test_lru_graph_counts_frames(gpu):
    """LRU cache inside a replayed graph (frame number kept on the device):
    per frame the same decoded sets, evictions and resident sets as the
    oracle's simulator."""
    import torch
    from paper_2510_08166_amd import jpt
    wl = configs.heavy(seed=32, n_tex=10, sides=(64, 128, 256), W=256, H=160, n_quads=30, n_frames=5)
    osc = oracle.Scene(wl.textures)
    vis_sets = [parity.visible_blocks(osc, [gb], wl.filter) for gb in wl.views]
    cap = max(len(v) for v in vis_sets) + 16
    r = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, n_slots=cap, policy=jpt.CACHE_LRU)
    s = torch.cuda.Stream()
    g = r.capture(s)
    assert r.frame_no == jpt.FRAME_AUTO
    sim = oracle.LruSim(cap)
    for f, gb in enumerate(wl.views):
        r.set_views([gb])
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        ctr = r.frame.counters_host()
        new, ev = sim.step(f, vis_sets[f])
        print("frame %d: visible %d new %d evicted %d" % (f, ctr[jpt.CTR_VISIBLE], ctr[jpt.CTR_NEW],
                                                         ctr[jpt.CTR_EVICTED]), flush=True)
        assert ctr[jpt.CTR_ERROR] == 0
        assert np.array_equal(r.frame.work_items(), parity.expected_items(osc, np.array(new, np.uint32)))
        assert ctr[jpt.CTR_EVICTED] == len(ev)
        assert np.array_equal(r.cache.resident_blocks(), np.array(sorted(sim.last_used), np.uint32))
        full, _, _ = osc.render(gb, wl.filter)
        assert parity.frame_diff(r.views.frame_host(), full) <= 1
    g.close()


def test_autotuner_keeps_results_and_caches(gpu, tmp_path):
    from paper_2510_08166_amd import jpt, tune
    wl = configs.batched_small(seed=10)
    r = jpt.Renderer(wl.textures, wl.views, wl.filter)
    r.render()
    ref = tune.frame_digest(r)
    path = str(tmp_path / "tune.json")
    t = tune.tune(r, reps=3, cache_path=path)
    r.render()
    assert tune.frame_digest(r) == ref
    r2 = jpt.Renderer(wl.textures, wl.views, wl.filter, host=r.host)
    t2 = tune.tune(r2, cache_path=path)          # served from the cache file
    assert tune.to_dict(t2) == tune.to_dict(t)
