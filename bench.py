#!/usr/bin/env python3
"""Benchmark of the on-demand JPEG texture path on one MI355X.

One step = one 1920x1080 frame through the whole per-frame path on resident
inputs: mark + compact (jpt_mark_blocks), entropy decode with dequant +
IDCT + colour in the same kernel (jpt_decode_blocks, fused; --idct mfma or
scalar: jpt_entropy_decode then jpt_idct_color) and filtered resolve
(jpt_resolve).  Workload: 32 textures of 2048^2 (q 50-90, 4:2:0,
8 mip levels), G-buffer from 200 seeded quads, bilinear, no cache (every
visible block is decoded every frame).

Prints one JSON line.  The value is milliseconds per frame (wall clock over
the timed steps, bracketed by device synchronisation); per-kernel times come
from HIP events recorded on the stream the kernels run on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/frame visible-block decode+resolve @1080p; Mblocks/s; fwd+bwd ms; HBM GB/s"
# the arithmetic of the path: integer entropy decode, index and blends; fp32 IDCT and colour
DTYPE = "int32+fp32"
HBM_PEAK_GBS = 8000.0
FRAME1080 = "1080p: 32 x 2048^2 q50-90 4:2:0 8 levels, 200 quads, bilinear"  # configs.frame1080().name

# HBM traffic per launch of a phase's kernel on the 1080p frame (only that
# workload: the entries do not apply to others), from
# `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` (KiB per dispatch), each
# scaled by what the same counter reads for one elementwise add of 1 GiB in
# and 1 GiB out (fetch_scale, write_scale).  An entry holds only for the
# kernel source it was measured on (sha256 prefix of the file); otherwise the
# bench reports traffic as null.
TRAFFIC = {
    # profiles/frame1080_hbm_traffic.txt (k_entropy<true, true, false> and k_resolve<1u, 2, true, false>,
    # fused decode, 1080p frame)
    "entropy": {"file": "paper_2510_08166_amd/csrc/decode.hip", "sha": "6ea4512cf277df21",
                "fetch_kib": 447.7, "write_kib": 4290.0, "fetch_scale": 2.0, "write_scale": 1.0},
    "resolve": {"file": "paper_2510_08166_amd/csrc/resolve.hip", "sha": "6b6e10c0c7960d85",
                "fetch_kib": 21393.0, "write_kib": 8100.0, "fetch_scale": 2.0, "write_scale": 1.0},
}


def source_sha(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(phase, workload):
    t = TRAFFIC.get(phase)
    if workload != FRAME1080 or not t or source_sha(t["file"]) != t["sha"]:
        return None
    return int(1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(r, ctr):
    """Bytes the method itself must move per frame (implementation scratch such as
    the coefficient round trip excluded).  Returns a dict per phase."""
    import numpy as np
    from paper_2510_08166_amd import jpt
    P = r.views.n_pixels
    n_new = int(ctr[jpt.CTR_NEW]); n_vis = int(ctr[jpt.CTR_VISIBLE]); n_items = int(ctr[jpt.CTR_ITEMS])
    items = r.frame.work_items()
    host = r.host
    # compressed bytes of the decoded MCUs (from the records) + their record share
    comp = 0.0
    bits = 0
    blocks = (items & 0x7FFFFFFF) >> 2
    lev = host.word_level[blocks >> 5]
    for L in np.unique(lev):
        li = host.levels[int(L)]
        inf = li.info
        rec = li.records.view(np.uint32).reshape(-1, 16)
        starts = np.zeros(inf.n_mcu + 1, np.int64)
        g = np.arange(inf.n_mcu) // 9; j = np.arange(inf.n_mcu) % 9
        rel = np.where(j == 0, 0, (rec[g, 1 + (np.maximum(j, 1) - 1) // 2] >> (16 * ((np.maximum(j, 1) - 1) % 2)))
                       & 0xFFFF)
        starts[:-1] = rec[g, 0].astype(np.int64) + rel
        starts[-1] = inf.stream_bits
        sel = blocks[lev == L] - host.blk_base[int(L)]
        bx = sel % inf.blk_cols; by = sel // inf.blk_cols
        mcu = by * inf.mcu_cols + bx
        nb = int((starts[mcu + 1] - starts[mcu]).sum())
        bits += nb
        comp += nb / 8.0 + 64.0 / 9.0 * len(mcu)
    nbw = host.n_blocks / 8.0
    return dict(
        mark=P * 16 + nbw,                       # G-buffer read, bitmask set
        compact=2 * nbw + n_items * 4 + n_new * 4,
        entropy=comp + n_items * 768,            # stream + records in, coefficients out
        idct=n_items * 768 + n_new * 1024,       # coefficients in, texels out
        resolve=P * 16 + P * 4 + n_vis * 1024,   # G-buffer, framebuffer, one read of each visible block
        method=P * 16 * 2 + P * 4 + comp + n_new * 1024 + n_vis * 1024 + 2 * nbw,
        compressed=comp,
        stream_bits=bits,                        # entropy-coded bits of the decoded MCUs
    )


def item_bits(r):
    """Entropy-coded bits of each listed work item's MCU (from the index records)."""
    import numpy as np
    items = r.frame.work_items()
    host = r.host
    blocks = (items & 0x7FFFFFFF) >> 2
    q = items & 3
    lev = host.word_level[blocks >> 5]
    out = np.zeros(len(items), np.int64)
    for L in np.unique(lev):
        inf = host.levels[int(L)].info
        rec = host.levels[int(L)].records.view(np.uint32).reshape(-1, 16)
        g = np.arange(inf.n_mcu) // 9; j = np.arange(inf.n_mcu) % 9
        jm = np.maximum(j, 1) - 1
        rel = np.where(j == 0, 0, (rec[g, 1 + jm // 2] >> (16 * (jm % 2))) & 0xFFFF)
        starts = np.zeros(inf.n_mcu + 1, np.int64)
        starts[:-1] = rec[g, 0].astype(np.int64) + rel
        starts[-1] = inf.stream_bits
        sel = lev == L
        r_ = blocks[sel] - host.blk_base[int(L)]
        bx = r_ % inf.blk_cols; by = r_ // inf.blk_cols
        if inf.sampling == 444:
            mx = 2 * bx + (q[sel] & 1); my = 2 * by + (q[sel] >> 1)
            ok = (mx < inf.mcu_cols) & (my < inf.mcu_rows)
            m = np.where(ok, my * inf.mcu_cols + mx, 0)
            out[sel] = np.where(ok, starts[m + 1] - starts[m], 0)
        else:
            m = by * inf.mcu_cols + bx
            out[sel] = starts[m + 1] - starts[m]
    return out


def chain_floor(r, steps):
    """The decode's latency floor on this frame: the kernel run on the
    frame's longest MCU alone (the frame cannot finish before that MCU's
    symbol chain does), and on no item (launch and prologue), next to the
    frame's own decode time."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt
    bits = item_bits(r)
    n = len(bits)
    i = int(np.argmax(bits))
    work = r.frame.work[:n].clone()
    ctr = r.frame.counters.clone()

    def timed(k):
        r.frame.counters[jpt.CTR_ITEMS] = k
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in ev:
            e0.record()
            r.decode()
            e1.record()
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))

    full = timed(n)
    r.frame.work[0] = work[i]
    alone = timed(1)
    empty = timed(0)
    r.frame.work[:n].copy_(work)
    r.frame.counters.copy_(ctr)
    torch.cuda.synchronize()
    return {"longest_mcu_bits": int(bits[i]), "median_mcu_bits": int(np.median(bits)),
            "decode_ms": round(full, 4), "longest_mcu_alone_ms": round(alone, 4), "no_item_ms": round(empty, 4),
            "frac_of_floor": round(alone / full, 3)}


def cpu_baseline(wl, budget_s=20.0):
    """The oracle as written (single thread): visible set, full sequential
    decode of every touched level, resolve.  Bounded sample: levels are
    decoded in order until the time budget is spent; the decode time is
    scaled by the touched levels' texel count, mark and resolve run in full."""
    import numpy as np
    import oracle
    osc = oracle.Scene(wl.textures)
    g = wl.views[0]
    t0 = time.perf_counter()
    vis, _ = osc.mark(g, wl.filter)
    t_mark = time.perf_counter() - t0
    touched = sorted(osc.levels_of_blocks(vis))
    tex_total = sum(int(osc.lev_w[L]) * int(osc.lev_h[L]) for L in touched)
    done_tex = 0
    levels = {}
    t0 = time.perf_counter()
    for L in touched:
        levels[L] = osc.decode_level(L)
        done_tex += int(osc.lev_w[L]) * int(osc.lev_h[L])
        if time.perf_counter() - t0 > budget_s:
            break
    t_dec = time.perf_counter() - t0
    full = len(levels) == len(touched)
    t_res = 0.0
    if full:
        t0 = time.perf_counter()
        osc.resolve(g, wl.filter, levels)
        t_res = time.perf_counter() - t0
    else:
        # resolve cost measured with the undecoded levels read as zeros
        t0 = time.perf_counter()
        osc.resolve(g, wl.filter, {L: levels.get(L, np.zeros((int(osc.lev_h[L]), int(osc.lev_w[L]), 3), np.uint8))
                                   for L in touched})
        t_res = time.perf_counter() - t0
    ms = 1000.0 * (t_mark + t_dec * tex_total / max(done_tex, 1) + t_res)
    sample = ("mark + resolve of the full frame; sequential decode of %d of %d touched levels (%.1f%% of their "
              "texels), decode time scaled by texel count" % (len(levels), len(touched), 100.0 * done_tex / tex_total))
    return {"value": round(ms, 1), "unit": "ms/frame", "cores": 1, "kind": "oracle", "sample": sample}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_ondemand_baseline(wl, gpu_ms, budget_s=15.0):
    """The CPU on-demand baseline: the oracle's routines doing the paper's
    per-frame method (mark, decode only the marked blocks' MCUs by random
    access through the oracle's own per-MCU index, resolve), on one thread
    and on all the host cores the box grants (at most 16).  The index is
    recorded before timing.  Median over repeated frames within the budget."""
    import numpy as np
    import oracle
    osc = oracle.Scene(wl.textures)
    t0 = time.perf_counter()
    od = oracle.OnDemand(osc)
    log("CPU on-demand index recorded in %.1f s" % (time.perf_counter() - t0))
    g = wl.views[0]
    ref = None
    out = {}
    n_all = max(1, min(os.cpu_count() or 1, 16))
    for threads in sorted({1, n_all}):
        times, t_start = [], time.perf_counter()
        while len(times) < 7 and (len(times) < 2 or time.perf_counter() - t_start < budget_s / 2):
            f, t, n, bad = od.frame(g, wl.filter, threads)
            if bad:
                raise SystemExit("CPU on-demand baseline: %d bad pixels or MCUs" % bad)
            if ref is None:
                ref = f
            elif not np.array_equal(f, ref):
                raise SystemExit("CPU on-demand baseline differs between thread counts")
            times.append(t)
        med = np.median(np.array(times), axis=0) * 1000.0
        out["threads_%d" % threads] = {"ms_per_frame": round(float(med.sum()), 2),
                                       "mark_ms": round(float(med[0]), 2), "list_ms": round(float(med[1]), 3),
                                       "decode_ms": round(float(med[2]), 2), "resolve_ms": round(float(med[3]), 2),
                                       "frames": len(times)}
    best = out["threads_%d" % n_all]["ms_per_frame"]
    out.update({"unit": "ms/frame", "cores_all": n_all, "os_cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
                "blocks_decoded": n, "kind": "oracle routines, on-demand (mark, random-access decode, resolve)",
                "gpu_speedup_vs_all_cores": round(best / gpu_ms, 1)})
    return out


def time_graph(r, steps, warmup):
    """Capture one frame of every view (jpt_graph_capture) on a side stream and
    time `steps` replays, back to back with nothing between them (wall clock
    from a synchronised start to a synchronised end); then `steps` more with
    a timing event after each, for the per-frame GPU times (an event between
    frames costs about 5 us of its own, so the wall clock comes from the
    first loop).  Returns (wall ms per frame, per-frame GPU ms)."""
    import numpy as np
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = r.capture(side)
    for _ in range(warmup):
        g.launch()
    side.synchronize()
    with torch.cuda.stream(side):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch()
        side.synchronize()
        wall = time.perf_counter() - t0
        gev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        gev[0].record(side)
        for s_ in range(steps):
            g.launch()
            gev[s_ + 1].record(side)
        side.synchronize()
    g.close()
    gpu = np.array([gev[i].elapsed_time(gev[i + 1]) for i in range(steps)])
    return 1000.0 * wall / steps, gpu


def time_cold(r, steps, warmup=3):
    """Frames with a cold cache hierarchy: before each frame a 512 MiB
    scratch buffer is read and written on the same stream (twice the
    MI355X's 256 MiB last-level cache), so no input of the frame is cached
    when it starts.  Returns per-frame GPU ms from events around the frame
    alone (the same instrumentation as the warm per-frame times)."""
    import numpy as np
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = r.capture(side)
    with torch.cuda.stream(side):
        scratch = torch.zeros((512 << 20) // 4, dtype=torch.int32, device="cuda")
        for _ in range(warmup):
            scratch.add_(1)
            g.launch()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in ev:
            scratch.add_(1)
            e0.record(side)
            g.launch()
            e1.record(side)
        side.synchronize()
    g.close()
    del scratch
    return np.array([e0.elapsed_time(e1) for e0, e1 in ev])


def time_phases(r, steps):
    """Eager frames with HIP events between the four C-ABI calls, all on the
    current stream: per-phase GPU milliseconds, median over steps."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fused = r.idct_mode == jpt.IDCT_FUSED_F32
    for e in evs:
        e[0].record()
        r.mark()
        e[1].record()
        if fused:  # one kernel: entropy decode, IDCT and colour (the IDCT phase is empty)
            r.decode()
            e[2].record()
        else:
            jpt.entropy_decode(r.scene, r.frame, r.tuning)
            e[2].record()
            jpt.idct_color(r.scene, r.frame, r.cache, r.idct_mode, r.tuning)
        e[3].record()
        r.resolve()
        e[4].record()
    torch.cuda.synchronize()
    eager_ms = 1000.0 * (time.perf_counter() - t0) / steps
    ph = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in evs])
    return eager_ms, np.median(ph, axis=0)


PHASES = ["mark+compact", "entropy", "idct", "resolve"]


def time_repeated(r, phase, reps=60):
    """Average GPU milliseconds of one launch of a phase's C-ABI call (the
    decode and the resolve rewrite the same outputs each time), from HIP
    events around `reps` launches back to back on the current stream, so
    that the events' own cost is spread over them."""
    import torch
    call = {"entropy": r.decode, "resolve": r.resolve, "mark+compact": r.mark}[phase]
    for _ in range(3):
        call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


IDCT_MODES = {"fused": 2, "mfma": 0, "mfma_bf16": 3, "scalar": 1}


def plain_form(args, wl, label, policy=0, n_slots=None):
    """The plain form on one workload: one step = one frame of all its views."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt
    t0 = time.perf_counter()
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, device="cuda:0", policy=policy, n_slots=n_slots,
                     idct_mode=IDCT_MODES[args.idct])
    torch.cuda.synchronize()
    log("index built and uploaded in %.1f s" % (time.perf_counter() - t0))
    if policy == jpt.CACHE_LRU:
        raise SystemExit("use the heavy leg for LRU")
    for _ in range(args.warmup):
        r.render()
    torch.cuda.synchronize()
    ctr = r.frame.counters_host().copy()
    if ctr[jpt.CTR_ERROR]:
        raise SystemExit("device error flags %x" % ctr[jpt.CTR_ERROR])
    ms_per_step, gpu_frame = time_graph(r, args.steps, args.warmup)
    ctr2 = r.frame.counters_host()
    if ctr2[jpt.CTR_ERROR] or ctr2[jpt.CTR_NEW] != ctr[jpt.CTR_NEW]:
        raise SystemExit("graph replay disagrees with eager launches")
    cold = time_cold(r, args.steps)
    eager_ms, med = time_phases(r, args.steps)
    ab = algorithmic_bytes(r, ctr)
    fused = r.idct_mode == jpt.IDCT_FUSED_F32
    ab_phase = {"mark+compact": ab["mark"] + ab["compact"],
                "entropy": ab["compressed"] + int(ctr[jpt.CTR_NEW]) * 1024 if fused else ab["entropy"],
                "idct": 0 if fused else ab["idct"], "resolve": ab["resolve"]}
    n_items = int(ctr[jpt.CTR_ITEMS]); n_du = n_items * 6
    # the fused decode is one kernel: the "idct" phase between its two events is empty
    dec_ms = float(med[1]) if fused else float(med[1] + med[2])
    # the dominant single kernel (mark+compact is two launches)
    single = [i for i, n in enumerate(PHASES) if n != "mark+compact"]
    dom = PHASES[max(single, key=lambda i: med[i])]
    # its launch duration: events around many launches (one pair per launch adds
    # about 2 us to a launch of 20); the phase medians above keep one pair each
    dom_ms = time_repeated(r, dom) if dom != "idct" else float(med[PHASES.index(dom)])
    achieved = ab_phase[dom] / (dom_ms * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, wl.name),
            "algorithmic_bytes_per_launch": int(ab_phase[dom]), "avg_launch_ms": round(dom_ms, 4)}
    out = {
        "metric": METRIC, "value": round(ms_per_step, 4), "unit": "ms/frame", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE,
        "data": "synthetic", "config": {"workload": label, "decode": args.idct, "views": r.views.n, "pixels": r.views.n_pixels,
                   "visible_blocks": int(ctr[jpt.CTR_VISIBLE]), "decoded_blocks": int(ctr[jpt.CTR_NEW]),
                   "data_units": n_du},
        "gpu_ms_per_frame_median": round(float(np.median(gpu_frame)), 4),
        "cold_gpu_ms_per_frame_median": round(float(np.median(cold)), 4),
        "eager_ms_per_frame": round(eager_ms, 4),
        "phases_ms_median": {n: (None if (fused and n == "idct") else round(float(m), 4)) for n, m in zip(PHASES, med)},
        "mblocks_per_s": round(n_du / (dec_ms * 1e-3) / 1e6, 1),
        # the entropy kernel is bound by its symbol chain, not by bandwidth:
        # entropy-coded bits of the decoded MCUs per second of the decode phase
        "entropy_gbit_per_s": round(ab["stream_bits"] / (dec_ms * 1e-3) / 1e9, 1),
        "hbm_gbps_algorithmic": round(ab["method"] / (float(np.median(gpu_frame)) * 1e-3) / 1e9, 1),
        "roofline": roof,
    }
    if fused:
        # the entropy kernel is bound by the latency of its longest symbol chains, not by a throughput
        out["roofline"]["chain_floor"] = chain_floor(r, max(10, args.steps // 2))
    return r, out


def diff_form(args):
    """Differentiable form: one step = forward (F -> frame) + L2 loss +
    backward (-> dL/dF) through torch.autograd on the diff1080 scene."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt
    from paper_2510_08166_amd.synth import configs, target_frame
    wl = configs.diff1080()
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, device="cuda:0")
    r.mark()
    jpt.entropy_decode(r.scene, r.frame)
    diff = jpt.DiffFrame(r)
    F = diff.dequantize()
    g = wl.views[0]
    tgt = torch.from_numpy(target_frame(22, *g.shape).reshape(-1, 3)).cuda()

    def step():
        Fl = F.detach().requires_grad_(True)
        loss = ((diff(Fl) - tgt) ** 2).sum()
        loss.backward()
        return Fl.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fw, bw = [], []
    dfr = torch.ones(diff.n_pixels, 3, device="cuda")
    for _ in range(args.steps):
        ev[0].record()
        diff.forward(F)
        ev[1].record()
        diff.backward(dfr, tuple(F.shape))
        ev[2].record()
        torch.cuda.synchronize()
        fw.append(ev[0].elapsed_time(ev[1])); bw.append(ev[1].elapsed_time(ev[2]))
    n = F.shape[0]
    return {"metric": "fwd+bwd ms (differentiable form)", "value": round(ms, 4), "unit": "ms/step", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "work_items": int(n), "coefficients": int(n * 384),
                       "pixels": int(diff.n_pixels)},
            "fwd_ms_median": round(float(np.median(fw)), 4), "bwd_ms_median": round(float(np.median(bw)), 4)}


def heavy_form(args, reps=None):
    """Heavy recipe: 256 textures (512..8192, q40-95, 4:2:0 / 4:4:4, full
    chains), 3840x2160, trilinear, an LRU cache of 2 GiB of texel slots, 8
    frames of camera drift.  One frame = one graph launch (the cache counts
    frames on the device); the 8-frame sequence runs `reps` times from an
    empty cache.  Reports the mean over frames of the per-frame median and
    the max of the per-frame medians."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt
    from paper_2510_08166_amd.synth import configs
    t0 = time.perf_counter()
    wl = configs.heavy(log=log)
    log("heavy workload generated in %.1f s" % (time.perf_counter() - t0))
    slots = (2 << 30) // 1024
    t0 = time.perf_counter()
    r = jpt.Renderer(wl.textures, [wl.views[0]], wl.filter, device="cuda:0", policy=jpt.CACHE_LRU, n_slots=slots,
                     max_items=1 << 20, idct_mode=IDCT_MODES[args.idct])
    views = [jpt.Views([g]) for g in wl.views]
    torch.cuda.synchronize()
    log("index built and uploaded in %.1f s (%d block ids, %.2f GB compressed)" % (
        time.perf_counter() - t0, r.scene.n_blocks, r.scene.compressed_bytes() / 1e9))
    # eager pass, frame by frame: error flags and per-frame counts
    counts = []
    r.frame_no = jpt.FRAME_AUTO
    for v in views:
        r.views = v
        r.render()
        torch.cuda.synchronize()
        c = r.frame.counters_host()
        if c[jpt.CTR_ERROR]:
            raise SystemExit("device error flags %x" % c[jpt.CTR_ERROR])
        counts.append((int(c[jpt.CTR_VISIBLE]), int(c[jpt.CTR_NEW]), int(c[jpt.CTR_EVICTED])))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graphs = [r.capture(side, v) for v in views]
    reps = reps or max(3, args.steps // len(views))
    nf = len(views)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(nf + 1)] for _ in range(reps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for rep in range(reps):
        r.cache.reset(r.scene, jpt.vp(side.cuda_stream))
        ev[rep][0].record(side)
        for f in range(nf):
            graphs[f].launch()
            ev[rep][f + 1].record(side)
    side.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([[ev[k][f].elapsed_time(ev[k][f + 1]) for f in range(nf)] for k in range(reps)])
    med = np.median(per, axis=0)
    for g in graphs:
        g.close()
    c = r.frame.counters_host()
    if c[jpt.CTR_ERROR]:
        raise SystemExit("device error flags %x after the timed sequences" % c[jpt.CTR_ERROR])
    # one more sequence, eager, with events between the phases of every frame
    r.cache.reset(r.scene)
    pev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nf)]
    for f, v in enumerate(views):
        r.views = v
        pev[f][0].record()
        r.mark()
        pev[f][1].record()
        r.decode()
        pev[f][2].record()
        r.resolve()
        pev[f][3].record()
    torch.cuda.synchronize()
    phases = np.array([[pev[f][i].elapsed_time(pev[f][i + 1]) for i in range(3)] for f in range(nf)])
    return {"metric": METRIC, "value": round(float(med.mean()), 4), "unit": "ms/frame", "n_gpus": 1,
            "steps": reps * nf, "warmup": 0, "ms_per_step": round(1000.0 * wall / (reps * nf), 4),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE,
            "data": "synthetic",
            "config": {"workload": wl.name + ", trilinear, LRU 2 GiB", "frames": nf, "repetitions": reps,
                       "pixels_per_frame": int(wl.views[0].size), "block_ids": int(r.scene.n_blocks)},
            "per_frame_ms_median": [round(float(x), 4) for x in med],
            "max_of_medians_ms": round(float(med.max()), 4),
            "phases_ms_eager": {"mark+compact+lru": [round(float(x), 4) for x in phases[:, 0]],
                                "decode": [round(float(x), 4) for x in phases[:, 1]],
                                "resolve": [round(float(x), 4) for x in phases[:, 2]]},
            "frames_visible_new_evicted": counts}


def reduced_form(args, r):
    """Reduced-resolution decode (paper: Discussion, lower resolutions from the
    DC and the first ACs instead of stored mip levels) on the 1080p frame's
    work list: the fused decode of the stored levels against
    jpt_decode_reduced at scales 1/2, 1/4 and 1/8 over the same MCUs (median
    GPU ms per launch), and what the stored mip levels cost in bytes.  A
    level-k block made by reduced decode needs the 4^k level-0 MCUs under it,
    so its cost per output block is 4^k times the reduced decode's per MCU."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt
    r.mark()
    torch.cuda.synchronize()
    n = int(r.frame.counters_host()[jpt.CTR_ITEMS])
    out = torch.empty(max(1, n) * 64, dtype=torch.int32, device="cuda")

    def timed(fn, reps=20):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        fn()
        for e0, e1 in ev:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    stored = timed(r.decode)
    red = {}
    for sc in (1, 2, 3):
        red["1/%d" % (1 << sc)] = timed(lambda: jpt.decode_reduced(r.scene, r.frame, sc, out, r.tuning))
    if r.frame.counters_host()[jpt.CTR_ERROR]:
        raise SystemExit("reduced decode: device error flags %x" % r.frame.counters_host()[jpt.CTR_ERROR])
    lv = r.host.levels
    first = {int(f) for f in r.host.tex_first}  # each texture's level 0
    total = sum(l.stream.nbytes + l.records.nbytes for l in lv)
    base = sum(l.stream.nbytes + l.records.nbytes for i, l in enumerate(lv) if i in first)
    per_mcu = {k: v / max(1, n) for k, v in red.items()}
    return {"items": n, "stored_levels_decode_ms": round(stored, 4),
            "reduced_decode_ms": {k: round(v, 4) for k, v in red.items()},
            "cost_per_output_block_vs_stored": {"level %d" % sc: round((4 ** sc) * per_mcu["1/%d" % (1 << sc)] /
                                                                        (stored / max(1, n)), 2)
                                                for sc in (1, 2, 3)},
            "mip_levels_bytes_fraction": round(1.0 - base / total, 4)}


def paper_variants(args, wl, host):
    """The paper's relative comparisons on the 1080p workload (Evaluation:
    Performance, Linear Interpolation): per-phase GPU ms of eager frames for
    nearest, bilinear and the single-MCU clamped bilinear (whose footprint is
    the centre block alone), and for bilinear with mip mapping off."""
    from paper_2510_08166_amd import jpt
    out = {}
    cases = (("nearest", jpt.FILTER_NEAREST, jpt.CACHE_NONE), ("bilinear", jpt.FILTER_BILINEAR, jpt.CACHE_NONE),
             ("bilinear_clamped", jpt.FILTER_BILINEAR_CLAMPED, jpt.CACHE_NONE),
             ("bilinear_mip_off", jpt.FILTER_BILINEAR | jpt.FILTER_MIP_OFF, jpt.CACHE_NONE),
             # the paper's own cache: a hash map probed per tap
             ("hash_nearest", jpt.FILTER_NEAREST, jpt.CACHE_HASH),
             ("hash_bilinear", jpt.FILTER_BILINEAR, jpt.CACHE_HASH),
             ("hash_bilinear_clamped", jpt.FILTER_BILINEAR_CLAMPED, jpt.CACHE_HASH))
    for name, filt, policy in cases:
        r = jpt.Renderer(wl.textures, wl.views, filt, device="cuda:0", host=host, idct_mode=IDCT_MODES[args.idct],
                         policy=policy)
        for _ in range(3):
            r.render()
        _, med = time_phases(r, max(10, args.steps // 2))
        ctr = r.frame.counters_host()
        if ctr[jpt.CTR_ERROR]:
            raise SystemExit("%s: device error flags %x" % (name, ctr[jpt.CTR_ERROR]))
        # (with the hash cache the timed frames after the first find their blocks resident)
        out[name] = {"mark_ms": round(float(med[0]), 4), "decode_ms": round(float(med[1] + med[2]), 4),
                     "resolve_ms": round(float(med[3]), 4), "frame_ms": round(float(med.sum()), 4),
                     "visible_blocks": int(ctr[jpt.CTR_VISIBLE])}
        del r
    return out


def motion_form(args, textures, reps, log_prefix="motion"):
    """The paper's motion protocol (Evaluation: Caching): a camera turning 6
    degrees per frame, a full turn every 60 frames, `reps` turns; per view
    direction the median frame time over the turns, then the maximum over
    the 60 directions (max-of-medians).  The scene is a room of textured
    quads (the atrium stand-in) rendered each frame by the GPU geometry
    pass; the timed frame is mark + decode + resolve (one graph launch), in
    three configurations: no mip maps and no cache, mip maps, mip maps and
    the paper's cache (evict every block a frame does not read)."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt, synth
    W, H = 1920, 1080
    tris = synth.room_scene(8, len(textures), tex_side=textures[0].width)
    tris_t = torch.from_numpy(np.ascontiguousarray(tris).view(np.uint8).copy()).cuda()
    host = jpt.HostScene(textures)
    dirs = 60
    cams = [synth.camera((0.0, 1.7, 0.0), 6.0 * d, -5.0, 90.0, W, H) for d in range(dirs)]
    configs = (("no_mip_no_cache", jpt.FILTER_BILINEAR | jpt.FILTER_MIP_OFF, jpt.CACHE_NONE),
               ("mip_no_cache", jpt.FILTER_BILINEAR, jpt.CACHE_NONE),
               ("mip_cache", jpt.FILTER_BILINEAR, jpt.CACHE_EVICT_INVISIBLE),
               ("mip_hash_cache", jpt.FILTER_BILINEAR, jpt.CACHE_HASH))
    res = {"protocol": "6 deg/frame, %d directions, %d turns, max over directions of the median over turns" % (
        dirs, reps), "pixels": W * H, "triangles": int(len(tris))}
    side = torch.cuda.Stream()
    for name, filt, policy in configs:
        g0 = np.zeros((H, W), synth.GPIXEL_DTYPE)
        r = jpt.Renderer(textures, [g0], filt, device="cuda:0", host=host, policy=policy,
                         n_slots=None if policy == jpt.CACHE_NONE else 1 << 20, max_items=1 << 20,
                         idct_mode=IDCT_MODES[args.idct])
        side.wait_stream(torch.cuda.current_stream())
        graph = r.capture(side)
        times = np.zeros((reps, dirs))
        geo = np.zeros((reps, dirs))
        blocks = np.zeros(dirs)
        with torch.cuda.stream(side):
            if policy != jpt.CACHE_NONE:
                r.cache.reset(r.scene, jpt.vp(side.cuda_stream))
            # one warm-up turn
            for d in range(dirs):
                jpt.geometry_pass(r.scene, tris_t, cams[d], r.views, stream=jpt.vp(side.cuda_stream))
                graph.launch()
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps * dirs)]
            for k in range(reps):
                for d in range(dirs):
                    e = ev[k * dirs + d]
                    e[0].record(side)
                    jpt.geometry_pass(r.scene, tris_t, cams[d], r.views, stream=jpt.vp(side.cuda_stream))
                    e[1].record(side)
                    graph.launch()
                    e[2].record(side)
                    if k == reps - 1:
                        side.synchronize()
                        blocks[d] = r.frame.counters_host()[jpt.CTR_NEW]
            side.synchronize()
        ctr = r.frame.counters_host()
        if ctr[jpt.CTR_ERROR]:
            raise SystemExit("%s %s: device error flags %x" % (log_prefix, name, ctr[jpt.CTR_ERROR]))
        for k in range(reps):
            for d in range(dirs):
                e = ev[k * dirs + d]
                geo[k, d] = e[0].elapsed_time(e[1])
                times[k, d] = e[1].elapsed_time(e[2])
        graph.close()
        med = np.median(times, axis=0)
        res[name] = {"max_of_medians_ms": round(float(med.max()), 4), "mean_of_medians_ms": round(float(med.mean()), 4),
                     "decoded_blocks_per_frame_mean": round(float(blocks.mean()), 1),
                     "decoded_blocks_per_frame_max": int(blocks.max())}
        res["geometry_pass_ms_median"] = round(float(np.median(geo)), 4)
        log("%s %s: max of medians %.4f ms" % (log_prefix, name, med.max()))
        del r
    return res


def bc1_form(args, wl, gpu_ms):
    """The fixed-rate baseline (Background: BC1): the same textures encoded
    as BC1 by our simple encoder, sampled by jpt_bc1_resolve over the 1080p
    G-buffer (no mark, decode or cache); resolve time per frame and storage
    against the JPEG pipeline's frame time and compressed size."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt, synth
    t0 = time.perf_counter()
    levels = [[(synth.bc1_encode(l), l.shape[1], l.shape[0]) for l in synth.mip_chain(synth.texture(t.seed, t.width,
                                                                                                      t.height), len(t.jpegs))]
              for t in wl.textures]
    log("BC1 textures encoded in %.1f s" % (time.perf_counter() - t0))
    sc = jpt.Bc1Scene(levels)
    views = jpt.Views(wl.views)
    for _ in range(5):
        jpt.bc1_resolve(sc, views, wl.filter)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in ev:
        e0.record()
        jpt.bc1_resolve(sc, views, wl.filter)
        e1.record()
    torch.cuda.synchronize()
    ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    jpeg_bytes = sum(len(j) for t in wl.textures for j in t.jpegs)
    return {"resolve_ms_per_frame": round(ms, 4), "jpeg_pipeline_ms_per_frame": gpu_ms,
            "bc1_bytes": sc.bytes, "jpeg_file_bytes": jpeg_bytes,
            "bc1_bits_per_texel": round(8.0 * sc.bytes / sum(w * h for t in levels for _, w, h in t), 3)}


def other_forms(args):
    """The batched (16 views, one graph launch) and differentiable (fwd+bwd)
    forms on their own workloads, timed the same way as their own bench
    lines but without the tuner and the per-view comparison, reported as
    extra keys of the default line."""
    from paper_2510_08166_amd.synth import configs
    t0 = time.perf_counter()
    d = diff_form(args)
    res = {"diff1080": {"workload": d["config"]["workload"], "fwd_bwd_ms_per_step": d["value"],
                        "fwd_ms_median": d["fwd_ms_median"], "bwd_ms_median": d["bwd_ms_median"],
                        "work_items": d["config"]["work_items"]}}
    log("diff1080 done in %.1f s" % (time.perf_counter() - t0))
    t0 = time.perf_counter()
    wl = configs.batched16(log=log)
    log("batched16 generated in %.1f s" % (time.perf_counter() - t0))
    r, b = plain_form(args, wl, "batched16")
    res["batched16"] = {"workload": wl.name, "ms_per_frame": b["value"],
                        "gpu_ms_per_frame_median": b["gpu_ms_per_frame_median"],
                        "ms_per_view": round(b["value"] / r.views.n, 4), "views": r.views.n,
                        "pixels": r.views.n_pixels, "decoded_blocks": b["config"]["decoded_blocks"],
                        "data_units": b["config"]["data_units"], "phases_ms_median": b["phases_ms_median"],
                        "mblocks_per_s": b["mblocks_per_s"], "hbm_gbps_algorithmic": b["hbm_gbps_algorithmic"],
                        "roofline": b["roofline"]}
    return res


def batched_extras(args, r, out):
    """Batched form: tune the launch knobs (results must not change), time
    the tuned graph, and compare the MFMA fp16 IDCT with the fp32 scalar one
    (time of the IDCT phase, texel differences between the two)."""
    import numpy as np
    import torch
    from paper_2510_08166_amd import jpt, tune
    t0 = time.perf_counter()
    import tempfile
    knobs = tune.tune(r, reps=5, cache_path=os.path.join(tempfile.gettempdir(), "jpt_tune.json"), log=log)
    log("tuned in %.1f s: %s" % (time.perf_counter() - t0, tune.to_dict(knobs)))
    ms_tuned, gpu_tuned = time_graph(r, args.steps, args.warmup)
    ex = {"tuning": tune.to_dict(knobs), "value_default_knobs": out["value"],
          "value_tuned_knobs": round(ms_tuned, 4),
          "gpu_ms_per_frame_median_tuned": round(float(np.median(gpu_tuned)), 4)}
    # the tuner's short trials can pick knobs that the full timing finds
    # slower: the line reports the knobs that timed faster here
    if ms_tuned < out["value"]:
        out["value"] = out["ms_per_step"] = round(ms_tuned, 4)
        ex["knobs_used"] = "tuned"
    else:
        ex["knobs_used"] = "default"
        r.tuning = None
    # every view alone (16 plain frames) against the batch: per-view ms and
    # the blocks the batch decodes once for several views
    full = r.views
    per_view, vis = [], []
    for i in range(full.n):
        r.views = full.view(i)
        r.render()
        torch.cuda.synchronize()
        vis.append(int(r.frame.counters_host()[jpt.CTR_VISIBLE]))
        per_view.append(time_graph(r, max(10, args.steps // 3), 3)[0])
    r.views = full
    r.render()
    torch.cuda.synchronize()
    union = int(r.frame.counters_host()[jpt.CTR_VISIBLE])
    ex["per_view_ms"] = [round(x, 4) for x in per_view]
    ex["plain_16_views_ms"] = round(sum(per_view), 4)
    ex["speedup_vs_plain_16"] = round(sum(per_view) / out["value"], 2)
    ex["dedupe"] = {"sum_of_view_visible_blocks": sum(vis), "batch_visible_blocks": union,
                    "ratio": round(sum(vis) / max(union, 1), 3)}
    # IDCT modes: the MFMA fp16 texels against the scalar fp32 ones
    mode0 = r.idct_mode
    r.idct_mode = jpt.IDCT_MFMA_F16
    r.render()
    torch.cuda.synchronize()
    n_new = min(int(r.frame.counters_host()[jpt.CTR_NEW]), r.cache.n_slots)
    tex_mfma = r.cache.texels[: n_new * 256].clone()
    times = {}
    for mode, name in ((jpt.IDCT_MFMA_F16, "mfma_f16"), (jpt.IDCT_MFMA_BF16, "mfma_bf16"),
                       (jpt.IDCT_SCALAR_F32, "scalar_f32")):
        r.idct_mode = mode
        _, med = time_phases(r, args.steps)
        times[name] = round(float(med[2]), 4)
    torch.cuda.synchronize()
    tex_sc = r.cache.texels[: n_new * 256]
    a = tex_mfma.cpu().numpy().view(np.uint8).astype(np.int16)
    b = tex_sc.cpu().numpy().view(np.uint8).astype(np.int16)
    d = np.abs(a - b)
    r.idct_mode = mode0
    ex["idct_ms"] = times
    ex["idct_mfma_vs_scalar"] = {"max_abs_diff": int(d.max()), "channels_differing": int((d > 0).sum()),
                                 "channels": int(d.size)}
    return ex


def calibrate_copy():
    """One device copy of 1 GiB, for scaling the FETCH_SIZE / WRITE_SIZE
    counters of a profiled run to bytes."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    torch.add(a, 1, out=b)  # one elementwise kernel: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    log("copy calibration: 1073741824 bytes read and written")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="frame1080",
                    choices=["frame1080", "batched16", "diff1080", "heavy", "motion"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--motion-reps", type=int, default=20,
                    help="turns of the 6 deg/frame motion protocol (the paper uses 100)")
    ap.add_argument("--no-extra-forms", action="store_true",
                    help="frame1080 only: skip the batched16 and diff1080 figures added to the line")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="batched16 only: skip the launch-knob tuner and the MFMA/scalar IDCT comparison")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--idct", default="fused", choices=sorted(IDCT_MODES),
                    help="decode kernels: fused entropy+IDCT+colour, or entropy then the MFMA (fp16, bf16) or scalar IDCT")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path is single-GPU (each device would run the same per-frame "
              "pipeline on its share of the screen); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_08166_amd.synth import configs
    if args.calibrate_copy:
        calibrate_copy()
    if args.workload == "diff1080":
        print(json.dumps(diff_form(args)), flush=True)
        return
    if args.workload == "heavy":
        print(json.dumps(heavy_form(args)), flush=True)
        return
    if args.workload == "motion":
        wl = configs.frame1080()
        m = motion_form(args, wl.textures, reps=args.motion_reps)
        print(json.dumps({"metric": METRIC, "value": m["mip_cache"]["max_of_medians_ms"], "unit": "ms/frame",
                          "n_gpus": 1, "steps": 60 * args.motion_reps, "warmup": 60, "higher_is_better": False,
                          "scaling": "weak", "vs_baseline": None, "dtype": DTYPE, "data": "synthetic",
                          "config": {"workload": "room of 480 quads over the 1080p texture set, 1920x1080, bilinear, "
                                                 "6 deg/frame, evict-invisible cache"}, "motion": m}), flush=True)
        return
    t0 = time.perf_counter()
    if args.workload == "frame1080":
        wl = configs.frame1080()
        label = ("1080p: 32 x 2048^2 textures (q50-90, 4:2:0, 8 levels), 1920x1080 G-buffer from 200 quads, "
                 "bilinear, no cache")
    else:
        wl = configs.batched16(log=log)
        label = ("batched: 16 views (2 stereo pairs 2064x2208 + 12 mono 1280x720..2560x1440) over a 128-texture "
                 "pool (512..4096, q50-90, 4:2:0), one graph launch per frame, bilinear, no cache")
    log("workload generated in %.1f s" % (time.perf_counter() - t0))
    r, out = plain_form(args, wl, label)
    if args.workload == "batched16" and not args.no_tune:
        out.update(batched_extras(args, r, out))
    if args.workload == "frame1080" and not args.no_cpu_baseline:
        log("timing the CPU oracle (budget %.0f s)" % args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
        log("timing the CPU on-demand baseline")
        out["cpu_ondemand_baseline"] = cpu_ondemand_baseline(wl, out["value"])
    if args.workload == "frame1080" and not args.no_extra_forms:
        out["reduced_decode"] = reduced_form(args, r)
        host = r.host
        del r
        t0 = time.perf_counter()
        out["paper_variants"] = paper_variants(args, wl, host)
        out["bc1_baseline"] = bc1_form(args, wl, out["gpu_ms_per_frame_median"])
        out["motion"] = motion_form(args, wl.textures, reps=args.motion_reps)
        log("paper variants, BC1 and motion legs in %.1f s" % (time.perf_counter() - t0))
        del host
        out["other_forms"] = other_forms(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
