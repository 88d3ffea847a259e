"""GPU parity of the differentiable form (jpt_dequantize / jpt_fwd_float /
jpt_backward and the autograd.Function above them) against the float64
reference in oracle.grad.

Bar (derived in the design notes from fp32 arithmetic): F bit-exact (integer
products); frame within 2e-3 absolute of the float64 frame (texels are
64-term fp32 sums of products of size <= 2^11); dL/dF within 1e-4 of the
largest float64 gradient entry and within 1e-5 relative L2; repeated
backward passes bit-identical (fixed-point accumulation).
"""
import time

import numpy as np
import pytest
import torch

import oracle
from oracle import grad, parity
from paper_2510_08166_amd.synth import GPIXEL_DTYPE, configs, make_textures, target_frame
from paper_2510_08166_amd.synth.configs import Workload, quad_scene

pytestmark = pytest.mark.gpu

FWD_ATOL = 2e-3
GRAD_MAX_REL = 1e-4
GRAD_L2_REL = 1e-5


def gpu_case(wl):
    from paper_2510_08166_amd import jpt
    r = jpt.Renderer(wl.textures, wl.views, wl.filter)
    r.mark()
    jpt.entropy_decode(r.scene, r.frame)
    diff = jpt.DiffFrame(r)
    F = diff.dequantize()
    torch.cuda.synchronize()
    assert r.frame.counters_host()[jpt.CTR_ERROR] == 0
    return r, diff, F


def oracle_case(wl, items):
    osc = oracle.Scene(wl.textures)
    blocks = parity.visible_blocks(osc, wl.views, wl.filter)
    assert np.array_equal(items, parity.expected_items(osc, blocks))
    return osc, grad.dequantized(osc, items)


def check_grad(g, g64, what):
    scale = np.abs(g64).max()
    err = np.abs(g - g64).max()
    l2 = np.linalg.norm(g - g64) / max(np.linalg.norm(g64), 1e-300)
    print("%s: max |dF - dF64| = %.3e (max |dF64| %.3e), rel L2 %.3e" % (what, err, scale, l2), flush=True)
    assert err <= GRAD_MAX_REL * scale and l2 <= GRAD_L2_REL


def vjp_parity(wl, seed=0, scale=1.0):
    r, diff, F = gpu_case(wl)
    items = r.frame.work_items()
    osc, F64 = oracle_case(wl, items)
    assert np.array_equal(F.cpu().numpy().astype(np.float64), F64)
    frame = diff.forward(F)
    rng = np.random.default_rng(seed)
    dframe = [rng.standard_normal(g.shape + (3,)) * scale for g in wl.views]
    dflat = torch.from_numpy(np.concatenate([d.reshape(-1, 3) for d in dframe]).astype(np.float32)).cuda()
    dF = diff.backward(dflat, tuple(F.shape))
    dF2 = diff.backward(dflat, tuple(F.shape))
    torch.cuda.synchronize()
    assert torch.equal(dF, dF2), "backward is not deterministic"
    fr = frame.cpu().numpy()
    off = 0
    g64 = np.zeros_like(F64)
    for g, d in zip(wl.views, dframe):
        f64, gv = grad.vjp(osc, items, F64, g, wl.filter, d.astype(np.float32).astype(np.float64))
        n = g.size
        err = np.abs(fr[off:off + n].reshape(f64.shape) - f64).max()
        print("%s: forward max |frame - frame64| = %.3e" % (wl.name, err), flush=True)
        assert err <= FWD_ATOL
        g64 += gv
        off += n
    check_grad(dF.cpu().numpy().astype(np.float64), g64, wl.name)


@pytest.mark.parametrize("filt", [oracle.NEAREST, oracle.BILINEAR, oracle.TRILINEAR])
def test_reduced_vjp(gpu, filt):
    vjp_parity(configs.reduced(seed=7, filt=filt))


@pytest.mark.parametrize("scale", ["mean", 1e-6, 1e6])
def test_vjp_at_any_loss_scale(gpu, scale):
    """dL/dframe of a mean-reduced loss (entries of order 1/(3 x pixels)),
    and of losses scaled by 1e-6 and 1e6: the backward's fixed-point unit
    follows max |dL/dframe|, so the gradient keeps the same relative
    accuracy (and does not overflow)."""
    wl = configs.reduced(seed=8, filt=oracle.BILINEAR)
    s = 1.0 / (3 * wl.n_pixels) if scale == "mean" else scale
    vjp_parity(wl, seed=3, scale=s)


def test_mixed_sampling_ragged_trilinear(gpu):
    tex = make_textures([(31, 72, 56, 70, 420, 3), (32, 60, 44, 85, 444, 3), (33, 200, 136, 55, 444, None)])
    rng = np.random.default_rng(5)
    H, W = 70, 130
    g = np.zeros((H, W), GPIXEL_DTYPE)
    g["u"] = rng.uniform(-1, 2, (H, W)).astype(np.float32)
    g["v"] = rng.uniform(-1, 2, (H, W)).astype(np.float32)
    g["tex"] = rng.integers(0, 3, (H, W))
    g["lod"] = rng.uniform(-0.5, 4.5, (H, W)).astype(np.float32)
    g["tex"][:3, :] = oracle.BACKGROUND
    vjp_parity(Workload("mixed 420/444 ragged", tex, [g], oracle.TRILINEAR))


def test_two_views_share_blocks(gpu):
    wl = quad_scene(13, 3, 256, 60, 80, 4, 160, 96, 12, sampling=444)
    wl2 = Workload("two views", wl.textures, [wl.views[0], wl.views[0][::-1].copy()], oracle.BILINEAR)
    vjp_parity(wl2, seed=4)


def test_autograd_l2_loss(gpu):
    from paper_2510_08166_amd import jpt
    wl = configs.reduced(seed=9)
    r, diff, F = gpu_case(wl)
    items = r.frame.work_items()
    osc, F64 = oracle_case(wl, items)
    g = wl.views[0]
    target = target_frame(21, *g.shape)
    tgt = torch.from_numpy(target.reshape(-1, 3)).cuda()
    Fl = F.clone().requires_grad_(True)
    loss = ((diff(Fl) - tgt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    L64, g64 = grad.l2_loss_grad(osc, items, F64, g, wl.filter, target.astype(np.float64))
    print("loss %.6e vs %.6e" % (float(loss), L64))
    assert abs(float(loss) - L64) <= 1e-5 * L64
    check_grad(Fl.grad.cpu().numpy().astype(np.float64), g64, "autograd L2")


def test_rejects_lru_cache(gpu):
    from paper_2510_08166_amd import jpt
    wl = configs.reduced(seed=7)
    r = jpt.Renderer(wl.textures, wl.views, wl.filter, policy=jpt.CACHE_LRU)
    with pytest.raises(ValueError):
        jpt.DiffFrame(r)


@pytest.mark.slow
def test_diff1080_full_size(gpu):
    """The differentiable-form scene at full size (1920x1080, 32 x 2048^2 q75),
    whole frame and whole gradient against float64."""
    t0 = time.time()
    wl = configs.diff1080()
    print("scene built in %.1f s" % (time.time() - t0), flush=True)
    r, diff, F = gpu_case(wl)
    items = r.frame.work_items()
    print("items %d" % len(items), flush=True)
    osc, F64 = oracle_case(wl, items)
    assert np.array_equal(F.cpu().numpy().astype(np.float64), F64)
    g = wl.views[0]
    target = target_frame(22, *g.shape)
    tgt = torch.from_numpy(target.reshape(-1, 3)).cuda()
    Fl = F.clone().requires_grad_(True)
    frame = diff(Fl)
    loss = ((frame - tgt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    L64, g64 = grad.l2_loss_grad(osc, items, F64, g, wl.filter, target.astype(np.float64))
    print("loss %.6e vs %.6e" % (float(loss), L64), flush=True)
    assert abs(float(loss) - L64) <= 1e-5 * L64
    check_grad(Fl.grad.cpu().numpy().astype(np.float64), g64, "diff1080")
