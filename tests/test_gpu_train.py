"""Parity of the HIP training path with the FP64 oracle: batch generation, loss and gradients
of the fused forward/backward (FP32 and 16-bit matrix cores), one Adam step, and an end-to-end
fit of a smooth target."""
import math

import numpy as np
import pytest

from gpu_common import gpu_context, say, scene_arrays, smooth_cache

pytestmark = pytest.mark.gpu


def odesc(orc, cfg):
    return orc.field_desc(levels=cfg.levels, feats=cfg.feats_per_level, base_res=cfg.base_res,
                          growth=cfg.growth, log2_table=cfg.log2_table,
                          hidden_layers=cfg.hidden_layers, width=cfg.width, psi=cfg.psi)


@pytest.fixture(scope="module")
def tctx():
    import torch
    w, vol, tf, lights = scene_arrays("c0")
    ctx = gpu_context(vol, tf, lights)
    cache = smooth_cache(16, 3, seed=9)
    ctx.set_cache(torch.tensor(cache, dtype=torch.float32, device="cuda:0"), [-0.5, 0.0, 0.5],
                  float(cache.max()))
    return ctx, cache


def test_training_batch_matches_oracle(orc, tctx):
    ctx, cache = tctx
    from paper_2304_07338_amd.pfn import FieldConfig
    ctx.field_select(0)
    ctx.field_init(FieldConfig(log2_table=12), seed=0)
    n = 5000
    xyz, dirs, g, b, tgt = (t.cpu().numpy() for t in ctx.train_batch(42, 17, n))
    oc = orc.OracleCache(cache, [-0.5, 0.0, 0.5], 16)
    ox, od, og, ob, ot = orc.train_batch(42, 17, n, oc, float(cache.max()))
    np.testing.assert_array_equal(xyz.astype(np.float64), ox)  # uniforms are exact in FP32
    np.testing.assert_array_equal(b, ob)
    np.testing.assert_array_equal(g, og.astype(np.float32))
    assert np.abs(dirs - od).max() < 2e-6
    d = np.abs(tgt - ot)
    say("  target max |d|", d.max())
    assert d.max() < 2e-5


def _random_params(orc, desc, seed):
    L = orc.field_layout(desc)
    rng = np.random.default_rng(seed)
    p = np.zeros(L.n_params, dtype=np.float32)
    p[:L.mlp_off] = rng.uniform(-0.3, 0.3, L.mlp_off)
    for m in range(L.n_mats):
        r, c = L.w_rows[m], L.w_cols[m]
        lim = math.sqrt(6.0 / (r + c))
        p[L.w_off[m]:L.w_off[m] + r * c] = rng.uniform(-lim, lim, r * c)
    return p, L


def _segments(L):
    segs = {"pos_grid": (0, L.pos_params), "dir_grid": (L.pos_params, L.mlp_off)}
    for m in range(L.n_mats):
        segs[f"W{m}"] = (L.w_off[m], L.w_off[m] + L.w_rows[m] * L.w_cols[m])
    return segs


@pytest.mark.parametrize("levels,hidden", [(16, 3), (8, 2), (16, 1)])
def test_forward_backward_gradients(orc, tctx, levels, hidden):
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig
    ctx, _ = tctx
    cfg = FieldConfig(levels=levels, hidden_layers=hidden, log2_table=12)
    desc = odesc(orc, cfg)
    ctx.field_select(1)
    ctx.field_init(cfg, seed=1)
    p, L = _random_params(orc, desc, seed=levels * 10 + hidden)
    ctx.field_set_params(torch.tensor(p, device="cuda:0"))
    n = 16 * 40 + 7
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(n, 3)).astype(np.float32)
    w = rng.normal(size=(n, 3))
    w = (w / np.linalg.norm(w, axis=1, keepdims=True)).astype(np.float32)
    g = rng.uniform(-0.8, 0.8, n).astype(np.float32)
    tgt = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    dev = [torch.tensor(a, device="cuda:0") for a in (x, w, g, tgt)]
    pd = p.astype(np.float64)
    for prec, rounding in (("f32", 0), ("f16", 1), ("bf16", 2)):
        loss, grad = ctx.field_forward_backward(*dev, precision=prec)
        grad = grad.cpu().numpy().astype(np.float64)
        oloss, ograd = orc.field_loss_grad(desc, pd, x, w, g, tgt, rounding=rounding)
        say(f"  {prec}: loss {loss:.6e} vs {oloss:.6e}")
        for name, (a0, a1) in _segments(L).items():
            gg, og = grad[a0:a1], ograd[a0:a1]
            rel = np.linalg.norm(gg - og) / max(np.linalg.norm(og), 1e-300)
            cos = gg @ og / max(np.linalg.norm(gg) * np.linalg.norm(og), 1e-300)
            say(f"    {name:8s} rel-L2 {rel:.2e} cos {cos:.6f}")
            if prec == "f32":
                assert rel <= 1e-5, name
            else:
                # activations and deltas are rounded to 16 bits after every product (relative
                # 2^-11 for f16, 2^-8 for bf16) along a chain of 2H+1 products
                tol_rel, tol_cos = (4e-2, 0.999) if prec == "f16" else (1.5e-1, 0.99)
                assert rel <= tol_rel and cos >= tol_cos, name
        if prec == "f32":
            assert loss == pytest.approx(oloss, rel=1e-6)
        else:
            assert loss == pytest.approx(oloss, rel=2e-2)


@pytest.mark.parametrize("hidden,growth,levels", [(3, 1.5, 16), (5, 2.0, 12)])
def test_relative_loss_gradients(orc, tctx, hidden, growth, levels):
    """Relative L2 (Section 3.5.1): loss and gradient against the oracle's, FP32, also for the
    paper's deeper network and level growth 2 (12 levels: the finest is 16 * 2^11 per axis)."""
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig
    ctx, _ = tctx
    cfg = FieldConfig(levels=levels, hidden_layers=hidden, growth=growth, log2_table=12)
    desc = odesc(orc, cfg)
    ctx.field_select(2)
    ctx.field_init(cfg, seed=3)
    p, L = _random_params(orc, desc, seed=70 + hidden)
    ctx.field_set_params(torch.tensor(p, device="cuda:0"))
    n = 16 * 30 + 5
    rng = np.random.default_rng(4)
    x = rng.uniform(size=(n, 3)).astype(np.float32)
    w = rng.normal(size=(n, 3))
    w = (w / np.linalg.norm(w, axis=1, keepdims=True)).astype(np.float32)
    g = rng.uniform(-0.8, 0.8, n).astype(np.float32)
    tgt = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    dev = [torch.tensor(a, device="cuda:0") for a in (x, w, g, tgt)]
    loss, grad = ctx.field_forward_backward(*dev, precision="f32", loss="rel")
    grad = grad.cpu().numpy().astype(np.float64)
    oloss, ograd = orc.field_loss_grad(desc, p.astype(np.float64), x, w, g, tgt, loss="rel")
    say(f"  relative L2, {hidden} hidden, growth {growth}: loss {loss:.6e} vs {oloss:.6e}")
    assert loss == pytest.approx(oloss, rel=1e-5)
    for name, (a0, a1) in _segments(L).items():
        gg, og = grad[a0:a1], ograd[a0:a1]
        rel = np.linalg.norm(gg - og) / max(np.linalg.norm(og), 1e-300)
        assert rel <= 2e-5, name
    ctx.field_select(0)


def test_adam_step_matches_oracle(orc, tctx):
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig
    ctx, _ = tctx
    cfg = FieldConfig(levels=4, hidden_layers=1, log2_table=8)
    ctx.field_select(2)
    ctx.field_init(cfg, seed=2)
    p0 = ctx.field_get_params().cpu().numpy().astype(np.float64)
    n = p0.size
    rng = np.random.default_rng(5)
    m = np.zeros(n)
    v = np.zeros(n)
    p = p0.copy()
    for t in range(1, 4):
        grad = rng.normal(scale=10.0 ** rng.uniform(-6, 1, n), size=n).astype(np.float32)
        ctx.field_adam_step(torch.tensor(grad, device="cuda:0"), t, 9e-4)
        orc.adam_step(p, grad.astype(np.float64), m, v, t, 9e-4)
    gp = ctx.field_get_params().cpu().numpy().astype(np.float64)
    err = np.abs(gp - p).max()
    say("  adam max |dp|", err, "step size", np.abs(p - p0).max())
    assert err <= 1e-6 * max(1.0, np.abs(p).max())


def test_training_fits_a_smooth_target(orc, tctx):
    from paper_2304_07338_amd.pfn import FieldConfig, TrainConfig
    ctx, cache = tctx
    ctx.field_select(3)
    ctx.field_init(FieldConfig(log2_table=14), seed=3)
    say("train 600 steps at 2^14 on a smooth 3-bin cache")
    hist = ctx.train_field(TrainConfig(steps=600, log2_batch=14, decay_start=420, seed=11))
    say("  loss", hist[0], "->", hist[-10:].mean())
    assert np.all(np.isfinite(hist))
    assert hist[-10:].mean() < 0.1 * hist[0]
    assert hist[-10:].mean() < 1e-3
