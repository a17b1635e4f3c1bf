"""The smallest and most lopsided volumes against the FP64 oracle: 2 x 2 x 2 (one brick, a light
grid of one texel, every lookup clamped at a face), 5 x 2 x 3 and 9 x 2 x 17 (nx, ny, nz), in
FP32 and binary16 (the oracle gets the rounded values).  The view holds the whole cube, so rays
enter through every face.  Checked: the fused kernel with exact shadow rays and a 2-bin cache
between its bins, and field-lit frames (FP32 field, light-transmittance volume) in the fused
kernel and in the wavefront rounds."""
import numpy as np
import pytest

from gpu_common import (check_err, gpu_context, oracle_desc, oracle_scene, random_params,
                        scene_arrays, smooth_cache, volume_as)

pytestmark = pytest.mark.gpu

SHAPES = [(2, 2, 2), (3, 2, 5), (17, 2, 9)]  # [z][y][x]


def _volume(shape, seed):
    import torch
    rng = np.random.default_rng(seed)
    return torch.tensor(rng.uniform(0.0, 1.0, shape), dtype=torch.float32)


def _camera():
    from paper_2304_07338_amd import scenegen as sg
    return sg.Camera((0.55, 0.65, -1.1), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 58.0, 19, 13)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("shape", SHAPES, ids=["2x2x2", "5x2x3", "9x2x17"])
def test_tiny_volume_cache_and_shadow_rays(orc, shape, dtype):
    import torch
    from paper_2304_07338_amd.pfn import RenderConfig, INDIRECT_CACHE
    w, _, tf, lights = scene_arrays("c0")
    vol = volume_as(_volume(shape, sum(shape)), dtype)
    ctx = gpu_context(vol, tf, lights)
    cache = smooth_cache(4, 2, seed=5)
    ctx.set_cache(torch.tensor(cache, dtype=torch.float32, device="cuda:0"), [-0.5, 0.5], 1.0)
    cam = _camera()
    img = ctx.render_frame(cam, RenderConfig(spp=2, indirect=INDIRECT_CACHE, g=0.1, seed=4))
    ctx.sync()
    ref = orc.render_pixels(oracle_scene(orc, vol, tf, lights), cam,
                            orc.render_params(indirect=orc.IND_CACHE, g=0.1, spp=2, seed=4),
                            cache=orc.OracleCache(cache, [-0.5, 0.5], 4))
    assert ref.max() > 0
    # the 64^3 frame's bars (FP32 march against FP64)
    check_err(img.cpu().numpy().reshape(-1, 3), ref, 1e-5, 1e-5, f"{shape} {dtype}")
    ctx.close()


@pytest.mark.parametrize("shape", SHAPES, ids=["2x2x2", "5x2x3", "9x2x17"])
def test_tiny_volume_field_and_light_volume(orc, shape):
    import torch
    from paper_2304_07338_amd.pfn import (FieldConfig, RenderConfig, DIRECT_LIGHT_VOLUME,
                                          INDIRECT_FIELD)
    w, _, tf, lights = scene_arrays("c0")
    vol = volume_as(_volume(shape, 7 + sum(shape)), "f16")
    ctx = gpu_context(vol, tf, lights)
    ctx.build_light_volume(0.5)
    cfg = FieldConfig(levels=8, log2_table=12, hidden_layers=2)
    desc = oracle_desc(orc, cfg)
    ctx.field_init(cfg, seed=2)
    p = random_params(orc, desc, seed=13, out_scale=0.2)
    ctx.field_set_params(torch.tensor(p, device="cuda:0"))
    ctx.field_set_kappa(5e-3)
    cam = _camera()
    rc = RenderConfig(spp=1, field_stride=2, g=0.3, indirect=INDIRECT_FIELD,
                      direct=DIRECT_LIGHT_VOLUME, field_precision="f32")
    ref = orc.render_pixels(oracle_scene(orc, vol, tf, lights), cam,
                            orc.render_params(indirect=orc.IND_FIELD, field_stride=2, g=0.3,
                                              direct=orc.DIR_LIGHTVOL),
                            field=(desc, p.astype(np.float64), 0, 5e-3))
    assert ref.max() > 0
    for strategy in ("fused", "wavefront"):
        ctx.set_render_strategy(strategy)
        img = ctx.render_frame(cam, rc)
        ctx.sync()
        # transmittances stored as binary16: the light-volume frame's bars
        check_err(img.cpu().numpy().reshape(-1, 3), ref, 6e-4, 1e-3, f"{shape} {strategy}")
    ctx.set_render_strategy("auto")
    ctx.close()
