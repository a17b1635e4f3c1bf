"""Parity of the HIP ray marcher (through the C ABI) with the FP64 oracle on the same inputs."""

import numpy as np
import pytest

from gpu_common import (check_err, gpu_context, oracle_scene, say, scene_arrays,
                        smooth_cache)
from paper_2304_07338_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c0(orc):
    import torch
    w, vol, tf, lights = scene_arrays("c0")
    ctx = gpu_context(vol, tf, lights)
    os_ = oracle_scene(orc, vol, tf, lights)
    return dict(w=w, vol=vol, tf=tf, lights=lights, ctx=ctx, os=os_)


def _render_both(orc, s, cam, cfg, ocfg, cache=None, field=None, pixels=None):
    from paper_2304_07338_amd.pfn import RenderConfig
    img = s["ctx"].render_frame(cam, cfg)
    s["ctx"].sync()
    g = img.cpu().numpy().reshape(-1, 3).astype(np.float64)
    ref = orc.render_pixels(s["os"], cam, ocfg, pixels=pixels, cache=cache, field=field)
    if pixels is not None:
        g = g[pixels]
    return g, ref


def test_c0_full_frame_cache_and_shadow_rays(orc, c0):
    """The plain-method configuration: 64^3 f32, 128x128, 1 spp, step 0.5 voxel, exact shadow
    rays, a 32^3 single-bin cache gathered every step, no early termination."""
    from paper_2304_07338_amd.pfn import RenderConfig, INDIRECT_CACHE
    import torch
    say("c0 full frame: cache + shadow rays 128x128")
    cache = smooth_cache(32, 1, seed=3)
    c0["ctx"].set_cache(torch.tensor(cache, dtype=torch.float32, device="cuda:0"), [0.0], 1.0)
    cam = sg.make_camera(c0["w"].seed, 0, 128, 128)
    cfg = RenderConfig(indirect=INDIRECT_CACHE, g=0.0)
    ocfg = orc.render_params(indirect=orc.IND_CACHE, g=0.0)
    g, ref = _render_both(orc, c0, cam, cfg, ocfg, cache=orc.OracleCache(cache, [0.0], 32))
    assert ref.max() > 0 and np.count_nonzero(ref) > 1000
    # FP32 march against FP64: measured 7.4e-7 / 1.0e-6
    check_err(g, ref, 1e-5, 1e-5, "c0 frame")


def test_ragged_image_direct_only(orc, c0):
    from paper_2304_07338_amd.pfn import RenderConfig
    say("ragged 37x29 direct only, g=0.6")
    cam = sg.make_camera(c0["w"].seed, 1, 37, 29)
    g, ref = _render_both(orc, c0, cam, RenderConfig(g=0.6), orc.render_params(g=0.6))
    check_err(g, ref, 2e-5, 1e-5, "ragged")  # measured 1.6e-6 / 7.1e-7


def test_light_volume_three_lights_and_mask(orc):
    import torch
    from paper_2304_07338_amd.pfn import RenderConfig, DIRECT_LIGHT_VOLUME
    say("light volume, 3 lights, mask 0b101, 48x40")
    w, vol, tf, _ = scene_arrays("c0")
    lights = sg.lights_array(sg.make_lights(3, 77))
    ctx = gpu_context(vol, tf, lights)
    ctx.build_light_volume(0.5)
    os_ = oracle_scene(orc, vol, tf, lights)
    cam = sg.make_camera(w.seed, 2, 48, 40)
    for mask in (0, 0b101):
        img = ctx.render_frame(cam, RenderConfig(direct=DIRECT_LIGHT_VOLUME, g=-0.3, light_mask=mask))
        ctx.sync()
        ref = orc.render_pixels(os_, cam, orc.render_params(direct=orc.DIR_LIGHTVOL, g=-0.3,
                                                            light_mask=mask))
        # transmittances are stored as binary16 (relative spacing 2^-11 = 4.9e-4); measured
        # 6.5e-5 / 1.05e-4, the bar is about two binary16 ulps per pixel
        check_err(img.cpu().numpy().reshape(-1, 3), ref, 6e-4, 1e-3, f"mask {mask}")


def test_spp_jitter_termination_cap_and_bins(orc, c0):
    import torch
    from paper_2304_07338_amd.pfn import RenderConfig, INDIRECT_CACHE
    say("spp 4, t_min 1e-3, max_steps 150, 2-bin cache at g=0.25, stride 3")
    cache = smooth_cache(16, 2, seed=5)
    c0["ctx"].set_cache(torch.tensor(cache, dtype=torch.float32, device="cuda:0"), [-0.5, 0.5], 1.0)
    cam = sg.make_camera(c0["w"].seed, 3, 40, 36)
    cfg = RenderConfig(spp=4, t_min=1e-3, max_steps=150, indirect=INDIRECT_CACHE, g=0.25,
                       field_stride=3, seed=99)
    ocfg = orc.render_params(spp=4, t_min=1e-3, max_steps=150, indirect=orc.IND_CACHE, g=0.25,
                             field_stride=3, seed=99)
    g, ref = _render_both(orc, c0, cam, cfg, ocfg, cache=orc.OracleCache(cache, [-0.5, 0.5], 16))
    # measured 7.0e-7 / 8.5e-7 (no early-termination decision flips between FP32 and FP64 on
    # this view; a flip would move a pixel by at most t_min times its remaining contribution)
    check_err(g, ref, 1e-5, 1e-5, "spp")


def test_degenerate_views(orc, c0):
    from paper_2304_07338_amd.pfn import RenderConfig
    say("camera looking away; zero step cap")
    cam = sg.Camera((0.5, 0.5, -1.7), (0.5, 0.5, -3.0), (0.0, 1.0, 0.0), 40.0, 16, 16)
    img = c0["ctx"].render_frame(cam, RenderConfig())
    c0["ctx"].sync()
    assert float(img.abs().max()) == 0.0
    cam = sg.make_camera(c0["w"].seed, 0, 16, 16)
    img = c0["ctx"].render_frame(cam, RenderConfig(max_steps=0))
    c0["ctx"].sync()
    assert float(img.abs().max()) == 0.0
    # a 1x1 image through the cube centre
    cam = sg.Camera((0.5, 0.5, -1.7), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 10.0, 1, 1)
    g, ref = _render_both(orc, c0, cam, RenderConfig(g=0.1), orc.render_params(g=0.1))
    check_err(g, ref, 1e-5, 1e-5, "1x1")  # measured 2.2e-7


def test_invalid_arguments_are_rejected(c0):
    from paper_2304_07338_amd.pfn import RenderConfig, PfnError, INDIRECT_FIELD
    cam = sg.make_camera(c0["w"].seed, 0, 8, 8)
    for bad in (RenderConfig(spp=0), RenderConfig(g=0.99), RenderConfig(step_voxels=-1.0),
                RenderConfig(field_stride=0)):
        with pytest.raises(PfnError) as e:
            c0["ctx"].render_frame(cam, bad)
        assert e.value.status == -1
    with pytest.raises(PfnError) as e:  # no field in slot 7
        c0["ctx"].render_frame(cam, RenderConfig(indirect=INDIRECT_FIELD, field_slot=7))
    assert e.value.status == -4
