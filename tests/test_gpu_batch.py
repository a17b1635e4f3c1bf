"""Batched ray-march launch of the fused kernel: many jobs of uneven sizes, cameras, lights, g and field slots in one
launch (plain or persistent, immediate or replayed from a captured HIP graph), bit-identical to
rendering each job alone, and checked against the FP64 oracle."""
import numpy as np
import pytest

from gpu_common import check_err, gpu_context, oracle_scene, say, scene_arrays
from paper_2304_07338_amd import scenegen as sg

pytestmark = pytest.mark.gpu

SIZES = [(17, 23), (64, 48), (100, 37), (8, 8), (1, 1), (55, 66), (33, 9)]


@pytest.fixture(scope="module")
def bctx(orc):
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig
    w, vol, tf, _ = scene_arrays("c0")
    lights = sg.lights_array(sg.make_lights(4, 55))
    ctx = gpu_context(vol, tf, lights)
    ctx.set_render_strategy("fused")  # the persistent and graph launches are fused kernels
    ctx.build_light_volume(0.5)
    for slot in (0, 1):
        ctx.field_select(slot)
        ctx.field_init(FieldConfig(log2_table=14), seed=slot)
        p = ctx.field_get_params()
        g = torch.Generator(device="cuda:0").manual_seed(slot)
        p = p + 0.3 * torch.rand(p.shape, device="cuda:0", generator=g) - 0.15
        ctx.field_set_params(p.contiguous())
        ctx.field_set_kappa(1e-2)
    return dict(w=w, ctx=ctx, vol=vol, tf=tf, lights=lights)


def jobs(bctx, indirect):
    from paper_2304_07338_amd.pfn import RenderConfig, DIRECT_LIGHT_VOLUME
    cams, cfgs = [], []
    g_vals = sg.uniform_g(99, len(SIZES))
    for i, (wd, ht) in enumerate(SIZES):
        cams.append(sg.make_camera(bctx["w"].seed, 10 + i, wd, ht))
        cfgs.append(RenderConfig(spp=1 + (i % 3), t_min=1e-3, max_steps=400, field_stride=4,
                                 g=float(g_vals[i]), indirect=indirect, direct=DIRECT_LIGHT_VOLUME,
                                 light_mask=1 << (i % 4), field_slot=i % 2, seed=i))
    return cams, cfgs


def singles(ctx, cams, cfgs):
    outs = []
    for c, f in zip(cams, cfgs):
        outs.append(ctx.render_frame(c, f).clone())
    ctx.sync()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("mode", ["field", "cache_none"])
def test_batch_equals_single_renders_in_every_launch_mode(bctx, mode):
    import torch
    from paper_2304_07338_amd.pfn import INDIRECT_FIELD, INDIRECT_NONE
    ctx = bctx["ctx"]
    cams, cfgs = jobs(bctx, INDIRECT_FIELD if mode == "field" else INDIRECT_NONE)
    ctx.set_launch_mode(0, False)
    ctx.set_tile_config(8, 2, 2)
    ref = singles(ctx, cams, cfgs)
    assert max(float(np.abs(r).max()) for r in ref) > 0
    for tile_w, bw, bh in ((8, 2, 2), (16, 4, 1), (32, 1, 4), (4, 2, 2)):
        for persistent in (0, 2):
            for graph in (False, True):
                ctx.set_tile_config(tile_w, bw, bh)
                ctx.set_launch_mode(persistent, graph)
                say(f"  {mode}: tile {tile_w} block {bw}x{bh} persistent {persistent} graph {graph}")
                for rep in range(3 if graph else 1):
                    outs = ctx.render_batch(cams, cfgs)
                    ctx.sync()
                    for o, r in zip(outs, ref):
                        np.testing.assert_array_equal(o.cpu().numpy(), r)
                    # eager work between graph replays
                    _ = (torch.ones(1000, device="cuda:0") * rep).sum().item()
    ctx.set_launch_mode(0, False)
    ctx.set_tile_config(8, 2, 2)


def test_graph_replay_follows_new_cameras(bctx):
    """The job table is refreshed before every replay: moving the cameras (same sizes) reuses
    the captured launch and still renders the new views."""
    from paper_2304_07338_amd.pfn import INDIRECT_FIELD
    ctx = bctx["ctx"]
    cams, cfgs = jobs(bctx, INDIRECT_FIELD)
    ctx.set_launch_mode(2, True)
    for shift in range(3):
        moved = [sg.make_camera(bctx["w"].seed, 100 + 7 * shift + i, c.width, c.height)
                 for i, c in enumerate(cams)]
        outs = ctx.render_batch(moved, cfgs)
        ctx.sync()
        ctx.set_launch_mode(0, False)
        ref = singles(ctx, moved, cfgs)
        ctx.set_launch_mode(2, True)
        for o, r in zip(outs, ref):
            np.testing.assert_array_equal(o.cpu().numpy(), r)
    ctx.set_launch_mode(0, False)


def test_batch_job_matches_oracle(orc, bctx):
    import torch
    from paper_2304_07338_amd.pfn import INDIRECT_FIELD
    ctx = bctx["ctx"]
    cams, cfgs = jobs(bctx, INDIRECT_FIELD)
    outs = ctx.render_batch(cams, cfgs)
    ctx.sync()
    os_ = oracle_scene(orc, bctx["vol"], bctx["tf"], bctx["lights"])
    from test_gpu_field import oracle_desc
    from paper_2304_07338_amd.pfn import FieldConfig
    desc = oracle_desc(orc, FieldConfig(log2_table=14))
    for i in (1, 5):
        ctx.field_select(cfgs[i].field_slot)
        p = ctx.field_get_params().cpu().numpy().astype(np.float64)
        op = orc.render_params(spp=cfgs[i].spp, t_min=1e-3, max_steps=400, field_stride=4,
                               g=cfgs[i].g, indirect=orc.IND_FIELD, direct=orc.DIR_LIGHTVOL,
                               light_mask=cfgs[i].light_mask, seed=cfgs[i].seed)
        ref = orc.render_pixels(os_, cams[i], op, field=(desc, p, 1, 1e-2))
        # binary16 light volume and field features; measured 1.2e-4 / 1.8e-4
        check_err(outs[i].cpu().numpy().reshape(-1, 3), ref, 1.5e-3, 2e-3,
                  f"job {i} ({cams[i].width}x{cams[i].height}, spp {cfgs[i].spp})")


def test_autotuner_picks_a_config_and_keeps_results_exact(bctx):
    from paper_2304_07338_amd.pfn import INDIRECT_FIELD
    ctx = bctx["ctx"]
    cams, cfgs = jobs(bctx, INDIRECT_FIELD)
    ctx.set_launch_mode(0, False)
    ctx.set_tile_config(8, 2, 2)
    ref = singles(ctx, cams, cfgs)
    best = ctx.autotune_batch(cams, cfgs, iters=1)
    say("  autotuner choice", best)
    assert best["tile_w"] in (4, 8, 16, 32) and best["block_w"] * best["block_h"] == 4
    assert best["ms"] > 0
    again = ctx.autotune_batch(cams, cfgs, iters=1)  # cached
    assert {k: again[k] for k in ("tile_w", "block_w", "block_h", "persistent")} == \
        {k: best[k] for k in ("tile_w", "block_w", "block_h", "persistent")}
    outs = ctx.render_batch(cams, cfgs)
    ctx.sync()
    for o, r in zip(outs, ref):
        np.testing.assert_array_equal(o.cpu().numpy(), r)
    ctx.set_launch_mode(0, False)
    ctx.set_tile_config(8, 2, 2)
