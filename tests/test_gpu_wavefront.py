"""The wavefront form of the field-lit ray marcher (march rounds, level-major position encoding,
matrix-core field tiles) against the fused kernel and the FP64 oracle.

Both forms run the same per-ray arithmetic; they differ in the order in which the FP32 terms
W * L_i are added to a pixel, so they agree to FP32 rounding (measured at most 6.1e-7 relative
RMSE and 5.7e-7 of the image maximum per value; bars 6e-6 for both) and give
identical march-step and query counts.  Cases cover many rounds per ray (stride 1, where a ray
stores up to 32 queries per round), frames of more ray samples than one round holds (2^21),
ragged tiles, several samples per pixel, every matrix-core precision, both direct-light modes,
and a batch of jobs that must render exactly as its jobs do alone."""
import numpy as np
import pytest

from gpu_common import check_err, gpu_context, oracle_scene, say, scene_arrays
from paper_2304_07338_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wctx(orc):
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig
    w, vol, tf, lights = scene_arrays("c0")
    ctx = gpu_context(vol, tf, lights)
    ctx.build_light_volume(0.5)
    ctx.field_select(0)
    ctx.field_init(FieldConfig(log2_table=14), seed=4)
    p = ctx.field_get_params()
    g = torch.Generator(device="cuda:0").manual_seed(4)
    p = p + 0.3 * torch.rand(p.shape, device="cuda:0", generator=g) - 0.15
    ctx.field_set_params(p.contiguous())
    ctx.field_set_kappa(1e-2)
    return dict(w=w, ctx=ctx, vol=vol, tf=tf, lights=lights)


def _cfg(**kw):
    from paper_2304_07338_amd.pfn import RenderConfig, INDIRECT_FIELD, DIRECT_LIGHT_VOLUME
    base = dict(spp=1, t_min=1e-3, max_steps=400, field_stride=4, g=0.35, indirect=INDIRECT_FIELD,
                direct=DIRECT_LIGHT_VOLUME, field_precision="f16", field_slot=0, seed=9)
    base.update(kw)
    return RenderConfig(**base)


def _both(ctx, cam, cfg):
    out = {}
    for strategy in ("fused", "wavefront"):
        ctx.set_render_strategy(strategy)
        ctx.count_enable(True)
        img = ctx.render_frame(cam, cfg)
        counts = ctx.count_get()
        ctx.count_enable(False)
        ctx.sync()
        out[strategy] = (img.cpu().numpy(), counts)
    ctx.set_render_strategy("auto")
    return out


CASES = [
    # (width, height, spp, stride, precision, direct, tag)
    (64, 48, 1, 4, "f16", 1, "plain"),
    (37, 23, 3, 4, "bf16", 1, "ragged, 3 spp"),
    (40, 40, 1, 1, "f32", 0, "stride 1 (many rounds), shadow rays"),
    (50, 30, 2, 2, "f16", 0, "stride 2, 2 spp, shadow rays"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[-1] for c in CASES])
def test_wavefront_matches_fused(wctx, case):
    wd, ht, spp, stride, prec, direct, tag = case
    cam = sg.make_camera(wctx["w"].seed, 21, wd, ht)
    cfg = _cfg(spp=spp, field_stride=stride, field_precision=prec, direct=direct,
               max_steps=1 << 20 if stride == 1 else 400, t_min=0.0 if stride == 1 else 1e-3)
    r = _both(wctx["ctx"], cam, cfg)
    (a, ca), (b, cb) = r["fused"], r["wavefront"]
    say(f"  {tag}: counts {ca} / {cb}, mean {a.mean():.4g}")
    assert a.mean() > 0
    assert tuple(ca) == tuple(cb)
    check_err(b, a, 6e-6, 6e-6, f"{tag}: wavefront vs fused")


def test_wavefront_matches_oracle(orc, wctx):
    from test_gpu_field import oracle_desc
    from paper_2304_07338_amd.pfn import FieldConfig
    ctx = wctx["ctx"]
    ctx.set_render_strategy("wavefront")
    cam = sg.make_camera(wctx["w"].seed, 22, 30, 26)
    cfg = _cfg(spp=2, field_precision="f32", field_stride=3)
    img = ctx.render_frame(cam, cfg)
    ctx.sync()
    ctx.set_render_strategy("auto")
    os_ = oracle_scene(orc, wctx["vol"], wctx["tf"], wctx["lights"])
    desc = oracle_desc(orc, FieldConfig(log2_table=14))
    p = ctx.field_get_params().cpu().numpy().astype(np.float64)
    op = orc.render_params(spp=2, t_min=1e-3, max_steps=400, field_stride=3, g=0.35,
                           indirect=orc.IND_FIELD, direct=orc.DIR_LIGHTVOL, seed=9)
    ref = orc.render_pixels(os_, cam, op, field=(desc, p, 0, 1e-2))
    # the light-transmittance volume is stored in binary16; measured 8.9e-5 / 8.3e-5
    check_err(img.cpu().numpy().reshape(-1, 3), ref, 6e-4, 1e-3, "wavefront f32 vs oracle")


@pytest.mark.parametrize("levels", [12, 8, 6])
def test_wavefront_level_counts(wctx, levels):
    """8 to 16 levels are encoded in one launch with the levels paired over the XCDs (with 12
    levels, four XCDs hold two levels and four hold one); fewer levels take the grouped
    launches.  Either way the image and counts equal the fused kernel's."""
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig
    ctx = wctx["ctx"]
    ctx.field_select(2)
    ctx.field_init(FieldConfig(levels=levels, log2_table=14), seed=6)
    p = ctx.field_get_params()
    g = torch.Generator(device="cuda:0").manual_seed(6)
    ctx.field_set_params((p + 0.3 * torch.rand(p.shape, device="cuda:0", generator=g) - 0.15)
                         .contiguous())
    ctx.field_set_kappa(1e-2)
    cam = sg.make_camera(wctx["w"].seed, 25, 48, 36)
    r = _both(ctx, cam, _cfg(spp=2, field_slot=2))
    (a, ca), (b, cb) = r["fused"], r["wavefront"]
    assert a.mean() > 0
    assert tuple(ca) == tuple(cb)
    check_err(b, a, 6e-6, 6e-6, f"{levels} levels: wavefront vs fused")


def test_wavefront_frame_larger_than_one_round(wctx):
    """1280 x 960 at 2 spp is 2,457,600 ray samples: more than the 2^21 rays of a round, so fresh
    rays enter over two rounds while the first rays continue."""
    cam = sg.make_camera(wctx["w"].seed, 23, 1280, 960)
    cfg = _cfg(spp=2, field_stride=4)
    r = _both(wctx["ctx"], cam, cfg)
    (a, ca), (b, cb) = r["fused"], r["wavefront"]
    assert tuple(ca) == tuple(cb)
    check_err(b, a, 6e-6, 6e-6, "1280x960x2: wavefront vs fused")


def test_wavefront_batch_equals_single_renders(wctx):
    ctx = wctx["ctx"]
    ctx.set_render_strategy("wavefront")
    sizes = [(17, 23), (64, 48), (1, 1), (55, 66), (33, 9)]
    g_vals = sg.uniform_g(5, len(sizes))
    cams = [sg.make_camera(wctx["w"].seed, 30 + i, wd, ht) for i, (wd, ht) in enumerate(sizes)]
    cfgs = [_cfg(spp=1 + i % 3, g=float(g_vals[i]), light_mask=1, seed=i) for i in range(len(sizes))]
    singles = []
    for c, f in zip(cams, cfgs):
        singles.append(ctx.render_frame(c, f).clone())
    ctx.sync()
    for rep in range(2):
        outs = ctx.render_batch(cams, cfgs)
        ctx.sync()
        for o, s1 in zip(outs, singles):
            np.testing.assert_array_equal(o.cpu().numpy(), s1.cpu().numpy())
    ctx.set_render_strategy("auto")


@pytest.mark.parametrize("wd,ht,spp,stride", [(40, 40, 1, 1), (1280, 960, 2, 4)])
def test_overlapped_rounds_equal_serial_rounds(wctx, wd, ht, spp, stride):
    """The march kernel of round r+1 running beside the encoding and field kernels of round r
    (two streams) gives exactly the image of the rounds run one after another."""
    ctx = wctx["ctx"]
    cam = sg.make_camera(wctx["w"].seed, 24, wd, ht)
    cfg = _cfg(spp=spp, field_stride=stride, max_steps=1 << 20 if stride == 1 else 400,
               t_min=0.0 if stride == 1 else 1e-3)
    imgs = {}
    for strategy in ("wavefront_serial", "wavefront"):
        ctx.set_render_strategy(strategy)
        for rep in range(2):
            imgs[(strategy, rep)] = ctx.render_frame(cam, cfg).cpu().numpy()
    ctx.set_render_strategy("auto")
    ref = imgs[("wavefront_serial", 0)]
    assert ref.mean() > 0
    for k, v in imgs.items():
        np.testing.assert_array_equal(v, ref, err_msg=str(k))


def test_wavefront_batch_with_two_field_slots(wctx):
    """A batch whose jobs read two field slots runs one pass of rounds per slot and still
    renders every job exactly as alone."""
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig
    ctx = wctx["ctx"]
    ctx.field_select(1)
    ctx.field_init(FieldConfig(log2_table=14), seed=5)
    p = ctx.field_get_params()
    g = torch.Generator(device="cuda:0").manual_seed(5)
    ctx.field_set_params((p + 0.3 * torch.rand(p.shape, device="cuda:0", generator=g) - 0.15)
                         .contiguous())
    ctx.field_set_kappa(1e-2)
    ctx.set_render_strategy("wavefront")
    sizes = [(31, 17), (48, 40), (9, 64), (40, 33)]
    cams = [sg.make_camera(wctx["w"].seed, 40 + i, wd, ht) for i, (wd, ht) in enumerate(sizes)]
    cfgs = [_cfg(spp=1 + i % 2, field_slot=i % 2, seed=i) for i in range(len(sizes))]
    singles = [ctx.render_frame(c, f).clone() for c, f in zip(cams, cfgs)]
    outs = ctx.render_batch(cams, cfgs)
    ctx.sync()
    ctx.set_render_strategy("auto")
    assert float(singles[0].mean()) != float(singles[1].mean())
    for o, s1 in zip(outs, singles):
        np.testing.assert_array_equal(o.cpu().numpy(), s1.cpu().numpy())


@pytest.mark.parametrize("use_graph", [False, True])
def test_autotuner_chooses_among_forms_and_keeps_results_exact(wctx, use_graph):
    """The autotuner times the fused kernel (graph-replayed when asked) and the wavefront rounds
    and makes the faster the context's form; later renders use that form, whatever the graph
    setting, and a batch still renders every job exactly as alone."""
    ctx = wctx["ctx"]
    ctx.set_render_strategy("auto")
    ctx.set_launch_mode(0, use_graph)
    sizes = [(64, 40), (33, 70), (80, 24)]
    cams = [sg.make_camera(wctx["w"].seed, 50 + i, wd, ht) for i, (wd, ht) in enumerate(sizes)]
    cfgs = [_cfg(spp=1, field_slot=0, seed=i) for i in range(len(sizes))]
    best = ctx.autotune_batch(cams, cfgs, iters=1)
    say("  autotuner choice", best)
    assert best["strategy"] in ("fused", "wavefront")
    singles = [ctx.render_frame(c, f).clone() for c, f in zip(cams, cfgs)]
    outs = ctx.render_batch(cams, cfgs)
    ctx.sync()
    for o, s1 in zip(outs, singles):
        np.testing.assert_array_equal(o.cpu().numpy(), s1.cpu().numpy())
    ctx.set_render_strategy("auto")
    ctx.set_tile_config(8, 2, 2)
    ctx.set_launch_mode(0, False)
