"""A context moved to another stream (pfn_set_stream): its work is ordered on that stream, and a
frame rendered there, in the fused kernel and in the wavefront rounds (whose side streams wait
on the context's stream), equals the frame rendered on the default stream bit for bit."""
import numpy as np
import pytest

from gpu_common import gpu_context, say, scene_arrays

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("strategy", ["fused", "wavefront"])
def test_render_on_another_stream_is_identical(strategy):
    import torch
    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd.pfn import (FieldConfig, RenderConfig, DIRECT_LIGHT_VOLUME,
                                          INDIRECT_FIELD)
    w, vol, tf, lights = scene_arrays("c0")
    ctx = gpu_context(vol, tf, lights)
    ctx.build_light_volume(0.5)
    ctx.field_init(FieldConfig(log2_table=14), seed=4)
    ctx.field_set_kappa(1e-2)
    ctx.set_render_strategy(strategy)
    cam = sg.make_camera(w.seed, 2, 57, 41)
    cfg = RenderConfig(spp=2, t_min=1e-3, field_stride=2, g=0.3, indirect=INDIRECT_FIELD,
                       direct=DIRECT_LIGHT_VOLUME, seed=9)
    ref = ctx.render_frame(cam, cfg)
    ctx.sync()
    ref = ref.cpu().numpy()
    side = torch.cuda.Stream()  # default priority
    ctx.set_stream(side)
    with torch.cuda.stream(side):
        out = torch.full((cam.height, cam.width, 3), -1.0, dtype=torch.float32, device="cuda:0")
        for _ in range(3):
            ctx.render_frame(cam, cfg, out)
        # ordered after the renders on the same stream, without a device synchronisation
        got = out.to("cpu", non_blocking=False)
    side.synchronize()
    say(f"  {strategy}: mean {ref.mean():.4g}")
    assert ref.mean() > 0
    np.testing.assert_array_equal(got.numpy(), ref)
    ctx.set_stream(torch.cuda.current_stream(0))
    ctx.set_render_strategy("auto")
    ctx.close()
