"""The entry point that allocates nothing (pfn_image_error_noalloc) against pfn_image_error:
two calls in a row, the second with a smaller input, and the size limit."""
import numpy as np
import pytest

from gpu_common import gpu_context, say, scene_arrays

pytestmark = pytest.mark.gpu

MAX_N = 2048 * 256 * 64


def test_noalloc_image_error_matches_the_allocating_call():
    import torch
    from paper_2304_07338_amd.pfn import PfnError
    w, vol, tf, lights = scene_arrays("c0")
    ctx = gpu_context(vol, tf, lights)
    rng = np.random.default_rng(3)
    out = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    for n in (3 * 1920 * 1080 + 7, 1000):  # several partial blocks and a ragged tail, then one
        ref = rng.uniform(0.0, 2.0, n).astype(np.float32)
        img = (ref + rng.normal(scale=0.02, size=n)).astype(np.float32)
        dimg, dref = torch.tensor(img, device="cuda:0"), torch.tensor(ref, device="cuda:0")
        ctx.image_error_noalloc(dimg, dref, out)
        ctx.sync()
        got = out.cpu().numpy()
        want = np.array(ctx.image_error(dimg, dref))
        d = img.astype(np.float64) - ref
        rm = np.sqrt(np.mean(d * d))
        exact = np.array([rm, rm / ref.astype(np.float64).mean(), 20 * np.log10(ref.max() / rm)])
        say(f"  n={n}: {got} vs {want}; rel diff {np.abs(got / want - 1).max():.2e}")
        # FP64 sums in two orders: agreement to a few FP64 roundings per added term
        np.testing.assert_allclose(got, want, rtol=1e-12)
        np.testing.assert_allclose(got, exact, rtol=1e-12)
    # the size limit is checked before anything runs
    big = torch.zeros(MAX_N + 1, dtype=torch.float32, device="cuda:0")
    with pytest.raises(PfnError) as e:
        ctx.image_error_noalloc(big, big, out)
    assert e.value.status == -1
    ctx.image_error_noalloc(big[:MAX_N], big[:MAX_N], out)  # at the limit: RMSE 0
    ctx.sync()
    assert out[0].item() == 0.0
    ctx.close()
