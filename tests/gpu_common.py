"""Shared set-up of the GPU parity tests: scenes built once from the seeded generator, given to
both the HIP library (through the C ABI) and the FP64 oracle."""
import functools

import numpy as np

from paper_2304_07338_amd import scenegen as sg
from paper_2304_07338_amd import workloads as wl


def say(*a):
    print(*a, flush=True)


@functools.lru_cache(maxsize=None)
def scene_arrays(name: str, n: int = 0):
    w = {"c0": wl.C0, "c1": wl.C1, "c2": wl.C2, "c3": wl.C3, "c4": wl.C4}[name]
    vol, tf, lights = wl.make_scene(w, device="cpu", n=n or None)
    return w, vol, tf, sg.lights_array(lights)


def oracle_scene(orc, vol_t, tf, lights, ext=20.0):
    return orc.OracleScene(vol_t.float().numpy().astype(np.float64), tf.astype(np.float64), ext,
                           lights)


def gpu_context(vol_t, tf, lights, ext=20.0):
    import torch
    from paper_2304_07338_amd.pfn import Context
    ctx = Context(0)
    dv = vol_t.to("cuda:0").contiguous()
    ctx.set_volume(dv)
    ctx.set_transfer_function(tf, ext)
    ctx.set_lights(lights)
    ctx.sync()
    return ctx


def smooth_cache(res: int, n_bins: int, seed: int = 0):
    """A smooth positive synthetic cache (an input array for render parity)."""
    rng = np.random.default_rng(seed)
    c = (np.arange(res) + 0.5) / res
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    out = np.zeros((n_bins, res, res, res, 3))
    for b in range(n_bins):
        for ch in range(3):
            k = rng.uniform(1, 4, 3)
            ph = rng.uniform(0, 6.28, 3)
            out[b, ..., ch] = 0.02 * (1.5 + np.sin(k[0] * 6.28 * xx + ph[0])
                                      * np.cos(k[1] * 6.28 * yy + ph[1])) * (1 + 0.5 * zz)
    return out


def rel_rmse(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.mean(np.abs(b)), 1e-300))
