"""The synthetic workloads the library is measured and checked on.

Sizes follow the configurations the build targets; the paper's scientific volumes (Table 3:
128^3 to 1024x1024x1080) are replaced by seeded synthetic volumes of comparable sizes.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

from . import scenegen as sg

C1_G_BINS = (-0.8, -0.4, 0.0, 0.4, 0.8)


@dataclasses.dataclass
class Workload:
    name: str
    n: int                  # volume resolution per axis
    vol_dtype: str          # "f32" or "f16"
    blobs: int
    octaves: int
    n_lights: int
    seed: int
    extinction: float = 20.0
    width: int = 128
    height: int = 128


# plain method, CPU-oracle-sized: 64^3 f32, 8 blobs, 2 octaves, 1 light, 128x128, 32^3 cache
C0 = Workload("c0_plain_64cube_128px", 64, "f32", 8, 2, 1, 1234, width=128, height=128)
# photon cache + field training: 256^3 f32, 32 blobs, 4 octaves, 3 lights, 2^22 photons
C1 = Workload("c1_cache_train_256cube", 256, "f32", 32, 4, 3, 2234)
# field inference render: 512^3 f16, 64 blobs, 4 octaves, 3 lights, 1920x1080
C2 = Workload("c2_field_render_512cube_1080p", 512, "f16", 64, 4, 3, 3234, width=1920,
              height=1080)
# batched persistent launch: 256^3 f32 (as C1), 16 cameras x 4 light positions
C3 = Workload("c3_batch_64jobs_256cube", 256, "f32", 32, 4, 4, 4234)
# large scale: 1024^3 f16, 256 blobs, 6 octaves, 3 lights, 1080p
C4 = Workload("c4_large_1024cube_1080p", 1024, "f16", 256, 6, 3, 5234, width=1920, height=1080)


def make_scene(w: Workload, device: str = "cpu", n: Optional[int] = None):
    """(density tensor, transfer function table, lights) of a workload (optionally resized)."""
    res = n or w.n
    vol = sg.make_volume(res, w.blobs, w.octaves, w.seed, w.vol_dtype, device=device)
    tf = sg.make_transfer_function(w.seed)
    lights = sg.make_lights(w.n_lights, w.seed)
    return vol, tf, lights


def camera(w: Workload, index: int = 0, width: Optional[int] = None, height: Optional[int] = None):
    return sg.make_camera(w.seed, index, width or w.width, height or w.height)


def batch_jobs(w: Workload = C3, n_cameras: int = 16, side_lo: int = 256, side_hi: int = 1024):
    """The batched-launch workload: n_cameras seeded views with width and height each drawn
    uniformly from {side_lo..side_hi}, times one job per light of the scene.  Job i of light l
    lights the volume with light l only, reads field slot l (one single-light field per light
    position) and takes its own g ~ U[-0.9, 0.9].  Returns (cameras, render configs) without
    the indirect mode, which the caller sets."""
    import numpy as np
    from .pfn import RenderConfig, DIRECT_LIGHT_VOLUME
    r = np.random.default_rng([int(w.seed), sg.SUB_CAMERAS, 7919])
    sides = r.integers(side_lo, side_hi + 1, size=(n_cameras, 2))
    g = sg.uniform_g(w.seed, n_cameras * w.n_lights)
    cams, cfgs = [], []
    for c in range(n_cameras):
        cam = sg.make_camera(w.seed, c, int(sides[c, 0]), int(sides[c, 1]))
        for l in range(w.n_lights):
            k = c * w.n_lights + l
            cams.append(cam)
            cfgs.append(RenderConfig(spp=1, step_voxels=0.5, max_steps=1024, t_min=1e-3,
                                     field_stride=4, g=float(g[k]), direct=DIRECT_LIGHT_VOLUME,
                                     light_mask=1 << l, field_slot=l, seed=k))
    return cams, cfgs
