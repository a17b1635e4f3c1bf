"""The synthetic workloads the library is measured and checked on.

Sizes follow the configurations the build targets; the paper's scientific volumes (Table 3:
128^3 to 1024x1024x1080) are replaced by seeded synthetic volumes of comparable sizes.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

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
