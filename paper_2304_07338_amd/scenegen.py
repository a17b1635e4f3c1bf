"""Seeded synthetic scene generator: volumes, transfer functions, lights, cameras.

This module produces the *inputs* of the method and nothing else: it holds none of the
method's arithmetic (no transport, no phase function, no encoding).  Both the HIP path and the
CPU oracle take its arrays as given.

The paper evaluates on seven scientific volumes (Table 3) that are not available here; these
synthetic volumes stand in for them at comparable sizes:
  - density = sum of B anisotropic Gaussian blobs + O octaves of value noise, clamped to [0,1];
  - transfer function = 256-entry RGBA table, piecewise linear through 4 seeded control points
    with an opacity-0 anchor at density 0 (opacity sets the extinction, RGB the albedo);
  - point lights at distance 1.2-1.6 from the cube centre;
  - pinhole cameras at distance 2.2 from the cube centre looking at it.
Random draws here use numpy's PCG64 seeded per purpose; they are input recipes, not the
method's random numbers (those come from Philox inside each implementation).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

# sub-stream ids of the generator (one per input kind)
SUB_VOLUME, SUB_TF, SUB_LIGHTS, SUB_CAMERAS, SUB_G = 1, 2, 3, 4, 5


def _rng(seed: int, sub: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(sub)])


@dataclasses.dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple
    fov_y_deg: float
    width: int
    height: int


@dataclasses.dataclass
class Light:
    pos: tuple
    intensity: tuple


def _rotation(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def blob_params(n_blobs: int, seed: int):
    r = _rng(seed, SUB_VOLUME)
    centres = r.uniform(0.15, 0.85, (n_blobs, 3))
    sigmas = r.uniform(3.0, 10.0, (n_blobs, 3)) / 64.0  # 3-10 voxels at 64^3, in cube units
    quats = r.normal(size=(n_blobs, 4))
    weights = r.uniform(0.5, 1.0, n_blobs)
    return centres, sigmas, quats, weights


def _interp_matrix(n: int, f: int):
    """Linear interpolation weights from f+1 lattice values on [0,1] to n voxel centres."""
    import torch
    u = (torch.arange(n, dtype=torch.float64) + 0.5) / n * f
    i0 = torch.clamp(torch.floor(u), max=f - 1).long()
    fr = u - i0
    M = torch.zeros((n, f + 1), dtype=torch.float64)
    M[torch.arange(n), i0] += 1.0 - fr
    M[torch.arange(n), i0 + 1] += fr
    return M


def make_volume(n: int, n_blobs: int, octaves: int, seed: int, dtype: str = "f32",
                device: str = "cpu"):
    """Density volume [n][n][n] (z, y, x; x fastest) as a torch tensor on `device`.

    dtype "f32" -> float32, "f16" -> float16 (round to nearest even).
    """
    import torch
    centres, sigmas, quats, weights = blob_params(n_blobs, seed)
    vol = torch.zeros((n, n, n), dtype=torch.float32, device=device)
    coords = (torch.arange(n, dtype=torch.float32, device=device) + 0.5) / n
    for b in range(n_blobs):
        R = torch.tensor(_rotation(quats[b]), dtype=torch.float32, device=device)
        c = centres[b]
        ext = 4.5 * float(sigmas[b].max())
        lo = [max(0, int(math.floor((c[a] - ext) * n))) for a in range(3)]
        hi = [min(n, int(math.ceil((c[a] + ext) * n)) + 1) for a in range(3)]
        xs = coords[lo[0]:hi[0]] - float(c[0])
        ys = coords[lo[1]:hi[1]] - float(c[1])
        zs = coords[lo[2]:hi[2]] - float(c[2])
        # local coordinates y = R^T (x - c); expand separably over the box
        inv = torch.tensor(1.0 / sigmas[b], dtype=torch.float32, device=device)
        e = torch.zeros((len(zs), len(ys), len(xs)), dtype=torch.float32, device=device)
        for a in range(3):
            comp = (zs[:, None, None] * R[2, a] + ys[None, :, None] * R[1, a]
                    + xs[None, None, :] * R[0, a]) * inv[a]
            e += comp * comp
        vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += float(weights[b]) * torch.exp(-0.5 * e)
    if octaves > 0:
        r = _rng(seed, SUB_VOLUME + 100)
        norm = sum(2.0 ** -o for o in range(octaves))
        for o in range(octaves):
            f = 8 * 2 ** o
            lat = torch.tensor(r.uniform(-1.0, 1.0, (f + 1, f + 1, f + 1)), dtype=torch.float32,
                               device=device)
            M = _interp_matrix(n, f).to(device=device, dtype=torch.float32)
            amp = 0.1 * 2.0 ** -o / norm
            # lat[k][j][i] -> noise[z][y][x] = sum M[z,k] M[y,j] M[x,i] lat[k,j,i]
            t = torch.tensordot(lat, M, dims=([2], [1]))            # [k][j][x]
            t = torch.tensordot(t, M, dims=([1], [1]))              # [k][x][y]
            t = torch.tensordot(t, M, dims=([0], [1]))              # [x][y][z]
            vol += amp * t.permute(2, 1, 0)
            del t
    vol.clamp_(0.0, 1.0)
    if dtype == "f16":
        return vol.to(torch.float16)
    return vol


def make_transfer_function(seed: int, n_points: int = 4) -> np.ndarray:
    """256 x RGBA float32 table sampled at density e/255."""
    r = _rng(seed, SUB_TF)
    pos = np.sort(r.uniform(0.1, 0.9, n_points))
    rgb = r.uniform(0.3, 1.0, (n_points, 3))
    a = r.uniform(0.1, 1.0, n_points)
    xs = np.concatenate([[0.0], pos])
    cols = np.concatenate([np.concatenate([rgb[:1], [[0.0]]], axis=1),
                           np.concatenate([rgb, a[:, None]], axis=1)], axis=0)
    e = np.arange(256) / 255.0
    table = np.stack([np.interp(e, xs, cols[:, c]) for c in range(4)], axis=1)
    return table.astype(np.float32)


def make_lights(n_lights: int, seed: int) -> List[Light]:
    r = _rng(seed, SUB_LIGHTS)
    out = []
    for l in range(n_lights):
        v = r.normal(size=3)
        v /= np.linalg.norm(v)
        rad = r.uniform(1.2, 1.6)
        p = 0.5 + rad * v
        inten = (1.0, 1.0, 1.0) if l == 0 else tuple(float(t) for t in r.uniform(0.5, 1.5, 3))
        out.append(Light(tuple(float(t) for t in p), inten))
    return out


def lights_array(lights: List[Light]) -> np.ndarray:
    return np.array([list(l.pos) + list(l.intensity) for l in lights], dtype=np.float64)


def make_camera(seed: int, index: int, width: int, height: int, fov_y_deg: float = 40.0,
                distance: float = 2.2) -> Camera:
    r = np.random.default_rng([int(seed), SUB_CAMERAS, int(index)])
    v = r.normal(size=3)
    v /= np.linalg.norm(v)
    eye = 0.5 + distance * v
    up = (0.0, 0.0, 1.0)
    if abs(v[2]) > 0.99:
        up = (0.0, 1.0, 0.0)
    return Camera(tuple(float(t) for t in eye), (0.5, 0.5, 0.5), up, float(fov_y_deg), int(width),
                  int(height))


def uniform_g(seed: int, n: int, lo: float = -0.9, hi: float = 0.9) -> np.ndarray:
    return _rng(seed, SUB_G).uniform(lo, hi, n)


def homogeneous_volume(n: int, value: float) -> np.ndarray:
    return np.full((n, n, n), value, dtype=np.float32)
