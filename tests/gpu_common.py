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


def volume_as(vol_t, dtype: str):
    """The volume as the library receives it: "f32" as is, "f16" rounded to binary16 (the
    oracle then gets the rounded values, exactly, in FP64)."""
    import torch
    return vol_t.float() if dtype == "f32" else vol_t.to(torch.float16)


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


# The library forms the normalised spherical coordinates (theta/pi, (phi+pi)/(2pi)) of a view
# direction in FP32: acosf / atan2f (a few ulps of an angle up to 2 pi), the shift by pi and the
# scaling each round once.  Their error stays below 8 ulps of 1 in either coordinate; the FP64
# oracle takes the exact coordinates.  Bars on results that depend on the direction are derived
# by moving the oracle's coordinates by this much.
DIR_COORD_EPS = 8.0 * 2.0 ** -24
# Typical size of that error for sums over many directions (gradients): 4 ulps of 1, random
# signs per direction (acosf and atan2f are within 2 ulps of the angle; the angle's ulp near pi is
# 2^-22, which is 2.6 ulps of 1 after the division by pi, plus the roundings of the shift and
# scaling).
DIR_JITTER_EPS = 4.0 * 2.0 ** -24


def dir_coords(w):
    w = np.asarray(w, dtype=np.float64).reshape(-1, 3)
    u0 = np.arccos(np.clip(w[:, 2], -1.0, 1.0)) / np.pi
    u1 = (np.arctan2(w[:, 1], w[:, 0]) + np.pi) / (2.0 * np.pi)
    return u0, u1


def dir_from_coords(u0, u1):
    th = np.pi * np.clip(u0, 0.0, 1.0)
    ph = 2.0 * np.pi * np.clip(u1, 0.0, 1.0) - np.pi
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def coord_moves(w, eps=DIR_COORD_EPS):
    """Directions with one normalised coordinate moved by +-eps: [(axis, sign, dirs)]."""
    u0, u1 = dir_coords(w)
    out = []
    for axis in (0, 1):
        for s in (1.0, -1.0):
            a0 = u0 + s * eps if axis == 0 else u0
            a1 = u1 + s * eps if axis == 1 else u1
            out.append((axis, s, dir_from_coords(a0, a1)))
    return out


def coord_jitter(w, seed, eps=DIR_JITTER_EPS):
    """Directions with both normalised coordinates moved by eps with random signs."""
    u0, u1 = dir_coords(w)
    rng = np.random.default_rng(seed)
    s = rng.choice([-1.0, 1.0], size=(u0.size, 2))
    return dir_from_coords(u0 + s[:, 0] * eps, u1 + s[:, 1] * eps)


def coord_sensitivity(fwd, w):
    """Per query and channel: sum over the two coordinates of the largest change of fwd(dirs)
    when that coordinate moves by +-DIR_COORD_EPS (fwd maps [n][3] directions to [n][3])."""
    base = fwd(np.asarray(w, dtype=np.float64))
    per_axis = [np.zeros_like(base), np.zeros_like(base)]
    for axis, _, d in coord_moves(w):
        per_axis[axis] = np.maximum(per_axis[axis], np.abs(fwd(d) - base))
    return per_axis[0] + per_axis[1]


def err_stats(got, ref):
    """rel-RMSE, largest |difference| / max|ref| and its 99th percentile, over all values."""
    a = np.asarray(got, dtype=np.float64).ravel()
    b = np.asarray(ref, dtype=np.float64).ravel()
    d = np.abs(a - b) / max(float(np.abs(b).max()), 1e-300)
    return dict(rel_rmse=rel_rmse(a, b), max_rel=float(d.max()),
                p99_rel=float(np.percentile(d, 99)) if d.size else 0.0)


def check_err(got, ref, rel_rmse_bar, max_rel_bar, label=""):
    """Print the error statistics of got against ref and assert both bars."""
    s = err_stats(got, ref)
    say(f"  {label} rel-RMSE {s['rel_rmse']:.3e} (bar {rel_rmse_bar:.1e}), max|d|/max|ref| "
        f"{s['max_rel']:.3e} (bar {max_rel_bar:.1e}), p99 {s['p99_rel']:.3e}")
    assert s["rel_rmse"] <= rel_rmse_bar, label
    assert s["max_rel"] <= max_rel_bar, label
    return s


def oracle_desc(orc, cfg):
    return orc.field_desc(levels=cfg.levels, feats=cfg.feats_per_level, base_res=cfg.base_res,
                          growth=cfg.growth, log2_table=cfg.log2_table,
                          hidden_layers=cfg.hidden_layers, width=cfg.width, psi=cfg.psi)


def random_params(orc, desc, seed, grid_scale=0.5, out_scale=0.3):
    """Parameters that exercise every part of the field (not the tiny initial grid values)."""
    L = orc.field_layout(desc)
    rng = np.random.default_rng(seed)
    p = np.zeros(L.n_params, dtype=np.float32)
    p[:L.mlp_off] = rng.uniform(-grid_scale, grid_scale, L.mlp_off)
    for m in range(L.n_mats):
        r, c = L.w_rows[m], L.w_cols[m]
        lim = np.sqrt(6.0 / (r + c))
        w = rng.uniform(-lim, lim, r * c)
        if m == L.n_mats - 1:
            w *= out_scale
        p[L.w_off[m]:L.w_off[m] + r * c] = w
    return p
