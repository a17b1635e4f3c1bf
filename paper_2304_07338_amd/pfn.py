"""Python binding of the photon-field library (include/pfn.h): argument marshalling only.

Every call goes to the HIP library libpfn.so; there is no fallback.  Device buffers are torch
tensors on the context's GPU; the library works on torch's current HIP stream unless another
stream is given.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import _ffi
from ._ffi import (DIRECT_LIGHT_VOLUME, DIRECT_SHADOW_RAYS, INDIRECT_CACHE, INDIRECT_FIELD,
                   INDIRECT_NONE, PFN_BF16, PFN_F16, PFN_F32)

DTYPES = {"f32": PFN_F32, "f16": PFN_F16, "bf16": PFN_BF16}
STRATEGIES = {"auto": 0, "fused": 1, "wavefront": 2, "wavefront_serial": 3}


class PfnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pfn error {_ffi.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


@dataclasses.dataclass
class FieldConfig:
    levels: int = 16
    feats_per_level: int = 2
    base_res: int = 16
    growth: float = 1.5
    log2_table: int = 19
    hidden_layers: int = 3
    width: int = 64
    psi: float = 5.0

    def struct(self) -> _ffi.FieldDesc:
        return _ffi.FieldDesc(self.levels, self.feats_per_level, self.base_res, self.growth,
                              self.log2_table, self.hidden_layers, self.width, self.psi)


@dataclasses.dataclass
class RenderConfig:
    spp: int = 1
    step_voxels: float = 0.5
    max_steps: int = 1 << 30
    t_min: float = 0.0
    field_stride: int = 1
    g: float = 0.0
    indirect: int = INDIRECT_NONE
    direct: int = DIRECT_SHADOW_RAYS
    field_precision: str = "f16"
    light_mask: int = 0
    field_slot: int = 0
    seed: int = 0

    def struct(self) -> _ffi.RenderParams:
        return _ffi.RenderParams(self.spp, self.step_voxels, min(self.max_steps, 2 ** 31 - 1),
                                 self.t_min, self.field_stride, self.g, self.indirect,
                                 self.direct, DTYPES[self.field_precision], self.light_mask,
                                 self.field_slot, self.seed)


LOSSES = {"l2": 0, "rel": 1}
G_SAMPLING = {"pool": 0, "uniform": 1}


@dataclasses.dataclass
class TrainConfig:
    steps: int = 2000
    log2_batch: int = 18
    lr: float = 9e-4
    beta1: float = 0.9
    beta2: float = 0.99
    eps: float = 1e-15
    decay: float = 0.92
    decay_start: int = 1400
    decay_interval: int = 25
    precision: str = "f16"
    seed: int = 0
    target: str = "cache"   # or "photon_map" (Eq. 5)
    knn_k: int = 0
    radius: float = 0.05
    staggered: bool = False
    loss: str = "l2"        # or "rel" (relative L2 of Section 3.5.1)
    g_sampling: str = "pool"  # or "uniform": g uniform between the first and last bin

    def struct(self) -> _ffi.TrainParams:
        return _ffi.TrainParams(self.steps, self.log2_batch, self.lr, self.beta1, self.beta2,
                                self.eps, self.decay, self.decay_start, self.decay_interval,
                                DTYPES[self.precision], self.seed,
                                {"cache": 0, "photon_map": 1}[self.target], self.knn_k,
                                self.radius, int(self.staggered), LOSSES[self.loss],
                                G_SAMPLING[self.g_sampling])


def train_step_radius(cfg: "TrainConfig", step: int) -> float:
    """The photon-map query radius that training uses at `step` (host only)."""
    lib = _ffi.load()
    r = C.c_float()
    p = cfg.struct()
    st = lib.pfn_train_step_radius(C.byref(p), step, C.byref(r))
    if st != 0:
        raise PfnError(st, "pfn_train_step_radius: bad arguments")
    return r.value


def train_lr_at(cfg: "TrainConfig", step: int) -> float:
    """The learning rate that training applies at `step` (host only)."""
    lib = _ffi.load()
    r = C.c_float()
    p = cfg.struct()
    st = lib.pfn_train_lr_at(C.byref(p), step, C.byref(r))
    if st != 0:
        raise PfnError(st, "pfn_train_lr_at: bad arguments")
    return r.value


def camera_struct(cam) -> _ffi.CameraS:
    c = _ffi.CameraS()
    for i in range(3):
        c.eye[i] = cam.eye[i]
        c.target[i] = cam.target[i]
        c.up[i] = cam.up[i]
    c.fov_y_deg = cam.fov_y_deg
    c.width = cam.width
    c.height = cam.height
    return c


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _check(t, dtype, numel=None, name="tensor"):
    import torch
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")


class Context:
    """One library context on one GPU (a thin owner of pfn_context)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = _ffi.load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.pfn_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != 0:
            raise PfnError(st, "pfn_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.pfn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, st: int):
        if st != 0:
            msg = self.lib.pfn_last_error(self.h)
            raise PfnError(st, msg.decode() if msg else "")

    # ------------------------------------------------------------------ scene
    def sync(self):
        self._ok(self.lib.pfn_sync(self.h))

    def set_stream(self, stream):
        """Enqueue later work on `stream` (a torch.cuda.Stream); waits for the current one."""
        self._ok(self.lib.pfn_set_stream(self.h, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def set_volume(self, density):
        import torch
        dt = {torch.float32: PFN_F32, torch.float16: PFN_F16}[density.dtype]
        nz, ny, nx = density.shape
        self._ok(self.lib.pfn_set_volume(self.h, _ptr(density), dt, nx, ny, nz))
        self._vol_shape = (nz, ny, nx)

    def set_transfer_function(self, table: np.ndarray, extinction_scale: float):
        t = np.ascontiguousarray(table, dtype=np.float32).reshape(256 * 4)
        self._ok(self.lib.pfn_set_transfer_function(
            self.h, t.ctypes.data_as(C.POINTER(C.c_float)), float(extinction_scale)))

    def set_lights(self, lights):
        """lights: array [n][6] (position, intensity) or a list of scenegen.Light."""
        arr = np.array([list(l.pos) + list(l.intensity) if hasattr(l, "pos") else list(l)
                        for l in lights], dtype=np.float64).reshape(-1, 6)
        buf = (_ffi.PointLight * len(arr))()
        for i, r in enumerate(arr):
            for c in range(3):
                buf[i].pos[c] = r[c]
                buf[i].intensity[c] = r[3 + c]
        self._ok(self.lib.pfn_set_lights(self.h, buf, len(arr)))

    def build_light_volume(self, step_voxels: float = 0.5):
        self._ok(self.lib.pfn_build_light_volume(self.h, step_voxels))

    def get_light_volume(self):
        """The light-transmittance grid as float16 [rz][ry][rx][4] (channel = light)."""
        import torch
        rz, ry, rx = ((n + 1) // 2 for n in self._vol_shape)
        out = torch.empty((rz, ry, rx, 4), dtype=torch.float16, device=f"cuda:{self.device}")
        self._ok(self.lib.pfn_get_light_volume(self.h, _ptr(out), rx * ry * rz))
        return out

    # ------------------------------------------------------------------ photon cache
    def trace_photon_cache(self, n_photons: int, g_bins: Sequence[float], cache_res: int,
                           seed: int = 0, max_collisions: int = 8, rr_start: int = 3) -> dict:
        p = _ffi.TraceParams()
        p.n_photons = n_photons
        p.n_bins = len(g_bins)
        for i, g in enumerate(g_bins):
            p.g_bins[i] = g
        p.cache_res = cache_res
        p.max_collisions = max_collisions
        p.rr_start = rr_start
        p.seed = seed
        s = _ffi.TraceStats()
        self._ok(self.lib.pfn_trace_photon_cache(self.h, C.byref(p), C.byref(s)))
        out = {}
        for name, _ in s._fields_:
            v = getattr(s, name)
            out[name] = np.array(list(v)) if hasattr(v, "__len__") else v
        return out

    def get_records(self, capacity: int):
        import torch
        dev = f"cuda:{self.device}"
        x = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        w = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        p = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        b = torch.empty(capacity, dtype=torch.int32, device=dev)
        ph = torch.empty(capacity, dtype=torch.int64, device=dev)
        n = C.c_uint64()
        self._ok(self.lib.pfn_get_records(self.h, _ptr(x), _ptr(w), _ptr(p), _ptr(b), _ptr(ph),
                                          capacity, C.byref(n)))
        k = n.value
        return dict(x=x[:k], w=w[:k], power=p[:k], bin=b[:k], photon=ph[:k])

    # -------------------------------------------------------------- photon map (Eq. 5)
    def photon_map_build(self, grid_res: int = 64):
        """Photon map from the last trace's records (sorted by HG bin and grid cell)."""
        self._ok(self.lib.pfn_photon_map_build(self.h, grid_res))

    def photon_map_set(self, x, w, power, bins, g_bins, grid_res: int = 64):
        """Photon map from caller records (device tensors [n, 3] float32 and [n] int32)."""
        import torch
        n = int(x.shape[0])
        for t, name in ((x, "x"), (w, "w"), (power, "power")):
            _check(t, torch.float32, 3 * n, name)
        _check(bins, torch.int32, n, "bins")
        g = (C.c_float * len(g_bins))(*[float(v) for v in g_bins])
        self._ok(self.lib.pfn_photon_map_set(self.h, _ptr(x), _ptr(w), _ptr(power), _ptr(bins), n,
                                             len(g_bins), g, grid_res))

    def photon_map_get(self, n_keys: int, capacity: int):
        import torch
        dev = f"cuda:{self.device}"
        start = torch.empty(n_keys, dtype=torch.int32, device=dev)
        pos = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        dirs = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        score = torch.empty((capacity, 3), dtype=torch.float32, device=dev)
        n = C.c_uint64()
        self._ok(self.lib.pfn_photon_map_get(self.h, _ptr(start), n_keys, _ptr(pos), _ptr(dirs),
                                             _ptr(score), capacity, C.byref(n)))
        k = min(n.value, capacity)
        return dict(start=start, pos=pos[:k], dir=dirs[:k], score=score[:k], n=n.value)

    def photon_map_estimate(self, xyz, dirs, bins, radius: float, k: int = 0):
        """Eq. (5) at the queries: returns (rgb [n, 3], r [n], count [n])."""
        import torch
        n = int(xyz.shape[0])
        _check(xyz, torch.float32, 3 * n, "xyz")
        _check(dirs, torch.float32, 3 * n, "dirs")
        _check(bins, torch.int32, n, "bins")
        dev = f"cuda:{self.device}"
        rgb = torch.empty((n, 3), dtype=torch.float32, device=dev)
        r = torch.empty(n, dtype=torch.float32, device=dev)
        cnt = torch.empty(n, dtype=torch.int32, device=dev)
        self._ok(self.lib.pfn_photon_map_estimate(self.h, _ptr(xyz), _ptr(dirs), _ptr(bins), n,
                                                  float(radius), int(k), _ptr(rgb), _ptr(r),
                                                  _ptr(cnt)))
        return rgb, r, cnt

    def cache_info(self):
        nb, res, kappa = C.c_int(), C.c_int(), C.c_double()
        self._ok(self.lib.pfn_cache_info(self.h, C.byref(nb), C.byref(res), C.byref(kappa)))
        return nb.value, res.value, kappa.value

    def get_cache(self):
        import torch
        nb, res, kappa = self.cache_info()
        out = torch.empty((nb, res, res, res, 3), dtype=torch.float32, device=f"cuda:{self.device}")
        self._ok(self.lib.pfn_get_cache(self.h, _ptr(out), out.numel()))
        return out

    def set_cache(self, cache, g_bins: Sequence[float], kappa: float):
        import torch
        _check(cache, torch.float32, name="cache")
        nb, res = cache.shape[0], cache.shape[1]
        g = (C.c_float * len(g_bins))(*g_bins)
        self._ok(self.lib.pfn_set_cache(self.h, _ptr(cache), nb, g, res, float(kappa)))

    # ------------------------------------------------------------------ field
    def field_select(self, slot: int):
        self._ok(self.lib.pfn_field_select(self.h, slot))

    def field_init(self, cfg: FieldConfig = FieldConfig(), seed: int = 0):
        d = cfg.struct()
        self._ok(self.lib.pfn_field_init(self.h, C.byref(d), seed))

    def field_num_params(self) -> int:
        n = C.c_size_t()
        self._ok(self.lib.pfn_field_num_params(self.h, C.byref(n)))
        return n.value

    def field_get_params(self):
        import torch
        n = self.field_num_params()
        out = torch.empty(n, dtype=torch.float32, device=f"cuda:{self.device}")
        self._ok(self.lib.pfn_field_get_params(self.h, _ptr(out), n))
        return out

    def field_set_params(self, p):
        import torch
        _check(p, torch.float32, name="params")
        self._ok(self.lib.pfn_field_set_params(self.h, _ptr(p), p.numel()))

    def field_set_kappa(self, kappa: float):
        self._ok(self.lib.pfn_field_set_kappa(self.h, float(kappa)))

    def field_query(self, xyz, dirs, g, precision: str = "f16", decode: bool = True):
        import torch
        n = xyz.shape[0]
        for t, nm in ((xyz, "xyz"), (dirs, "dirs")):
            _check(t, torch.float32, 3 * n, nm)
        _check(g, torch.float32, n, "g")
        lp = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
        rgb = torch.empty((n, 3), dtype=torch.float32, device=xyz.device) if decode else None
        self._ok(self.lib.pfn_field_query(self.h, DTYPES[precision], _ptr(xyz), _ptr(dirs),
                                          _ptr(g), n, _ptr(lp), _ptr(rgb)))
        return (lp, rgb) if decode else lp

    def field_forward_backward(self, xyz, dirs, g, target, precision: str = "f32",
                               loss: str = "l2"):
        """Loss ("l2" or "rel": relative L2) over n x 3 outputs and its parameter gradient."""
        import torch
        n = xyz.shape[0]
        grad = torch.empty(self.field_num_params(), dtype=torch.float32, device=xyz.device)
        val = C.c_double()
        self._ok(self.lib.pfn_field_forward_backward(self.h, DTYPES[precision], _ptr(xyz),
                                                     _ptr(dirs), _ptr(g), _ptr(target), n,
                                                     LOSSES[loss], C.byref(val), _ptr(grad)))
        return val.value, grad

    def train_field(self, cfg: TrainConfig = TrainConfig(), history: bool = True):
        hist = np.zeros(cfg.steps, dtype=np.float32) if history else None
        p = cfg.struct()
        ptr = hist.ctypes.data_as(C.POINTER(C.c_float)) if history else None
        self._ok(self.lib.pfn_train_field(self.h, C.byref(p), ptr))
        return hist

    def train_batch(self, seed: int, step: int, n: int, g_sampling: str = "pool"):
        import torch
        dev = f"cuda:{self.device}"
        xyz = torch.empty((n, 3), dtype=torch.float32, device=dev)
        dirs = torch.empty((n, 3), dtype=torch.float32, device=dev)
        g = torch.empty(n, dtype=torch.float32, device=dev)
        b = torch.empty(n, dtype=torch.int32, device=dev)
        tgt = torch.empty((n, 3), dtype=torch.float32, device=dev)
        self._ok(self.lib.pfn_train_batch(self.h, seed, step, n, G_SAMPLING[g_sampling], _ptr(xyz),
                                          _ptr(dirs), _ptr(g), _ptr(b), _ptr(tgt)))
        return xyz, dirs, g, b, tgt

    def field_adam_step(self, grad, t: int, lr: float, beta1=0.9, beta2=0.99, eps=1e-15):
        self._ok(self.lib.pfn_field_adam_step(self.h, _ptr(grad), t, lr, beta1, beta2, eps))

    # ------------------------------------------------------------------ rendering
    def render_frame(self, cam, cfg: RenderConfig, out=None):
        import torch
        if out is None:
            out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        _check(out, torch.float32, cam.width * cam.height * 3, "out")
        c = camera_struct(cam)
        p = cfg.struct()
        self._ok(self.lib.pfn_render_frame(self.h, C.byref(c), C.byref(p), _ptr(out)))
        return out

    def render_first_interaction(self, cam, cfg: RenderConfig, out=None):
        """Algorithm 2 of the paper: delta-tracked first interactions along the pixel-centre
        ray (cfg.spp per pixel), one batched field (or cache) pass over the compacted
        interactions, next-event estimation with delta-tracking visibility, albedo-weighted
        composition.  Uses spp, g, indirect, field_precision, light_mask, field_slot, seed."""
        import torch
        if out is None:
            out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        _check(out, torch.float32, cam.width * cam.height * 3, "out")
        c = camera_struct(cam)
        p = cfg.struct()
        self._ok(self.lib.pfn_render_first_interaction(self.h, C.byref(c), C.byref(p), _ptr(out)))
        return out

    def _jobs(self, cams, cfgs, outs):
        import torch
        n = len(cams)
        jobs = (_ffi.RenderJob * n)()
        if outs is None:
            outs = [torch.empty((c.height, c.width, 3), dtype=torch.float32,
                                device=f"cuda:{self.device}") for c in cams]
        for i in range(n):
            jobs[i].cam = camera_struct(cams[i])
            jobs[i].params = cfgs[i].struct()
            jobs[i].dev_rgb_out = _ptr(outs[i])
        return jobs, outs

    def render_batch(self, cams: List, cfgs: List[RenderConfig], outs=None):
        jobs, outs = self._jobs(cams, cfgs, outs)
        self._ok(self.lib.pfn_render_batch(self.h, jobs, len(cams)))
        return outs

    def autotune_batch(self, cams: List, cfgs: List[RenderConfig], outs=None, iters: int = 2):
        jobs, outs = self._jobs(cams, cfgs, outs)
        tw, bw, bh, pz, sg_ = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int()
        ms = C.c_double()
        self._ok(self.lib.pfn_autotune_batch(self.h, jobs, len(cams), iters, C.byref(tw),
                                             C.byref(bw), C.byref(bh), C.byref(pz), C.byref(sg_),
                                             C.byref(ms)))
        names = {v: k for k, v in STRATEGIES.items()}
        return dict(tile_w=tw.value, block_w=bw.value, block_h=bh.value, persistent=pz.value,
                    strategy=names.get(sg_.value, sg_.value), ms=ms.value)

    def set_launch_mode(self, persistent_per_cu: int = 0, use_graph: bool = False):
        self._ok(self.lib.pfn_set_launch_mode(self.h, persistent_per_cu, int(use_graph)))

    def set_render_strategy(self, strategy: str = "auto"):
        """"auto", "fused", "wavefront" or "wavefront_serial" (field-lit frames)."""
        self._ok(self.lib.pfn_set_render_strategy(self.h, STRATEGIES[strategy]))

    def render_path_traced(self, cam, spp: int, max_bounces: int = 8, g: float = 0.0,
                           rr_start: int = 0, light_mask: int = 0, seed: int = 0, out=None):
        import torch
        if out is None:
            out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        c = camera_struct(cam)
        self._ok(self.lib.pfn_render_path_traced(self.h, C.byref(c), spp, max_bounces, g,
                                                 rr_start, light_mask, seed, _ptr(out)))
        return out

    def image_error(self, img, ref):
        rm, rel, ps = C.c_double(), C.c_double(), C.c_double()
        self._ok(self.lib.pfn_image_error(self.h, _ptr(img), _ptr(ref), img.numel(),
                                          C.byref(rm), C.byref(rel), C.byref(ps)))
        return rm.value, rel.value, ps.value

    def image_error_noalloc(self, img, ref, out):
        """The same figures into `out` (3 float64 on the device), with no allocation and no
        synchronisation (pfn_image_error_noalloc)."""
        import torch
        _check(out, torch.float64, 3, "out")
        self._ok(self.lib.pfn_image_error_noalloc(self.h, _ptr(img), _ptr(ref), img.numel(),
                                                  _ptr(out)))
        return out

    # ------------------------------------------------------------------ tuning / timing
    def set_tile_config(self, tile_w: int, block_w: int, block_h: int):
        self._ok(self.lib.pfn_set_tile_config(self.h, tile_w, block_w, block_h))

    def timing_enable(self, on: bool = True):
        self._ok(self.lib.pfn_timing_enable(self.h, int(on)))

    def timing_reset(self):
        self._ok(self.lib.pfn_timing_reset(self.h))

    def timing_get(self, kernel: int):
        ms, n = C.c_double(), C.c_int64()
        self._ok(self.lib.pfn_timing_get(self.h, kernel, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def count_enable(self, on: bool = True):
        self._ok(self.lib.pfn_count_enable(self.h, int(on)))

    def count_get(self):
        st, q = C.c_uint64(), C.c_uint64()
        self._ok(self.lib.pfn_count_get(self.h, C.byref(st), C.byref(q)))
        return st.value, q.value
