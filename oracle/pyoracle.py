"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use this module.
It never touches the HIP library and the HIP library never touches it.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int)
i64p = C.POINTER(C.c_int64)
u64p = C.POINTER(C.c_uint64)
u32p = C.POINTER(C.c_uint32)


class Scene(C.Structure):
    _fields_ = [("density", dp), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("tf", dp), ("ext_scale", C.c_double), ("lights", dp), ("n_lights", C.c_int)]


class Cache(C.Structure):
    _fields_ = [("data", dp), ("n_bins", C.c_int), ("g_bins", dp), ("res", C.c_int)]


class FieldDesc(C.Structure):
    _fields_ = [("levels", C.c_int), ("feats", C.c_int), ("base_res", C.c_int),
                ("growth", C.c_double), ("log2_table", C.c_int), ("hidden_layers", C.c_int),
                ("width", C.c_int), ("psi", C.c_double)]


class FieldLayout(C.Structure):
    _fields_ = [("pos_off", C.c_size_t * 33), ("dir_off", C.c_size_t * 33),
                ("pos_res", C.c_int * 32), ("dir_res", C.c_int * 32),
                ("pos_dense", C.c_int * 32), ("dir_dense", C.c_int * 32),
                ("pos_params", C.c_size_t), ("dir_params", C.c_size_t), ("mlp_off", C.c_size_t),
                ("w_off", C.c_size_t * 8), ("w_rows", C.c_int * 8), ("w_cols", C.c_int * 8),
                ("n_mats", C.c_int), ("n_in", C.c_int), ("n_params", C.c_size_t)]


class TraceParams(C.Structure):
    _fields_ = [("n_photons", C.c_uint64), ("n_bins", C.c_int), ("g_bins", C.c_double * 8),
                ("max_collisions", C.c_int), ("rr_start", C.c_int), ("seed", C.c_uint64)]


class TraceStats(C.Structure):
    _fields_ = [("emitted", C.c_double * 3), ("entered", C.c_double * 3),
                ("escaped", C.c_double * 3), ("escaped_uncollided", C.c_double * 3),
                ("absorbed", C.c_double * 3), ("truncated", C.c_double * 3),
                ("rr_killed", C.c_double * 3), ("stored", C.c_double * 3),
                ("collisions", C.c_double), ("null_events", C.c_double),
                ("n_records", C.c_uint64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = np.array(list(v)) if hasattr(v, "__len__") else v
        return d


class CameraS(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("width", C.c_int), ("height", C.c_int)]


class RenderParams(C.Structure):
    _fields_ = [("spp", C.c_int), ("step_voxels", C.c_double), ("max_steps", C.c_int),
                ("t_min", C.c_double), ("field_stride", C.c_int), ("g", C.c_double),
                ("indirect", C.c_int), ("direct", C.c_int), ("light_mask", C.c_int),
                ("lv_step_voxels", C.c_double), ("seed", C.c_uint64)]


class FiParams(C.Structure):
    _fields_ = [("spp", C.c_int), ("g", C.c_double), ("indirect", C.c_int),
                ("light_mask", C.c_int), ("seed", C.c_uint64)]


class Field(C.Structure):
    _fields_ = [("desc", C.POINTER(FieldDesc)), ("params", dp), ("rounding", C.c_int),
                ("kappa", C.c_double)]


IND_NONE, IND_CACHE, IND_FIELD = 0, 1, 2
DIR_SHADOW, DIR_LIGHTVOL = 0, 1


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_u01.restype = C.c_double
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_int, dp]
        L.orc_hg_eval.restype = C.c_double
        L.orc_hg_eval.argtypes = [C.c_double, C.c_double]
        L.orc_hg_sample_mu.restype = C.c_double
        L.orc_hg_sample_mu.argtypes = [C.c_double, C.c_double]
        L.orc_hg_sample_dir.argtypes = [C.c_double, dp, C.c_double, C.c_double, dp]
        L.orc_density.restype = C.c_double
        L.orc_density.argtypes = [C.POINTER(Scene), dp]
        L.orc_transfer.argtypes = [C.POINTER(Scene), C.c_double, dp, dp]
        L.orc_majorant.restype = C.c_double
        L.orc_majorant.argtypes = [C.POINTER(Scene)]
        L.orc_clip_cube.restype = C.c_int
        L.orc_clip_cube.argtypes = [dp, dp, dp, dp]
        L.orc_shadow_transmittance.restype = C.c_double
        L.orc_shadow_transmittance.argtypes = [C.POINTER(Scene), dp, dp, C.c_double]
        L.orc_cache_gather.argtypes = [C.POINTER(Cache), dp, C.c_double, dp]
        L.orc_field_make_layout.restype = C.c_int
        L.orc_field_make_layout.argtypes = [C.POINTER(FieldDesc), C.POINTER(FieldLayout)]
        L.orc_field_num_params.restype = C.c_size_t
        L.orc_field_num_params.argtypes = [C.POINTER(FieldDesc)]
        L.orc_field_forward.argtypes = [C.POINTER(FieldDesc), dp, C.c_int, C.c_int64, dp, dp, dp,
                                        dp]
        L.orc_field_loss_grad.restype = C.c_double
        L.orc_field_loss_grad.argtypes = [C.POINTER(FieldDesc), dp, C.c_int, C.c_int64, dp, dp,
                                          dp, dp, dp]
        L.orc_field_loss_grad_mode.restype = C.c_double
        L.orc_field_loss_grad_mode.argtypes = [C.POINTER(FieldDesc), dp, C.c_int, C.c_int,
                                               C.c_int64, dp, dp, dp, dp, dp]
        L.orc_field_encode.argtypes = [C.POINTER(FieldDesc), dp, C.c_int, dp, dp, C.c_double, dp]
        L.orc_round_half.restype = C.c_double
        L.orc_round_half.argtypes = [C.c_double]
        L.orc_round_bf16.restype = C.c_double
        L.orc_round_bf16.argtypes = [C.c_double]
        L.orc_log_encode.restype = C.c_double
        L.orc_log_encode.argtypes = [C.c_double, C.c_double]
        L.orc_exp_decode.restype = C.c_double
        L.orc_exp_decode.argtypes = [C.c_double, C.c_double]
        L.orc_adam_step.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_int64, C.c_double, C.c_double,
                                    C.c_double, C.c_double]
        L.orc_lr_at.restype = C.c_double
        L.orc_lr_at.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_int64, C.c_int64]
        L.orc_train_batch.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.POINTER(Cache),
                                      C.c_double, C.c_double, dp, dp, dp, ip, dp]
        L.orc_train_batch_mode.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.POINTER(Cache),
                                           C.c_double, C.c_double, C.c_int, dp, dp, dp, ip, dp]
        L.orc_train_batch_range.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int64,
                                            C.POINTER(Cache), C.c_double, C.c_double, C.c_int,
                                            dp, dp, dp, ip, dp]
        L.orc_trace.argtypes = [C.POINTER(Scene), C.POINTER(TraceParams), C.c_uint64, C.c_uint64,
                                C.POINTER(TraceStats), C.c_uint64, dp, dp, dp, ip, u64p, u64p]
        L.orc_splat_cache.restype = C.c_double
        L.orc_splat_cache.argtypes = [C.POINTER(Scene), C.c_int64, dp, dp, ip, C.c_int, C.c_int,
                                      dp]
        L.orc_camera_ray.argtypes = [C.POINTER(CameraS), C.c_double, C.c_double, dp, dp]
        L.orc_render_pixels.argtypes = [C.POINTER(Scene), C.POINTER(CameraS),
                                        C.POINTER(RenderParams), C.POINTER(Cache),
                                        C.POINTER(Field), C.c_int64, i64p, dp]
        L.orc_lightvol_point.restype = C.c_double
        L.orc_lightvol_point.argtypes = [C.POINTER(Scene), C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_int, C.c_double]
        L.orc_lightvol_res.restype = C.c_int
        L.orc_lightvol_res.argtypes = [C.c_int]
        L.orc_pt_pixels.argtypes = [C.POINTER(Scene), C.POINTER(CameraS), C.c_int, C.c_int,
                                    C.c_double, C.c_int, C.c_uint64, C.c_int, C.c_int64, i64p, dp]
        L.orc_fi_samples.argtypes = [C.POINTER(Scene), C.POINTER(CameraS), C.POINTER(FiParams),
                                     C.POINTER(Cache), C.POINTER(Field), C.c_int64, i64p,
                                     C.POINTER(C.c_int), dp, dp, dp, dp]
        L.orc_fi_pixels.argtypes = [C.POINTER(Scene), C.POINTER(CameraS), C.POINTER(FiParams),
                                    C.POINTER(Cache), C.POINTER(Field), C.c_int64, i64p, dp]
        L.orc_pm_scores.argtypes = [C.POINTER(Scene), C.c_int64, dp, dp, dp]
        L.orc_pm_estimate.argtypes = [C.c_int64, dp, dp, dp, ip, dp, C.c_double, C.c_int,
                                      C.c_int64, dp, dp, ip, dp, dp, i64p]
        L.orc_image_error.argtypes = [C.c_int64, dp, dp, dp, dp, dp]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray, t=dp):
    return a.ctypes.data_as(t)


# ------------------------------------------------------------------ RNG / phase
def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, u32p), _ptr(k, u32p), _ptr(o, u32p))
    return o


def u01(x: int) -> float:
    return lib().orc_u01(int(x))


def uniforms(seed: int, item: int, stream: int, n: int) -> np.ndarray:
    o = np.zeros(n)
    lib().orc_uniforms(seed, item, stream, n, _ptr(o))
    return o


def hg_eval(g: float, mu: float) -> float:
    return lib().orc_hg_eval(g, mu)


def hg_sample_mu(g: float, u: float) -> float:
    return lib().orc_hg_sample_mu(g, u)


def hg_sample_dir(g, w, u1, u2) -> np.ndarray:
    w = _d(w)
    o = np.zeros(3)
    lib().orc_hg_sample_dir(g, _ptr(w), u1, u2, _ptr(o))
    return o


def num_threads() -> int:
    return lib().orc_num_threads()


# ------------------------------------------------------------------ scene
class OracleScene:
    """Holds the double-precision copies of the scene arrays and the C struct pointing at them."""

    def __init__(self, density: np.ndarray, tf: np.ndarray, ext_scale: float, lights: np.ndarray):
        d = np.asarray(density)
        assert d.ndim == 3
        self.density = _d(d.astype(np.float64))
        self.tf = _d(tf).reshape(256, 4)
        self.lights = _d(lights).reshape(-1, 6)
        self.s = Scene(_ptr(self.density), d.shape[2], d.shape[1], d.shape[0], _ptr(self.tf),
                       float(ext_scale), _ptr(self.lights), self.lights.shape[0])

    @property
    def ref(self):
        return C.byref(self.s)

    def density_at(self, pts) -> np.ndarray:
        pts = _d(pts).reshape(-1, 3)
        return np.array([lib().orc_density(self.ref, _ptr(p)) for p in pts])

    def transfer(self, rho: float):
        sig = C.c_double()
        alb = np.zeros(3)
        lib().orc_transfer(self.ref, rho, C.byref(sig), _ptr(alb))
        return sig.value, alb

    def majorant(self) -> float:
        return lib().orc_majorant(self.ref)

    def shadow_T(self, x, p, step: float) -> float:
        return lib().orc_shadow_transmittance(self.ref, _ptr(_d(x)), _ptr(_d(p)), step)


def clip_cube(o, d):
    t0, t1 = C.c_double(), C.c_double()
    hit = lib().orc_clip_cube(_ptr(_d(o)), _ptr(_d(d)), C.byref(t0), C.byref(t1))
    return bool(hit), t0.value, t1.value


class OracleCache:
    def __init__(self, data: np.ndarray, g_bins: Sequence[float], res: int):
        self.data = _d(data).reshape(-1)
        self.g_bins = _d(g_bins)
        self.c = Cache(_ptr(self.data), len(self.g_bins), _ptr(self.g_bins), int(res))
        assert self.data.size == len(self.g_bins) * res ** 3 * 3

    @property
    def ref(self):
        return C.byref(self.c)

    def gather(self, x, g: float) -> np.ndarray:
        o = np.zeros(3)
        lib().orc_cache_gather(self.ref, _ptr(_d(x)), g, _ptr(o))
        return o


# ------------------------------------------------------------------ field
def field_desc(levels=16, feats=2, base_res=16, growth=1.5, log2_table=19, hidden_layers=3,
               width=64, psi=5.0) -> FieldDesc:
    return FieldDesc(levels, feats, base_res, growth, log2_table, hidden_layers, width, psi)


def field_layout(desc: FieldDesc) -> FieldLayout:
    L = FieldLayout()
    rc = lib().orc_field_make_layout(C.byref(desc), C.byref(L))
    assert rc == 0
    return L


def field_num_params(desc: FieldDesc) -> int:
    return int(lib().orc_field_num_params(C.byref(desc)))


def field_forward(desc, params, xyz, dirs, g, rounding=0) -> np.ndarray:
    params = _d(params)
    xyz, dirs, g = _d(xyz).reshape(-1, 3), _d(dirs).reshape(-1, 3), _d(g).reshape(-1)
    n = xyz.shape[0]
    out = np.zeros((n, 3))
    lib().orc_field_forward(C.byref(desc), _ptr(params), rounding, n, _ptr(xyz), _ptr(dirs),
                            _ptr(g), _ptr(out))
    return out


def field_loss_grad(desc, params, xyz, dirs, g, target, rounding=0, loss="l2"):
    """Mean of the loss over n x 3 outputs and its gradient; loss "l2" or
    "rel" (relative L2, denominator held constant in the gradient)."""
    params = _d(params)
    xyz, dirs, g = _d(xyz).reshape(-1, 3), _d(dirs).reshape(-1, 3), _d(g).reshape(-1)
    target = _d(target).reshape(-1, 3)
    grad = np.zeros(params.size)
    mode = {"l2": 0, "rel": 1}[loss]
    val = lib().orc_field_loss_grad_mode(C.byref(desc), _ptr(params), rounding, mode,
                                         xyz.shape[0], _ptr(xyz), _ptr(dirs), _ptr(g),
                                         _ptr(target), _ptr(grad))
    return val, grad


def field_encode(desc, params, x, w, g, rounding=0) -> np.ndarray:
    L = field_layout(desc)
    z = np.zeros(L.n_in)
    lib().orc_field_encode(C.byref(desc), _ptr(_d(params)), rounding, _ptr(_d(x)), _ptr(_d(w)),
                           float(g), _ptr(z))
    return z


def round_half(v: float) -> float:
    return lib().orc_round_half(v)


def round_bf16(v: float) -> float:
    return lib().orc_round_bf16(v)


def log_encode(v: float, psi: float) -> float:
    return lib().orc_log_encode(v, psi)


def exp_decode(lp: float, psi: float) -> float:
    return lib().orc_exp_decode(lp, psi)


def adam_step(param, grad, m, v, t, lr, beta1=0.9, beta2=0.99, eps=1e-15):
    """In-place on float64 arrays param, m, v."""
    for a in (param, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _d(grad)
    lib().orc_adam_step(param.size, _ptr(param), _ptr(g), _ptr(m), _ptr(v), t, lr, beta1, beta2,
                        eps)


def lr_at(step, lr0=9e-4, decay=0.92, start_step=1400, interval=25) -> float:
    return lib().orc_lr_at(step, lr0, decay, start_step, interval)


def train_batch(seed, step, n, cache: OracleCache, kappa, psi=5.0, g_sampling="pool", first=0):
    """g_sampling "pool": g from the cache's bins; "uniform": g uniform over [g_0, g_last] with
    targets interpolated linearly in g between the neighbouring bins.  Returns samples
    first .. first + n - 1 of the batch."""
    xyz = np.zeros((n, 3))
    dirs = np.zeros((n, 3))
    g = np.zeros(n)
    b = np.zeros(n, dtype=np.int32)
    tgt = np.zeros((n, 3))
    mode = {"pool": 0, "uniform": 1}[g_sampling]
    lib().orc_train_batch_range(seed, step, first, n, cache.ref, kappa, psi, mode, _ptr(xyz),
                                _ptr(dirs), _ptr(g), _ptr(b, ip), _ptr(tgt))
    return xyz, dirs, g, b, tgt


# ------------------------------------------------------------------ tracing
def trace(scene: OracleScene, n_photons, g_bins, seed, first=0, count=None, max_collisions=8,
          rr_start=3, want_records=True):
    count = n_photons - first if count is None else count
    tp = TraceParams()
    tp.n_photons = n_photons
    tp.n_bins = len(g_bins)
    for i, g in enumerate(g_bins):
        tp.g_bins[i] = g
    tp.max_collisions = max_collisions
    tp.rr_start = rr_start
    tp.seed = seed
    st = TraceStats()
    nrec = C.c_uint64()
    if want_records:
        cap = count * max(1, max_collisions - 1)
        rx = np.zeros((cap, 3))
        rw = np.zeros((cap, 3))
        rp = np.zeros((cap, 3))
        rb = np.zeros(cap, dtype=np.int32)
        rid = np.zeros(cap, dtype=np.uint64)
        lib().orc_trace(scene.ref, C.byref(tp), first, count, C.byref(st), cap, _ptr(rx), _ptr(rw),
                        _ptr(rp), _ptr(rb, ip), _ptr(rid, u64p), C.byref(nrec))
        k = nrec.value
        recs = dict(x=rx[:k], w=rw[:k], power=rp[:k], bin=rb[:k], photon=rid[:k])
    else:
        lib().orc_trace(scene.ref, C.byref(tp), first, count, C.byref(st), 0, None, None, None,
                        None, None, C.byref(nrec))
        recs = None
    return st.as_dict(), recs


def splat_cache(scene: OracleScene, recs, res, n_bins):
    x = _d(recs["x"])
    p = _d(recs["power"])
    b = np.ascontiguousarray(recs["bin"], dtype=np.int32)
    out = np.zeros((n_bins, res, res, res, 3))
    kappa = lib().orc_splat_cache(scene.ref, x.shape[0], _ptr(x), _ptr(p), _ptr(b, ip), res, n_bins,
                                  _ptr(out))
    return out, kappa


# ------------------------------------------------------------------ rendering
def camera_struct(cam) -> CameraS:
    c = CameraS()
    for i in range(3):
        c.eye[i] = cam.eye[i]
        c.target[i] = cam.target[i]
        c.up[i] = cam.up[i]
    c.fov_y_deg = cam.fov_y_deg
    c.width = cam.width
    c.height = cam.height
    return c


def camera_ray(cam, px, py):
    cs = camera_struct(cam)
    o = np.zeros(3)
    d = np.zeros(3)
    lib().orc_camera_ray(C.byref(cs), px, py, _ptr(o), _ptr(d))
    return o, d


def render_params(spp=1, step_voxels=0.5, max_steps=1 << 30, t_min=0.0, field_stride=1, g=0.0,
                  indirect=IND_NONE, direct=DIR_SHADOW, light_mask=0, lv_step_voxels=0.5,
                  seed=0) -> RenderParams:
    return RenderParams(spp, step_voxels, max_steps, t_min, field_stride, g, indirect, direct,
                        light_mask, lv_step_voxels, seed)


def render_pixels(scene: OracleScene, cam, params: RenderParams, pixels=None,
                  cache: Optional[OracleCache] = None, field=None) -> np.ndarray:
    """field = (desc, params_array, rounding, kappa) or None."""
    if pixels is None:
        pixels = np.arange(cam.width * cam.height, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    cs = camera_struct(cam)
    out = np.zeros((pixels.size, 3))
    if params.indirect == IND_CACHE and cache is None:
        raise ValueError("indirect = cache needs a cache")
    if params.indirect == IND_FIELD and field is None:
        raise ValueError("indirect = field needs a field")
    cref = cache.ref if cache is not None else None
    fref = None
    keep = None
    if field is not None:
        desc, fp, rounding, kappa = field
        keep = _d(fp)
        fs = Field(C.pointer(desc), _ptr(keep), rounding, kappa)
        fref = C.byref(fs)
    lib().orc_render_pixels(scene.ref, C.byref(cs), C.byref(params), cref, fref, pixels.size,
                            _ptr(pixels, i64p), _ptr(out))
    del keep
    return out


def lightvol_point(scene: OracleScene, res, l, i, j, k, step) -> float:
    return lib().orc_lightvol_point(scene.ref, res, l, i, j, k, step)


def lightvol_res(n: int) -> int:
    return lib().orc_lightvol_res(n)


def pt_pixels(scene: OracleScene, cam, spp, max_bounces=8, g=0.0, rr_start=0, seed=0,
              light_mask=0, pixels=None) -> np.ndarray:
    if pixels is None:
        pixels = np.arange(cam.width * cam.height, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    cs = camera_struct(cam)
    out = np.zeros((pixels.size, 3))
    lib().orc_pt_pixels(scene.ref, C.byref(cs), spp, max_bounces, g, rr_start, seed, light_mask,
                        pixels.size, _ptr(pixels, i64p), _ptr(out))
    return out


def _fi_refs(params, cache, field):
    if params.indirect == IND_CACHE and cache is None:
        raise ValueError("indirect = cache needs a cache")
    if params.indirect == IND_FIELD and field is None:
        raise ValueError("indirect = field needs a field")
    cref = cache.ref if cache is not None else None
    if field is None:
        return cref, None, None
    desc, fp, rounding, kappa = field
    keep = _d(fp)
    fs = Field(C.pointer(desc), _ptr(keep), rounding, kappa)
    return cref, fs, keep


def fi_params(spp=1, g=0.0, indirect=IND_NONE, light_mask=0, seed=0) -> FiParams:
    return FiParams(spp, g, indirect, light_mask, seed)


def fi_samples(scene: OracleScene, cam, params: FiParams, pixels=None,
               cache: Optional[OracleCache] = None, field=None):
    """First-interaction renderer, per sample: dict of valid [n, spp], x, albedo, Ld, Li
    [n, spp, 3].  field = (desc, params_array, rounding, kappa) or None."""
    if pixels is None:
        pixels = np.arange(cam.width * cam.height, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    n, S = pixels.size, params.spp
    cs = camera_struct(cam)
    valid = np.zeros((n, S), dtype=np.int32)
    out = {k: np.zeros((n, S, 3)) for k in ("x", "albedo", "Ld", "Li")}
    cref, fs, keep = _fi_refs(params, cache, field)
    lib().orc_fi_samples(scene.ref, C.byref(cs), C.byref(params), cref,
                         C.byref(fs) if fs is not None else None, n, _ptr(pixels, i64p),
                         valid.ctypes.data_as(C.POINTER(C.c_int)), _ptr(out["x"]),
                         _ptr(out["albedo"]), _ptr(out["Ld"]), _ptr(out["Li"]))
    del keep
    out["valid"] = valid
    return out


def fi_pixels(scene: OracleScene, cam, params: FiParams, pixels=None,
              cache: Optional[OracleCache] = None, field=None) -> np.ndarray:
    if pixels is None:
        pixels = np.arange(cam.width * cam.height, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    cs = camera_struct(cam)
    out = np.zeros((pixels.size, 3))
    cref, fs, keep = _fi_refs(params, cache, field)
    lib().orc_fi_pixels(scene.ref, C.byref(cs), C.byref(params), cref,
                        C.byref(fs) if fs is not None else None, pixels.size,
                        _ptr(pixels, i64p), _ptr(out))
    del keep
    return out


def pm_scores(scene: OracleScene, x, power) -> np.ndarray:
    """Collision-estimator scores Phi / sigma_t(x) of photon records."""
    x, power = _d(x).reshape(-1, 3), _d(power).reshape(-1, 3)
    out = np.zeros_like(power)
    lib().orc_pm_scores(scene.ref, x.shape[0], _ptr(x), _ptr(power), _ptr(out))
    return out


def pm_estimate(rec_x, rec_w, rec_s, rec_bin, g_bins, radius, k, qx, qw, qbin):
    """Eq. (5) estimates at the queries; returns (L [n, 3], r_used [n], n_used [n])."""
    rx, rw, rs = (_d(a).reshape(-1, 3) for a in (rec_x, rec_w, rec_s))
    rb = np.ascontiguousarray(rec_bin, dtype=np.int32)
    qx, qw = _d(qx).reshape(-1, 3), _d(qw).reshape(-1, 3)
    qb = np.ascontiguousarray(qbin, dtype=np.int32)
    gb = _d(g_bins)
    n = qx.shape[0]
    out, r_used, n_used = np.zeros((n, 3)), np.zeros(n), np.zeros(n, dtype=np.int64)
    lib().orc_pm_estimate(rx.shape[0], _ptr(rx), _ptr(rw), _ptr(rs), _ptr(rb, ip), _ptr(gb),
                          float(radius), int(k), n, _ptr(qx), _ptr(qw), _ptr(qb, ip), _ptr(out),
                          _ptr(r_used), _ptr(n_used, i64p))
    return out, r_used, n_used


def image_error(img, ref):
    img, ref = _d(img).reshape(-1), _d(ref).reshape(-1)
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_image_error(img.size, _ptr(img), _ptr(ref), C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value
