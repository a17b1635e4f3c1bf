"""Pins of the oracle's transport: photon tracer tallies, cache normalisation, the ray marcher,
the path tracer, and the split L = L_d + L_i between them (brute force on tiny volumes)."""
import math

import numpy as np
import pytest
from scipy.integrate import dblquad, quad

from paper_2304_07338_amd.scenegen import Camera


def gray_tf(albedo, opacity):
    tf = np.zeros((256, 4))
    tf[:, :3] = albedo
    tf[:, 3] = opacity
    return tf


def cone_share(p):
    """Share of the full sphere of directions in the emission cone toward the cube."""
    d = np.linalg.norm(np.asarray(p) - 0.5)
    R = math.sqrt(3) / 2
    return 1.0 if d <= R else 0.5 * (1 - math.sqrt(1 - (R / d) ** 2))


def homog_scene(orc, rho, albedo=0.7, opacity=None, ext=20.0, lights=None, n=8):
    tf = gray_tf(albedo, 1.0 if opacity is None else opacity)
    if opacity is None:
        tf[:, 3] = np.arange(256) / 255.0
    if lights is None:
        lights = np.array([[2.0, 0.5, 0.5, 1.0, 1.0, 1.0]])
    return orc.OracleScene(np.full((n, n, n), rho), tf, ext, lights)


# ------------------------------------------------------------------ photon tracer
@pytest.mark.parametrize("albedo", [1.0, 0.8])
def test_tracer_energy_conservation_exact_without_roulette(orc, albedo):
    lights = np.array([[2.0, 0.5, 0.5, 1.0, 0.5, 2.0], [0.5, -1.0, 0.4, 0.3, 0.3, 0.3]])
    rng = np.random.default_rng(0)
    vol = rng.uniform(0, 1, (8, 8, 8))
    tf = gray_tf(albedo, 0.5)
    tf[:, 3] = np.linspace(0, 1, 256)
    s = orc.OracleScene(vol, tf, 10.0, lights)
    st, _ = orc.trace(s, 6000, [-0.5, 0.0, 0.6], seed=5, rr_start=0, max_collisions=64,
                      want_records=False)
    # every HG bin is a complete photon map of the scene: per bin, each light emits exactly
    # 4 pi I into its emission cone's share of directions, split over the pair's photons
    emitted_expected = 3 * 4 * math.pi * sum(cone_share(L[:3]) * L[3:] for L in lights)
    np.testing.assert_allclose(st["emitted"], emitted_expected, rtol=1e-12)
    balance = st["escaped"] + st["absorbed"] + st["truncated"] + st["rr_killed"]
    np.testing.assert_allclose(balance, st["emitted"], rtol=1e-12)  # misses count as escaped
    assert np.all(st["rr_killed"] == 0)
    if albedo == 1.0:
        assert np.all(st["absorbed"] == 0)


def test_tracer_albedo_weighting_closed_form(orc):
    """Light at the centre of a very dense homogeneous cube (no escape): after c_max collisions
    the absorbed fraction is 1 - a^c_max and the truncated fraction a^c_max, per channel."""
    a = np.array([0.5, 0.8, 0.95])
    tf = np.zeros((256, 4))
    tf[:, :3] = a
    tf[:, 3] = 1.0
    s = orc.OracleScene(np.full((4, 4, 4), 0.5), tf, 4000.0,
                        np.array([[0.5, 0.5, 0.5, 1.0, 1.0, 1.0]]))
    st, recs = orc.trace(s, 2000, [0.3], seed=1, rr_start=0, max_collisions=8)
    assert np.all(st["escaped"] == 0)
    np.testing.assert_allclose(st["absorbed"] / st["entered"], 1 - a ** 8, rtol=1e-12)
    np.testing.assert_allclose(st["truncated"] / st["entered"], a ** 8, rtol=1e-12)
    # every photon stores collisions 2..8 with the power it arrives with
    assert recs["x"].shape[0] == 2000 * 7
    first = recs["power"][recs["photon"] == 0]
    phi0 = 4 * math.pi / 2000
    np.testing.assert_allclose(first, phi0 * a[None, :] ** np.arange(1, 8)[:, None], rtol=1e-12)
    np.testing.assert_allclose(st["stored"], phi0 * 2000 * (a ** np.arange(1, 8)[:, None]).sum(0),
                               rtol=1e-12)


def test_tracer_roulette_is_unbiased(orc):
    a = np.array([0.5, 0.8, 0.95])
    tf = np.zeros((256, 4))
    tf[:, :3] = a
    tf[:, 3] = 1.0
    s = orc.OracleScene(np.full((4, 4, 4), 0.5), tf, 4000.0,
                        np.array([[0.5, 0.5, 0.5, 1.0, 1.0, 1.0]]))
    n = 40000
    st, _ = orc.trace(s, n, [0.0], seed=2, rr_start=3, max_collisions=8, want_records=False)
    expected = (1 - a ** 8)
    frac = st["absorbed"] / st["entered"]
    # per-photon absorbed power is bounded by 1 in units of phi0 -> generous z bound
    assert np.all(np.abs(frac - expected) < 5 * 0.5 / math.sqrt(n))
    assert np.all(st["rr_killed"] > 0)


def test_tracer_uncollided_escape_matches_quadrature(orc):
    """Light at the centre of a homogeneous cube: P(escape uncollided) =
    E_w[exp(-sigma * 0.5 / max|w_i|)] for isotropic w."""
    sig = 3.0
    tf = gray_tf(0.5, 1.0)
    s = orc.OracleScene(np.full((4, 4, 4), 0.5), tf, sig, np.array([[0.5, 0.5, 0.5, 1, 1, 1]]))
    n = 100000
    st, _ = orc.trace(s, n, [0.0], seed=3, rr_start=0, max_collisions=1, want_records=False)
    frac = st["escaped_uncollided"][0] / st["entered"][0]

    def integrand(phi, mu):
        st_ = math.sqrt(1 - mu * mu)
        w = (st_ * math.cos(phi), st_ * math.sin(phi), mu)
        return math.exp(-sig * 0.5 / max(abs(c) for c in w)) / (4 * math.pi)

    ref = dblquad(integrand, -1, 1, 0, 2 * math.pi, epsabs=1e-10)[0]
    sd = math.sqrt(ref * (1 - ref) / n)
    assert abs(frac - ref) < 5 * sd


def test_tracer_stratification_over_lights_and_bins(orc):
    lights = np.array([[2.0, 0.5, 0.5, 1, 1, 1], [0.5, 2.0, 0.5, 1, 1, 1], [0.5, 0.5, 2.0, 1, 1, 1]])
    s = homog_scene(orc, 0.5, albedo=0.9, lights=lights)
    bins = [-0.8, -0.4, 0.0, 0.4, 0.8]
    st, recs = orc.trace(s, 3000 + 7, bins, seed=4)
    np.testing.assert_allclose(st["emitted"], 5 * 4 * math.pi * sum(cone_share(L[:3]) for L in lights),
                               rtol=1e-12)
    ids = recs["photon"]
    np.testing.assert_array_equal(recs["bin"], (ids // 3) % 5)


def test_tracer_entered_power_is_the_solid_angle_of_the_cube(orc):
    """A light on the z axis at height 2 sees the cube's top face (side 1, distance 1) as its
    silhouette: the power entering the cube is I * Omega with
    Omega = 4 arcsin(a b / sqrt((a^2 + 4 d^2)(b^2 + 4 d^2))) = 4 arcsin(1/5) (solid angle of a
    centred rectangle).  Independent of how the emitter samples directions."""
    s = homog_scene(orc, 0.5, albedo=0.9, lights=np.array([[0.5, 0.5, 2.0, 1.0, 2.0, 0.5]]))
    n = 200000
    st, _ = orc.trace(s, n, [0.0], seed=8, want_records=False)
    omega = 4 * math.asin(1 / 5)
    expect = omega * np.array([1.0, 2.0, 0.5])
    frac_hit = st["entered"][0] / st["emitted"][0]
    sd = math.sqrt(frac_hit * (1 - frac_hit) / n) * st["emitted"][0]
    assert np.all(np.abs(st["entered"] - expect) < 5 * sd * np.array([1.0, 2.0, 0.5]))
    assert frac_hit > 0.3  # the cone keeps most photons on the volume


def test_cache_mass_conservation(orc):
    s = homog_scene(orc, 0.5, albedo=0.8)
    st, recs = orc.trace(s, 20000, [-0.4, 0.4], seed=6)
    res = 8
    cache, kappa = orc.splat_cache(s, recs, res, 2)
    sig, _ = s.transfer(0.5)
    vcell = 1.0 / res ** 3
    for b in range(2):
        m = recs["bin"] == b
        np.testing.assert_allclose(cache[b].sum(axis=(0, 1, 2)) * 4 * math.pi * vcell,
                                   recs["power"][m].sum(axis=0) / sig, rtol=1e-12)
    assert kappa == cache.max()


# ------------------------------------------------------------------ ray marcher
def axis_camera(w=1, h=1, fov=10.0):
    return Camera((0.5, 0.5, -1.7), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), fov, w, h)


@pytest.mark.parametrize("step_voxels", [0.5, 0.37, 2.0])
def test_marcher_homogeneous_constant_source_closed_form(orc, step_voxels):
    """Constant in-scattered radiance S and no direct light: C = a S (1 - exp(-sigma L))."""
    rho, a, S = 0.6, 0.7, 0.25
    s = homog_scene(orc, rho, albedo=a, lights=np.array([[2.0, 0.5, 0.5, 0.0, 0.0, 0.0]]))
    sig, _ = s.transfer(rho)
    cache = orc.OracleCache(np.full((1, 4, 4, 4, 3), S), [0.0], 4)
    p = orc.render_params(step_voxels=step_voxels, indirect=orc.IND_CACHE)
    out = orc.render_pixels(s, axis_camera(), p, cache=cache)
    np.testing.assert_allclose(out[0], a * S * (1 - math.exp(-sig * 1.0)), rtol=1e-12)
    # the field stride only changes when the held value is refreshed
    p.field_stride = 3
    out = orc.render_pixels(s, axis_camera(), p, cache=cache)
    np.testing.assert_allclose(out[0], a * S * (1 - math.exp(-sig * 1.0)), rtol=1e-12)


def test_marcher_early_termination(orc):
    rho, a, S = 1.0, 0.7, 0.25
    s = homog_scene(orc, rho, albedo=a, lights=np.array([[2.0, 0.5, 0.5, 0.0, 0.0, 0.0]]))
    sig, _ = s.transfer(rho)
    cache = orc.OracleCache(np.full((1, 4, 4, 4, 3), S), [0.0], 4)
    step = 0.5 / 8
    p = orc.render_params(step_voxels=0.5, indirect=orc.IND_CACHE, t_min=1e-3)
    out = orc.render_pixels(s, axis_camera(), p, cache=cache)
    # stops after the first step whose end transmittance falls below t_min
    k = math.ceil(-math.log(1e-3) / (sig * step))
    assert k * step < 1.0
    np.testing.assert_allclose(out[0], a * S * (1 - math.exp(-sig * k * step)), rtol=1e-12)


def test_marcher_direct_light_converges_to_quadrature(orc):
    rho, a, g = 0.3, 0.8, 0.4
    I = np.array([1.0, 0.5, 0.25])
    s = homog_scene(orc, rho, albedo=a, lights=np.array([[2.0, 0.5, 0.5, *I]]))
    sig, _ = s.transfer(rho)

    def integrand(z):
        r = math.sqrt(1.5 ** 2 + (z - 0.5) ** 2)
        mu = (0.5 - z) / r
        return (math.exp(-sig * z) * sig * a * orc.hg_eval(g, mu) * math.exp(-sig * r / 3)
                / (r * r))

    ref = quad(integrand, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)[0] * I
    errs = []
    for sv in [0.5, 0.25, 0.125, 0.0625]:
        p = orc.render_params(step_voxels=sv, g=g)
        out = orc.render_pixels(s, axis_camera(), p)
        errs.append(np.max(np.abs(out[0] / ref - 1)))
    assert errs[-1] < 1e-5
    for e0, e1 in zip(errs[:-1], errs[1:]):
        assert e1 < e0 / 3.0  # second-order midpoint convergence


def test_light_volume_converges_to_exact_shadows(orc):
    """The half-resolution light-transmittance grid approximates the exact shadow march; its
    image error shrinks as the volume (and with it the grid) is refined.  The size of the error
    is a property of the approximation, reported here, not an exact pin."""
    errs = []
    for n in (16, 32):
        zz, yy, xx = np.meshgrid(*[(np.arange(n) + 0.5) / n] * 3, indexing="ij")
        vol = np.clip(0.8 * np.exp(-((xx - 0.5) ** 2 + (yy - 0.5) ** 2 + (zz - 0.5) ** 2) / 0.03),
                      0, 1)
        tf = gray_tf(0.8, 1.0)
        tf[:, 3] = np.arange(256) / 255.0
        s = orc.OracleScene(vol, tf, 20.0,
                            np.array([[2.0, 0.3, 0.6, 1, 1, 1], [0.4, 0.5, 1.8, 0.5, 0.5, 0.5]]))
        cam = Camera((0.5, -1.7, 0.5), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 40.0, 8, 8)
        p = orc.render_params(step_voxels=0.5, g=0.2)
        exact = orc.render_pixels(s, cam, p)
        p.direct = orc.DIR_LIGHTVOL
        lv = orc.render_pixels(s, cam, p)
        errs.append(orc.image_error(lv, exact)[1])
    assert errs[1] < errs[0] / 3
    assert errs[1] < 4e-2
    s = homog_scene(orc, 0.4, albedo=0.8, n=16,
                    lights=np.array([[2.0, 0.3, 0.6, 1, 1, 1], [0.4, 0.5, 1.8, 0.5, 0.5, 0.5]]))
    # grid values are exact shadow transmittances at the grid points
    res = orc.lightvol_res(16)
    assert res == 8
    x = np.array([(2 + 0.5) / 8, (5 + 0.5) / 8, (1 + 0.5) / 8])
    assert orc.lightvol_point(s, res, 1, 2, 5, 1, 0.5 / 16) == pytest.approx(
        s.shadow_T(x, [0.4, 0.5, 1.8], 0.5 / 16), rel=1e-14)


# ------------------------------------------------------------------ path tracer and the split
def small_het_scene(orc, lights, albedo=0.75):
    rng = np.random.default_rng(12)
    zz, yy, xx = np.meshgrid(*[(np.arange(8) + 0.5) / 8] * 3, indexing="ij")
    vol = np.clip(0.6 * np.exp(-((xx - 0.5) ** 2 + (yy - 0.45) ** 2 + (zz - 0.55) ** 2) / 0.08)
                  + 0.05 * rng.uniform(size=xx.shape), 0, 1)
    tf = gray_tf(albedo, 1.0)
    tf[:, 0] = albedo * 0.9
    tf[:, 3] = np.linspace(0.0, 1.0, 256)
    return orc.OracleScene(vol, tf, 6.0, lights)


def _pt_batches(orc, s, cam, spp, nb, **kw):
    outs = np.stack([orc.pt_pixels(s, cam, spp, seed=100 + i, **kw) for i in range(nb)])
    return outs.mean(0), outs.std(0, ddof=1) / math.sqrt(nb)


def test_path_tracer_single_bounce_matches_direct_marcher(orc):
    lights = np.array([[0.5, 0.5, 2.0, 1.0, 1.0, 1.0]])
    s = small_het_scene(orc, lights)
    cam = Camera((0.5, -1.7, 0.5), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 30.0, 4, 4)
    g = 0.3
    p = orc.render_params(step_voxels=0.125, g=g)
    ref = orc.render_pixels(s, cam, p)
    # PT uses jittered sub-pixel positions: compare the image mean and per-pixel with jitter
    # averaged out by supersampling the marcher at the same sub-pixel distribution
    mean, se = _pt_batches(orc, s, cam, 2048, 8, max_bounces=1, g=g)
    sup = []
    for jx in (0.125, 0.375, 0.625, 0.875):
        for jy in (0.125, 0.375, 0.625, 0.875):
            cam2 = Camera(cam.eye, cam.target, cam.up, cam.fov_y_deg, cam.width * 4,
                          cam.height * 4)
            pix = [(4 * iy + int(jy * 4)) * cam2.width + 4 * ix + int(jx * 4)
                   for iy in range(4) for ix in range(4)]
            sup.append(orc.render_pixels(s, cam2, p, pixels=np.array(pix)))
    sup = np.mean(sup, axis=0)
    z = (mean - sup) / np.maximum(se, 1e-12)
    assert np.all(np.abs(z) < 6), z
    assert abs(mean.mean() / sup.mean() - 1) < 0.02


def test_marcher_with_photon_cache_matches_path_tracer(orc):
    """L = L_d + L_i: the marcher with exact shadows plus the g=0 photon cache agrees with a
    multiple-scattering path tracer of the same collision budget (image mean within 4%)."""
    lights = np.array([[0.5, 0.5, 2.0, 1.0, 1.0, 1.0]])
    s = small_het_scene(orc, lights, albedo=0.8)
    st, recs = orc.trace(s, 1 << 20, [0.0], seed=21, rr_start=0, max_collisions=8)
    res = 8
    cache_arr, kappa = orc.splat_cache(s, recs, res, 1)
    cache = orc.OracleCache(cache_arr, [0.0], res)
    cam = Camera((0.5, -1.7, 0.5), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 30.0, 8, 8)
    p = orc.render_params(step_voxels=0.25, g=0.0, indirect=orc.IND_CACHE)
    m_full = orc.render_pixels(s, cam, p, cache=cache)
    p.indirect = orc.IND_NONE
    m_direct = orc.render_pixels(s, cam, p)
    pt, se = _pt_batches(orc, s, cam, 512, 8, max_bounces=8, g=0.0)
    pt1, _ = _pt_batches(orc, s, cam, 512, 8, max_bounces=1, g=0.0)
    ind_m = (m_full - m_direct).mean()
    ind_pt = (pt - pt1).mean()
    assert ind_m > 0.1 * m_full.mean()  # indirect light is a sizeable part of the image
    assert abs(m_full.mean() / pt.mean() - 1) < 0.04
    assert abs(ind_m / ind_pt - 1) < 0.08
