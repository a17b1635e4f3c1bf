"""Pins of the oracle's first-interaction renderer (Section 3.6, Algorithm 2): its estimator is
unbiased for the same integral the ray marcher approximates, so it is checked in distribution
against closed forms and quadrature on homogeneous media, against the (separately pinned) ray
marcher at a fine step on a heterogeneous volume, and on its degenerate cases."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2304_07338_amd.scenegen import Camera
from test_oracle_transport import axis_camera, gray_tf, homog_scene, small_het_scene


def _contrib(smp):
    """Per-sample contributions a (L_d + L_i) of valid samples (zero otherwise)."""
    return smp["albedo"] * (smp["Ld"] + smp["Li"]) * smp["valid"][..., None]


def _z(samples_c, ref):
    n = samples_c.shape[0]
    mean = samples_c.mean(0)
    se = samples_c.std(0, ddof=1) / math.sqrt(n)
    return (mean - ref) / se, mean, se


def test_direct_light_matches_quadrature_in_a_homogeneous_cube(orc):
    """Light at (2, .5, .5), view ray along +z through the cube's axis: the first collision has
    density sigma exp(-sigma z) on [0, 1], the visibility walk succeeds with probability
    exp(-sigma r / 3) (a third of the way to the light lies inside the cube), so the pixel's
    expectation is the integral of sigma e^(-sigma z) a p_g(mu) e^(-sigma r/3) / r^2 times I."""
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
    smp = orc.fi_samples(s, axis_camera(), orc.fi_params(spp=1000000, g=g, seed=3))
    c = _contrib(smp)[0]
    z, mean, se = _z(c, ref)
    assert np.all(np.abs(z) < 5), (z, mean, ref)
    assert np.all(se < 0.01 * ref)
    # collision points lie on the view ray inside the cube
    x = smp["x"][0][smp["valid"][0] == 1]
    np.testing.assert_allclose(x[:, :2], 0.5, atol=1e-12)
    assert x[:, 2].min() >= 0.0 and x[:, 2].max() <= 1.0
    # and their depths follow sigma e^(-sigma z) truncated to [0, 1]: mean depth
    mz = (1 / sig - math.exp(-sig) * (1 + 1 / sig)) / (1 - math.exp(-sig))
    assert abs(x[:, 2].mean() - mz) < 5 * x[:, 2].std() / math.sqrt(len(x))


def test_constant_indirect_source_closed_form(orc):
    """No lights, a constant photon cache S: every collision contributes a S exactly and a walk
    collides with probability 1 - exp(-sigma), so E = a S (1 - exp(-sigma))."""
    rho, a, S = 0.25, 0.6, np.array([0.3, 0.2, 0.1])
    s = homog_scene(orc, rho, albedo=a, lights=np.array([[2.0, 0.5, 0.5, 0.0, 0.0, 0.0]]))
    sig, _ = s.transfer(rho)
    res = 4
    cache = orc.OracleCache(np.tile(S, (1, res ** 3, 1)), [0.0], res)
    smp = orc.fi_samples(s, axis_camera(), orc.fi_params(spp=100000, indirect=orc.IND_CACHE,
                                                         seed=5), cache=cache)
    v = smp["valid"][0] == 1
    np.testing.assert_allclose(smp["Li"][0][v], np.tile(S, (v.sum(), 1)), rtol=1e-13)
    assert np.all(smp["Li"][0][~v] == 0.0)
    p = 1 - math.exp(-sig)
    n = v.size
    assert abs(v.mean() - p) < 5 * math.sqrt(p * (1 - p) / n)
    out = orc.fi_pixels(s, axis_camera(), orc.fi_params(spp=100000, indirect=orc.IND_CACHE,
                                                        seed=5), cache=cache)
    np.testing.assert_allclose(out[0], a * S * v.mean(), rtol=1e-10)  # summation order


def test_agrees_with_the_fine_step_ray_marcher_on_a_heterogeneous_volume(orc):
    """Both estimate the integral of T sigma_t a (L_d + L_i) along the ray: the marcher with
    exact shadow transmittance at a fine step, the first-interaction renderer in expectation."""
    lights = np.array([[0.5, 0.5, 2.0, 1.0, 1.0, 1.0], [2.0, 0.3, 0.4, 0.4, 0.6, 0.8]])
    s = small_het_scene(orc, lights)
    res = 4
    rng = np.random.default_rng(3)
    cache = orc.OracleCache(rng.uniform(0.05, 0.2, (2, res ** 3, 3)), [-0.5, 0.5], res)
    cam = Camera((0.5, -1.7, 0.5), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 30.0, 6, 6)
    pix = np.array([7, 14, 21, 28])
    g = 0.3
    p = orc.render_params(step_voxels=0.0625, g=g, indirect=orc.IND_CACHE)
    ref = orc.render_pixels(s, cam, p, pixels=pix, cache=cache)
    smp = orc.fi_samples(s, cam, orc.fi_params(spp=60000, g=g, indirect=orc.IND_CACHE, seed=7),
                         pixels=pix, cache=cache)
    c = _contrib(smp)
    for i in range(len(pix)):
        z, mean, se = _z(c[i], ref[i])
        assert np.all(np.abs(z) < 5), (i, z, mean, ref[i])
        assert np.all(se < 0.02 * ref[i])


def test_light_mask_selects_lights(orc):
    lights = np.array([[0.5, 0.5, 2.0, 1.0, 1.0, 1.0], [2.0, 0.3, 0.4, 0.4, 0.6, 0.8]])
    s = small_het_scene(orc, lights)
    cam = Camera((0.5, -1.7, 0.5), (0.5, 0.5, 0.5), (0.0, 0.0, 1.0), 30.0, 3, 3)
    both = orc.fi_samples(s, cam, orc.fi_params(spp=40, g=0.2, seed=9))
    one = orc.fi_samples(s, cam, orc.fi_params(spp=40, g=0.2, seed=9, light_mask=1))
    two = orc.fi_samples(s, cam, orc.fi_params(spp=40, g=0.2, seed=9, light_mask=2))
    # the walks do not depend on the lights; the visibility walks of light 2 follow light 1's
    # in the same stream, so only light 1's term is unchanged when light 2 is dropped
    np.testing.assert_array_equal(both["valid"], one["valid"])
    np.testing.assert_array_equal(both["x"], two["x"])
    assert np.all(both["Ld"] >= one["Ld"] - 1e-15)
    assert (one["Ld"] > 0).any() and (two["Ld"] > 0).any()


@pytest.mark.parametrize("case", ["transparent", "miss"])
def test_degenerate_cases_are_black(orc, case):
    if case == "transparent":
        s = orc.OracleScene(np.full((4, 4, 4), 0.5), gray_tf(0.8, 0.0), 20.0,
                            np.array([[2.0, 0.5, 0.5, 1.0, 1.0, 1.0]]))
        cam = axis_camera(3, 3, fov=40.0)
    else:
        s = homog_scene(orc, 0.5)
        cam = Camera((0.5, 0.5, -1.7), (0.5, 0.5, -3.0), (0.0, 1.0, 0.0), 20.0, 3, 3)
    smp = orc.fi_samples(s, cam, orc.fi_params(spp=17, seed=1))
    assert not smp["valid"].any()
    assert np.all(orc.fi_pixels(s, cam, orc.fi_params(spp=17, seed=1)) == 0.0)
