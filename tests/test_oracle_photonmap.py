"""Pins of the oracle's photon-map radiance estimate (Eq. 5, Section 3.3): the phase weighting
against the normalisation of the HG phase function and its forward/backward orientation, the
fixed-radius and K-nearest estimates against the Poisson closed forms of uniform photon
sets, the K nearest on a lattice against its shells, bin selection, and the scores
Phi / sigma_t in a homogeneous medium."""
import math

import numpy as np
import pytest

from test_oracle_transport import homog_scene


def _sphere_quadrature(n_theta=96, n_phi=192):
    """Directions and weights of a product Gauss-Legendre x trapezoid rule on the sphere."""
    z, wz = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    zz, pp = np.meshgrid(z, phi, indexing="ij")
    s = np.sqrt(1 - zz ** 2)
    dirs = np.stack([s * np.cos(pp), s * np.sin(pp), zz], -1).reshape(-1, 3)
    w = (wz[:, None] * np.full(n_phi, 2 * math.pi / n_phi)[None, :]).reshape(-1)
    return dirs, w


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


@pytest.mark.parametrize("g", [0.0, 0.6, -0.8])
def test_direction_average_is_the_isotropic_estimate(orc, g):
    """Integrating Eq. (5) over all w gives sum(score) / V (the phase function integrates to 1),
    the estimate an isotropic cache makes from the same records."""
    rng = np.random.default_rng(1)
    n = 40
    rx = 0.5 + rng.uniform(-0.05, 0.05, (n, 3))
    rw = _unit(rng.normal(size=(n, 3)))
    rs = rng.uniform(0.1, 1.0, (n, 3))
    rb = np.zeros(n, dtype=np.int32)
    dirs, wq = _sphere_quadrature()
    x = np.tile([0.5, 0.5, 0.5], (dirs.shape[0], 1))
    L, r_used, n_used = orc.pm_estimate(rx, rw, rs, rb, [g], 0.2, 0, x, dirs,
                                        np.zeros(dirs.shape[0], dtype=np.int32))
    avg = (L * wq[:, None]).sum(0)
    V = 4 / 3 * math.pi * 0.2 ** 3
    np.testing.assert_allclose(avg, rs.sum(0) / V, rtol=1e-6 if g != -0.8 else 1e-4)
    assert np.all(n_used == n) and np.all(r_used == 0.2)


@pytest.mark.parametrize("g", [0.7, -0.7])
def test_phase_orientation_forward_for_positive_g(orc, g):
    """One photon travelling along +z: with g > 0 the scattered light is brightest along +z
    (forward), with g < 0 along -z."""
    rx, rw, rs = np.array([[0.5, 0.5, 0.5]]), np.array([[0.0, 0.0, 1.0]]), np.ones((1, 3))
    qw = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    L, _, _ = orc.pm_estimate(rx, rw, rs, [0], [g], 0.1, 0, np.tile([0.52, 0.5, 0.5], (3, 1)), qw,
                              [0, 0, 0])
    fwd, bwd, side = L[:, 0]
    assert (fwd > side > bwd) if g > 0 else (bwd > side > fwd)
    # the ratio of forward to backward is ((1 + |g|) / (1 - |g|))^3 for HG
    assert max(fwd, bwd) / min(fwd, bwd) == pytest.approx(((1 + abs(g)) / (1 - abs(g))) ** 3,
                                                         rel=1e-12)


def test_fixed_radius_estimate_of_a_uniform_photon_set(orc):
    """Photons of intensity lam per unit volume (Poisson), isotropic phase: E[L] = lam s / (4 pi)
    for any radius (the count in the sphere is Poisson with mean lam V)."""
    rng = np.random.default_rng(2)
    lam, s = 20000.0, 0.5
    n = rng.poisson(lam)
    rx = rng.uniform(0, 1, (n, 3))
    rw = _unit(rng.normal(size=(n, 3)))
    rs = np.full((n, 3), s)
    nq = 400
    qx = rng.uniform(0.2, 0.8, (nq, 3))
    qw = _unit(rng.normal(size=(nq, 3)))
    r = 0.08
    L, _, n_used = orc.pm_estimate(rx, rw, rs, np.zeros(n, np.int32), [0.0], r, 0, qx, qw,
                                   np.zeros(nq, np.int32))
    expect = lam * s / (4 * math.pi)
    # the mean count is lam V = 42.9; queries overlap, so bound the error loosely by 4 SE of
    # independent spheres
    se = expect / math.sqrt(lam * 4 / 3 * math.pi * r ** 3) / math.sqrt(nq) * 3
    assert abs(L[:, 0].mean() - expect) < 4 * se
    np.testing.assert_allclose(L[:, 0], n_used * s / (4 * math.pi) / (4 / 3 * math.pi * r ** 3),
                               rtol=1e-12)


def test_knn_estimate_of_a_uniform_photon_set(orc):
    """K nearest of a Poisson set of intensity lam: 1/V_K is lam / Gamma(K) distributed, so
    E[K s / (4 pi V_K)] = lam s K / ((K - 1) 4 pi)."""
    rng = np.random.default_rng(3)
    lam, s, K = 50000.0, 0.25, 32
    n = rng.poisson(lam)
    rx = rng.uniform(0, 1, (n, 3))
    rw = _unit(rng.normal(size=(n, 3)))
    rs = np.full((n, 3), s)
    nq = 3000
    qx = rng.uniform(0.3, 0.7, (nq, 3))
    qw = _unit(rng.normal(size=(nq, 3)))
    L, r_used, n_used = orc.pm_estimate(rx, rw, rs, np.zeros(n, np.int32), [0.0], 0.2, K, qx, qw,
                                        np.zeros(nq, np.int32))
    assert np.all(n_used == K)
    expect = lam * s * K / ((K - 1) * 4 * math.pi)
    # Var of 1/Gamma(K): lam^2 / ((K-1)^2 (K-2)); the queries are nearly independent
    se = expect / math.sqrt(K - 2) / math.sqrt(nq)
    assert abs(L[:, 0].mean() - expect) < 5 * se
    # r_used is the distance to the K-th nearest: exactly K records lie within it
    d = np.linalg.norm(rx[None, :50] - qx[:1, None], axis=-1)  # sanity on the first query
    dd = np.sort(np.linalg.norm(rx - qx[0], axis=1))
    assert r_used[0] == pytest.approx(dd[K - 1], rel=1e-14)
    assert d.shape == (1, 50)


def test_knn_on_a_lattice_takes_whole_shells(orc):
    """Records on a cubic lattice of spacing h with one at the query: the shells hold 1 (at 0),
    6 (at h), 12 (at h sqrt 2) and 8 (at h sqrt 3) records."""
    h = 0.01
    ii = np.arange(-3, 4)
    g = np.stack(np.meshgrid(ii, ii, ii, indexing="ij"), -1).reshape(-1, 3) * h + 0.5
    n = g.shape[0]
    rw = np.tile([0.0, 0.0, 1.0], (n, 1))
    rs = np.ones((n, 3))
    for k, r_exp in ((7, h), (19, h * math.sqrt(2)), (27, h * math.sqrt(3))):
        L, r_used, n_used = orc.pm_estimate(g, rw, rs, np.zeros(n, np.int32), [0.0], 0.05, k,
                                            [[0.5, 0.5, 0.5]], [[1.0, 0.0, 0.0]], [0])
        assert n_used[0] == k
        assert r_used[0] == pytest.approx(r_exp, rel=1e-12)
        np.testing.assert_allclose(L[0], k / (4 * math.pi) / (4 / 3 * math.pi * r_exp ** 3),
                                   rtol=1e-12)
    # fewer records than k within the maximum radius: all of them, r = the farthest found
    L, r_used, n_used = orc.pm_estimate(g, rw, rs, np.zeros(n, np.int32), [0.0], 1.5 * h, 100,
                                        [[0.5, 0.5, 0.5]], [[1.0, 0.0, 0.0]], [0])
    assert n_used[0] == 19 and r_used[0] == pytest.approx(h * math.sqrt(2), rel=1e-12)
    # nothing within the radius: zero
    L, r_used, n_used = orc.pm_estimate(g, rw, rs, np.zeros(n, np.int32), [0.0], 0.001, 4,
                                        [[0.505, 0.505, 0.505]], [[1.0, 0.0, 0.0]], [0])
    assert n_used[0] == 0 and r_used[0] == 0.0 and np.all(L == 0.0)


def test_only_the_query_bin_counts(orc):
    rng = np.random.default_rng(4)
    n = 500
    rx = 0.5 + rng.uniform(-0.1, 0.1, (n, 3))
    rw = _unit(rng.normal(size=(n, 3)))
    rs = rng.uniform(0, 1, (n, 3))
    rb = rng.integers(0, 3, n).astype(np.int32)
    qx, qw = [[0.5, 0.5, 0.5]], [[0.0, 1.0, 0.0]]
    full, _, nf = orc.pm_estimate(rx, rw, rs, rb, [-0.5, 0.0, 0.5], 0.08, 16, qx, qw, [2])
    sel = rb == 2
    only, _, no = orc.pm_estimate(rx[sel], rw[sel], rs[sel], rb[sel], [-0.5, 0.0, 0.5], 0.08, 16,
                                  qx, qw, [2])
    np.testing.assert_array_equal(full, only)
    assert nf[0] == no[0] == 16


def test_scores_in_a_homogeneous_medium(orc):
    s = homog_scene(orc, 0.4, albedo=0.7)
    sig, _ = s.transfer(0.4)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.05, 0.95, (10, 3))
    p = rng.uniform(0, 2, (10, 3))
    np.testing.assert_allclose(orc.pm_scores(s, x, p), p / sig, rtol=1e-14)
