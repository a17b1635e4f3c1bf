"""Pins of the FP64 oracle's core definitions against facts fixed outside the oracle:
published known-answer vectors, closed forms, quadrature by library routines, invariants."""
import math
import os

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = orc.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_u01_exact_and_open_interval(orc):
    assert orc.u01(0) == 2.0 ** -24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    # every value is an odd multiple of 2^-24, hence exact in binary32 as well
    for x in [1, 511, 512, 123456789, 0x80000000]:
        v = orc.u01(x)
        k = v * 2 ** 24
        assert k == int(k) and int(k) % 2 == 1
        assert np.float32(v) == v


def test_uniform_stream_statistics(orc):
    u = np.concatenate([orc.uniforms(7, i, 3, 64) for i in range(2000)])
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("g", [-0.9, -0.5, 0.0, 0.3, 0.8, 0.95])
def test_hg_normalised_and_mean_cosine(orc, g):
    # integral over the sphere = 2 pi * int_{-1}^{1} p(mu) dmu, by 64-point Gauss-Legendre;
    # strongly peaked lobes are split at the peak side for accuracy
    x, w = leggauss(64)
    edges = np.array([-1.0, 0.0, 0.9, 0.99, 1.0]) if g > 0 else np.array([-1.0, -0.99, -0.9, 0.0, 1.0])
    tot = mean = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        mu = 0.5 * (b - a) * x + 0.5 * (b + a)
        p = np.array([orc.hg_eval(g, m) for m in mu])
        tot += 2 * math.pi * 0.5 * (b - a) * np.sum(w * p)
        mean += 2 * math.pi * 0.5 * (b - a) * np.sum(w * p * mu)
    assert abs(tot - 1.0) < 1e-9
    assert abs(mean - g) < 1e-9
    if g == 0.0:
        assert orc.hg_eval(0.0, 0.3) == pytest.approx(1 / (4 * math.pi), rel=1e-15)


@pytest.mark.parametrize("g", [-0.8, 0.0, 0.4, 0.8])
def test_hg_sampler_distribution(orc, g):
    n = 40000
    u = orc.uniforms(11, 0, 1, n)
    mu = np.array([orc.hg_sample_mu(g, v) for v in u])
    # mean cosine of the sampler equals g
    var = np.var(mu)
    assert abs(mu.mean() - g) < 4 * math.sqrt(var / n)
    # chi^2 against the HG density integrated by quadrature per bin (library quadrature)
    from scipy.integrate import quad
    edges = np.linspace(-1, 1, 33)
    probs = np.array([2 * math.pi * quad(lambda m: orc.hg_eval(g, m), a, b)[0]
                      for a, b in zip(edges[:-1], edges[1:])])
    counts, _ = np.histogram(mu, edges)
    ok = probs * n > 5
    chi = stats.chisquare(counts[ok], probs[ok] * n * counts[ok].sum() / (probs[ok] * n).sum())
    assert chi.pvalue > 1e-3


def test_hg_sample_direction_frame(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        g = rng.uniform(-0.9, 0.9)
        u1, u2 = rng.uniform(size=2)
        d = orc.hg_sample_dir(g, w, u1, u2)
        assert abs(np.linalg.norm(d) - 1) < 1e-12
        assert abs(d @ w - orc.hg_sample_mu(g, u1)) < 1e-12
    # azimuth is uniform: the perpendicular component averages to zero
    w = np.array([0.3, -0.5, 0.81])
    w /= np.linalg.norm(w)
    perp = np.zeros(3)
    n = 4000
    for i in range(n):
        u1, u2 = (i + 0.5) / n, ((i * 0.618034) % 1.0)
        d = orc.hg_sample_dir(0.0, w, u1, u2)
        perp += d - (d @ w) * w
    assert np.linalg.norm(perp / n) < 0.01


def _scene(orc, density, tf=None, ext=20.0, lights=None):
    if tf is None:
        tf = np.zeros((256, 4))
        tf[:, :3] = 0.7
        tf[:, 3] = np.arange(256) / 255.0
    if lights is None:
        lights = np.array([[2.0, 0.5, 0.5, 1.0, 1.0, 1.0]])
    return orc.OracleScene(density, tf, ext, lights)


def test_trilinear_exact_at_centres_and_linear_fields(orc):
    n = (5, 6, 7)  # nx, ny, nz
    rng = np.random.default_rng(1)
    vol = rng.uniform(size=(n[2], n[1], n[0]))
    s = _scene(orc, vol)
    for _ in range(50):
        i, j, k = rng.integers(0, n[0]), rng.integers(0, n[1]), rng.integers(0, n[2])
        x = [(i + 0.5) / n[0], (j + 0.5) / n[1], (k + 0.5) / n[2]]
        assert s.density_at(x)[0] == pytest.approx(vol[k, j, i], abs=1e-15)
    # a linear field is reproduced exactly between the first and last cell centres
    zz, yy, xx = np.meshgrid(*[(np.arange(m) + 0.5) / m for m in (n[2], n[1], n[0])], indexing="ij")
    lin = 0.1 + 0.2 * xx + 0.3 * yy + 0.25 * zz
    s2 = _scene(orc, lin)
    for _ in range(50):
        x = [rng.uniform(0.5 / n[a], 1 - 0.5 / n[a]) for a in range(3)]
        assert s2.density_at(x)[0] == pytest.approx(0.1 + 0.2 * x[0] + 0.3 * x[1] + 0.25 * x[2],
                                                     abs=1e-14)
    # clamp-to-edge inside the half-voxel border, zero outside the cube
    assert s.density_at([0.0, (0.5) / n[1], (0.5) / n[2]])[0] == pytest.approx(vol[0, 0, 0])
    assert s.density_at([1.0, 1.0, 1.0])[0] == pytest.approx(vol[-1, -1, -1])
    assert s.density_at([-1e-9, 0.5, 0.5])[0] == 0.0
    assert s.density_at([0.5, 1.0 + 1e-9, 0.5])[0] == 0.0


def test_transfer_function_interpolation(orc):
    rng = np.random.default_rng(2)
    tf = rng.uniform(size=(256, 4))
    s = _scene(orc, np.zeros((2, 2, 2)), tf=tf, ext=20.0)
    for e in [0, 1, 77, 254, 255]:
        sig, alb = s.transfer(e / 255.0)
        assert sig == pytest.approx(20.0 * tf[e, 3], rel=1e-14)
        np.testing.assert_allclose(alb, tf[e, :3], rtol=1e-14)
    sig, alb = s.transfer(100.25 / 255.0)
    np.testing.assert_allclose(alb, 0.75 * tf[100, :3] + 0.25 * tf[101, :3], rtol=1e-13)
    assert s.majorant() == pytest.approx(20.0 * tf[:, 3].max())


def test_clip_cube_cases(orc):
    hit, t0, t1 = orc.clip_cube([0.5, 0.5, -1.0], [0, 0, 1.0])
    assert hit and t0 == pytest.approx(1.0) and t1 == pytest.approx(2.0)
    hit, t0, t1 = orc.clip_cube([0.5, 0.5, 0.5], [1.0, 0, 0])  # from inside
    assert hit and t0 == 0.0 and t1 == pytest.approx(0.5)
    d = np.array([1.0, 1.0, 1.0]) / math.sqrt(3)
    hit, t0, t1 = orc.clip_cube([-1.0, -1.0, -1.0], d)
    assert hit and t0 == pytest.approx(math.sqrt(3)) and t1 == pytest.approx(2 * math.sqrt(3))
    hit, _, _ = orc.clip_cube([2.0, 0.5, 0.5], [0, 1.0, 0])  # parallel, outside
    assert not hit
    hit, _, _ = orc.clip_cube([0.5, 0.5, -1.0], [0, 0, -1.0])  # pointing away
    assert not hit


@pytest.mark.parametrize("step", [1 / 128, 0.013, 0.1])
def test_shadow_transmittance_beer_lambert(orc, step):
    """Homogeneous cube: T = exp(-sigma * chord) for any step (the last step is clipped)."""
    rho = 0.6
    s = _scene(orc, np.full((8, 8, 8), rho))
    sig, _ = s.transfer(rho)
    cases = [
        ([0.5, 0.5, 0.5], [2.0, 0.5, 0.5], 0.5),          # to the +x face
        ([0.25, 0.5, 0.5], [0.25, 0.5, 3.0], 0.5),        # to the +z face
        ([0.2, 0.2, 0.2], [2.0, 2.0, 2.0], 0.8 * math.sqrt(3)),  # along the diagonal
        ([0.5, 0.5, 0.5], [0.5, 0.9, 0.5], 0.4),          # light inside the cube
        ([0.1, 0.5, 0.5], [-5.0, 0.5, 0.5], 0.1),         # to the -x face
    ]
    for x, p, chord in cases:
        assert s.shadow_T(x, p, step) == pytest.approx(math.exp(-sig * chord), rel=1e-12)


def test_cache_gather_trilinear_and_g_interpolation(orc):
    res = 4
    rng = np.random.default_rng(3)
    data = rng.uniform(size=(3, res, res, res, 3))
    c = orc.OracleCache(data, [-0.5, 0.0, 0.5], res)
    x = [(1 + 0.5) / res, (2 + 0.5) / res, (0 + 0.5) / res]
    np.testing.assert_allclose(c.gather(x, 0.0), data[1, 0, 2, 1], rtol=1e-14)
    np.testing.assert_allclose(c.gather(x, -0.9), data[0, 0, 2, 1], rtol=1e-14)  # clamped low
    np.testing.assert_allclose(c.gather(x, 0.7), data[2, 0, 2, 1], rtol=1e-14)  # clamped high
    np.testing.assert_allclose(c.gather(x, 0.125), 0.75 * data[1, 0, 2, 1] + 0.25 * data[2, 0, 2, 1],
                               rtol=1e-13)
    # midway between two cell centres along x
    xm = [(1 + 1.0) / res, (2 + 0.5) / res, (0 + 0.5) / res]
    np.testing.assert_allclose(c.gather(xm, -0.5), 0.5 * (data[0, 0, 2, 1] + data[0, 0, 2, 2]),
                               rtol=1e-13)


def test_image_error_metrics(orc):
    rng = np.random.default_rng(4)
    ref = rng.uniform(size=1000)
    img = ref + rng.normal(scale=0.01, size=1000)
    rmse, rel, psnr = orc.image_error(img, ref)
    r = np.sqrt(np.mean((img - ref) ** 2))
    assert rmse == pytest.approx(r, rel=1e-12)
    assert rel == pytest.approx(r / ref.mean(), rel=1e-12)
    assert psnr == pytest.approx(20 * np.log10(ref.max() / r), rel=1e-12)
