"""Pins of the oracle's photon field, target encoding, optimiser and batch generator."""
import math

import numpy as np
import pytest
import torch

C1_DESC = dict(levels=16, feats=2, base_res=16, growth=1.5, log2_table=19, hidden_layers=3,
               width=64, psi=5.0)


def small_desc(orc, **kw):
    d = dict(levels=4, feats=2, base_res=4, growth=1.5, log2_table=8, hidden_layers=2, width=8,
             psi=5.0)
    d.update(kw)
    return orc.field_desc(**d)


def test_layout_counts_for_the_c1_field(orc):
    """16 levels x 2 features, base 16, growth 1.5, T = 2^19: level resolutions floor(16*1.5^l),
    dense levels where (N+1)^d <= T, MLP 65-64-64-64-3 without biases."""
    d = orc.field_desc(**C1_DESC)
    L = orc.field_layout(d)
    res = [int(math.floor(16 * 1.5 ** l)) for l in range(16)]
    assert list(L.pos_res)[:16] == res
    assert [l for l in range(16) if L.pos_dense[l]] == [0, 1, 2, 3]
    assert [l for l in range(16) if L.dir_dense[l]] == list(range(10))
    assert L.pos_off[16] == 6529022 and L.dir_off[16] == 3829586
    assert L.n_in == 65
    assert L.n_params - L.mlp_off == 64 * 65 + 64 * 64 + 64 * 64 + 3 * 64 == 12544
    assert L.n_params == 2 * (6529022 + 3829586) + 12544 == 20729760


def test_dense_level_index_is_row_major(orc):
    d = small_desc(orc)
    L = orc.field_layout(d)
    n = L.n_params
    p = np.zeros(n)
    # feature 0 of entry e = its index within its level, feature 1 = -index
    for l in range(d.levels):
        if not L.pos_dense[l]:
            continue
        cnt = (L.pos_res[l] + 1) ** 3
        e = np.arange(cnt)
        p[2 * (L.pos_off[l] + e)] = e
        p[2 * (L.pos_off[l] + e) + 1] = -e
    for l in range(d.levels):
        if not L.pos_dense[l]:
            continue
        N = L.pos_res[l]
        for v in [(0, 0, 0), (1, 2, 3), (N, N, N), (N - 1, 0, N)]:
            x = np.array(v, dtype=float) / N
            z = orc.field_encode(d, p, x, [0, 0, 1.0], 0.0)
            idx = v[0] + v[1] * (N + 1) + v[2] * (N + 1) ** 2
            assert z[2 * l] == pytest.approx(idx, abs=1e-9)
            assert z[2 * l + 1] == pytest.approx(-idx, abs=1e-9)


def test_hashed_level_uses_the_instant_ngp_hash(orc):
    """For a hashed level, the feature at vertex v is table[(v0*1 ^ v1*2654435761 ^ v2*805459861)
    mod T] (Mueller et al. 2022, Section 3; primes as published)."""
    d = orc.field_desc(**C1_DESC)
    L = orc.field_layout(d)
    l = 6
    assert not L.pos_dense[l]
    T = 1 << 19
    N = L.pos_res[l]
    p = np.zeros(L.n_params)
    e = np.arange(T)
    p[2 * (L.pos_off[l] + e)] = e
    # at a level vertex the interpolation weight of that corner is 1, so the feature is the
    # table entry at the hashed index; the primes are 2654435761 = 0x9E3779B1 and 805459861
    cases = {(0, 1, 0): 0x9E3779B1 & 0x7FFFF, (0, 0, 1): 805459861 & 0x7FFFF, (1, 0, 0): 1,
             (3, 0, 0): 3}
    for v, expected in cases.items():
        x = np.array(v, dtype=float) / N
        z = orc.field_encode(d, p, x, [0, 0, 1.0], 0.0)
        assert z[2 * l] == pytest.approx(expected, abs=1e-6), v


def test_direction_encoding_spherical_coordinates(orc):
    """w -> (theta/pi, (phi+pi)/(2pi)); dense 2-D level 0 with N=16: vertex (i,j) has index
    i + 17 j."""
    d = small_desc(orc, base_res=16, levels=1, log2_table=12)
    L = orc.field_layout(d)
    p = np.zeros(L.n_params)
    cnt = 17 * 17
    e = np.arange(cnt)
    p[L.pos_params + 2 * e] = e
    cases = [([1.0, 0, 0], (8, 8)),        # theta = pi/2, phi = 0
             ([0, 0, 1.0], (0, 8)),         # theta = 0, atan2(0, 0) = 0
             ([0, 1.0, 0], (8, 12)),        # phi = pi/2 -> 0.75
             ([0, -1.0, 0], (8, 4))]        # phi = -pi/2 -> 0.25
    for w, (i, j) in cases:
        z = orc.field_encode(d, p, [0.5, 0.5, 0.5], w, 0.0)
        assert z[2] == pytest.approx(i + 17 * j, abs=1e-9)
    # g passes through unencoded as the last input
    z = orc.field_encode(d, p, [0.3, 0.3, 0.3], [0, 0, 1.0], -0.37)
    assert z[-1] == -0.37


def test_partition_of_unity(orc):
    d = orc.field_desc(**C1_DESC)
    L = orc.field_layout(d)
    p = np.ones(L.n_params)
    rng = np.random.default_rng(5)
    for _ in range(5):
        x = rng.uniform(size=3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        z = orc.field_encode(d, p, x, w, 0.2)
        np.testing.assert_allclose(z[:-1], 1.0, atol=1e-12)


def _mats(orc, d, p):
    L = orc.field_layout(d)
    return [p[L.w_off[m]:L.w_off[m] + L.w_rows[m] * L.w_cols[m]].reshape(L.w_rows[m], L.w_cols[m])
            for m in range(L.n_mats)]


def test_mlp_forward_matches_library_matmul(orc):
    d = small_desc(orc, hidden_layers=3, width=16)
    L = orc.field_layout(d)
    rng = np.random.default_rng(6)
    p = rng.normal(scale=0.5, size=L.n_params)
    xs = rng.uniform(size=(20, 3))
    ws = rng.normal(size=(20, 3))
    ws /= np.linalg.norm(ws, axis=1, keepdims=True)
    gs = rng.uniform(-0.9, 0.9, 20)
    out = orc.field_forward(d, p, xs, ws, gs)
    W = _mats(orc, d, p)
    for i in range(20):
        z = orc.field_encode(d, p, xs[i], ws[i], gs[i])
        h = z
        for m in range(len(W) - 1):
            h = np.maximum(W[m] @ h, 0.0)
        np.testing.assert_allclose(out[i], W[-1] @ h, rtol=1e-12, atol=1e-14)


def test_zero_input_gives_zero_output(orc):
    d = small_desc(orc)
    L = orc.field_layout(d)
    rng = np.random.default_rng(7)
    p = rng.normal(size=L.n_params)
    p[:L.mlp_off] = 0.0
    out = orc.field_forward(d, p, [[0.3, 0.4, 0.5]], [[0, 0, 1.0]], [0.0])
    assert np.all(out == 0.0)


def test_loss_gradient_matches_finite_differences(orc):
    d = small_desc(orc, levels=5, base_res=3, log2_table=7, hidden_layers=2, width=8)
    L = orc.field_layout(d)
    rng = np.random.default_rng(8)
    p = rng.normal(scale=0.3, size=L.n_params)
    n = 16
    xs = rng.uniform(size=(n, 3))
    ws = rng.normal(size=(n, 3))
    ws /= np.linalg.norm(ws, axis=1, keepdims=True)
    gs = rng.uniform(-0.8, 0.8, n)
    tgt = rng.uniform(size=(n, 3))
    loss, grad = orc.field_loss_grad(d, p, xs, ws, gs, tgt)
    out = orc.field_forward(d, p, xs, ws, gs)
    assert loss == pytest.approx(np.mean((out - tgt) ** 2), rel=1e-12)
    # central differences on every touched parameter and a sample of the rest
    idx = np.concatenate([np.flatnonzero(grad)[:: max(1, np.count_nonzero(grad) // 150)],
                          rng.integers(0, L.n_params, 20)])
    h = 1e-6
    for j in idx:
        pp = p.copy()
        pp[j] += h
        lp = np.mean((orc.field_forward(d, pp, xs, ws, gs) - tgt) ** 2)
        pp[j] -= 2 * h
        lm = np.mean((orc.field_forward(d, pp, xs, ws, gs) - tgt) ** 2)
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(grad[j], rel=1e-5, abs=1e-9), j


def test_relative_loss_gradient_is_the_weighted_l2_gradient(orc):
    """Relative L2: sum (y - t)^2 / (y^2 + 0.01) with the denominator held constant, i.e. the
    gradient of sum w (y - t)^2 with w frozen at the current prediction (checked by central
    differences of that frozen-weight loss), and the loss value at the current parameters."""
    d = small_desc(orc, levels=5, base_res=3, log2_table=7, hidden_layers=2, width=8)
    L = orc.field_layout(d)
    rng = np.random.default_rng(18)
    p = rng.normal(scale=0.3, size=L.n_params)
    n = 16
    xs = rng.uniform(size=(n, 3))
    ws = rng.normal(size=(n, 3))
    ws /= np.linalg.norm(ws, axis=1, keepdims=True)
    gs = rng.uniform(-0.8, 0.8, n)
    tgt = rng.uniform(size=(n, 3))
    loss, grad = orc.field_loss_grad(d, p, xs, ws, gs, tgt, loss="rel")
    out = orc.field_forward(d, p, xs, ws, gs)
    wfz = 1.0 / (out ** 2 + 0.01)
    assert loss == pytest.approx(np.mean((out - tgt) ** 2 * wfz), rel=1e-12)
    l2, g2 = orc.field_loss_grad(d, p, xs, ws, gs, tgt)
    assert not np.allclose(grad, g2)  # the weighting changes the gradient
    idx = np.concatenate([np.flatnonzero(grad)[:: max(1, np.count_nonzero(grad) // 100)],
                          rng.integers(0, L.n_params, 10)])
    h = 1e-6
    for j in idx:
        pp = p.copy()
        pp[j] += h
        lp = np.mean(wfz * (orc.field_forward(d, pp, xs, ws, gs) - tgt) ** 2)
        pp[j] -= 2 * h
        lm = np.mean(wfz * (orc.field_forward(d, pp, xs, ws, gs) - tgt) ** 2)
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(grad[j], rel=5e-5, abs=1e-8), j  # weights up to 100


def test_rounding_matches_library_conversions(orc):
    rng = np.random.default_rng(9)
    vals = np.concatenate([rng.normal(scale=s, size=2000) for s in (1e-6, 1e-3, 1.0, 300.0)])
    vals = np.concatenate([vals, [0.0, 65504.0, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 2 ** -24, 3 * 2 ** -25]])
    h = np.array([orc.round_half(v) for v in vals])
    np.testing.assert_array_equal(h, vals.astype(np.float16).astype(np.float64))
    b = np.array([orc.round_bf16(v) for v in vals])
    ref = torch.tensor(vals, dtype=torch.float64).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(b, ref)


def test_log_encoding_round_trip(orc):
    psi = 5.0
    for v in [1.0, 0.5, 1e-3, 1.0000001e-5, 3e-5]:
        lp = orc.log_encode(v, psi)
        assert 0.0 <= lp <= 1.0
        assert orc.exp_decode(lp, psi) == pytest.approx(v, rel=1e-14)
    assert orc.log_encode(1e-5, psi) == 1.0      # at the threshold: not above it
    assert orc.log_encode(1e-9, psi) == 1.0
    assert orc.log_encode(0.0, psi) == 1.0
    assert orc.exp_decode(1.0, psi) == pytest.approx(1e-5, rel=1e-15)
    assert orc.log_encode(1.0, psi) == 0.0


def test_adam_matches_library_optimizer(orc):
    rng = np.random.default_rng(10)
    n = 257
    p0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * s for s in (1.0, 0.1, 3.0, 1e-3, 0.5)]
    lrs = [9e-4, 9e-4, 8e-4, 7e-4, 1e-4]
    p = p0.copy()
    m = np.zeros(n)
    v = np.zeros(n)
    for t, (g, lr) in enumerate(zip(grads, lrs), start=1):
        orc.adam_step(p, g, m, v, t, lr)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=lrs[0], betas=(0.9, 0.99), eps=1e-15)
    for g, lr in zip(grads, lrs):
        for grp in opt.param_groups:
            grp["lr"] = lr
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_adam_first_step_is_signed_lr(orc):
    g = np.array([3.0, -2e-3, 5e-7, -40.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    orc.adam_step(p, g, m, v, 1, 9e-4)
    np.testing.assert_allclose(p, -9e-4 * np.sign(g), rtol=1e-7)


def test_learning_rate_schedule(orc):
    """9e-4, x0.92 at 70% of 2000 steps (step 1400) and every 25 steps after."""
    assert orc.lr_at(0) == 9e-4
    assert orc.lr_at(1399) == 9e-4
    assert orc.lr_at(1400) == pytest.approx(9e-4 * 0.92, rel=1e-15)
    assert orc.lr_at(1424) == pytest.approx(9e-4 * 0.92, rel=1e-15)
    assert orc.lr_at(1425) == pytest.approx(9e-4 * 0.92 ** 2, rel=1e-15)
    assert orc.lr_at(1999) == pytest.approx(1.2166e-4, rel=1e-4)
    assert orc.lr_at(1999) == pytest.approx(9e-4 * 0.92 ** 24, rel=1e-14)


def test_training_batch_distribution_and_targets(orc):
    res = 8
    rng = np.random.default_rng(11)
    data = rng.uniform(1e-4, 1.0, size=(5, res, res, res, 3))
    gb = [-0.8, -0.4, 0.0, 0.4, 0.8]
    cache = orc.OracleCache(data, gb, res)
    kappa = data.max()
    n = 20000
    xyz, dirs, g, b, tgt = orc.train_batch(123, 7, n, cache, kappa)
    assert xyz.min() > 0 and xyz.max() < 1
    assert abs(xyz.mean() - 0.5) < 0.01
    np.testing.assert_allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-12)
    assert np.all(np.abs(dirs.mean(axis=0)) < 0.03)
    counts = np.bincount(b, minlength=5)
    assert stats_chi_ok(counts)
    np.testing.assert_array_equal(g, np.array(gb)[b])
    for i in range(0, n, 997):
        v = cache.gather(xyz[i], g[i]) / kappa
        for c in range(3):
            assert tgt[i, c] == pytest.approx(orc.log_encode(v[c], 5.0), rel=1e-14)
    # different steps give different batches, equal seeds give equal batches
    xyz2 = orc.train_batch(123, 8, 10, cache, kappa)[0]
    xyz3 = orc.train_batch(123, 7, 10, cache, kappa)[0]
    assert not np.allclose(xyz2, xyz[:10])
    np.testing.assert_array_equal(xyz3, xyz[:10])
    # a range of the batch: the same samples as rows first .. first + n - 1 of the whole batch
    part = orc.train_batch(123, 7, 40, cache, kappa, first=9000)
    for a, whole in zip(part, (xyz, dirs, g, b, tgt)):
        np.testing.assert_array_equal(a, whole[9000:9040])


def test_uniform_g_batch_pins(orc):
    """Batches with g uniform over [g_0, g_last] (targets interpolated linearly in g): the same
    positions and directions as pool batches (the same draws), g mapping back to the pool's bin
    draw, a uniform distribution of g, and closed-form targets for a cache that is constant in
    space and linear in g (so that linear interpolation between bins is exact)."""
    res = 4
    gb = [-0.75, -0.1, 0.3, 0.8]
    alpha = np.array([0.5, 0.3, 0.2])
    beta = np.array([0.2, -0.1, 0.15])
    data = np.zeros((4, res, res, res, 3))
    for b, gv in enumerate(gb):
        data[b] = alpha + beta * gv
    cache = orc.OracleCache(data, gb, res)
    kappa = 0.9
    n = 40000
    px, pd, pg, pb, _ = orc.train_batch(77, 3, n, cache, kappa)
    ux, ud, ug, ub, ut = orc.train_batch(77, 3, n, cache, kappa, g_sampling="uniform")
    np.testing.assert_array_equal(ux, px)
    np.testing.assert_array_equal(ud, pd)
    assert ug.min() > gb[0] and ug.max() < gb[-1]
    # the uniform draw behind both: u = (g - g0) / (g_last - g0) gives the pool's bin floor(u n)
    u = (ug - gb[0]) / (gb[-1] - gb[0])
    np.testing.assert_array_equal(np.minimum(np.floor(u * 4).astype(int), 3), pb)
    from scipy import stats
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # reported bin: the lower neighbour of g
    edges = np.array(gb)
    np.testing.assert_array_equal(ub, np.clip(np.searchsorted(edges, ug, side="right") - 1, 0, 2))
    # closed form: the cache value at g is alpha + beta g
    want = np.array([[orc.log_encode(v / kappa, 5.0) for v in alpha + beta * gg] for gg in ug[:500]])
    np.testing.assert_allclose(ut[:500], want, rtol=1e-13, atol=1e-15)


def stats_chi_ok(counts):
    from scipy import stats
    return stats.chisquare(counts).pvalue > 1e-3
