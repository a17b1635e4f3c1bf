"""Batches larger than one dispatch can hold.  A dispatch's grid counts fewer than 2^32
work-items, so the batched entry points split larger batches into several launches.  Each test
runs a batch past that limit:

  - field queries (one work-item per query) and photon-map estimates (one wavefront per query)
    over inputs that repeat with period T: every output must equal, bit for bit, the output of
    one launch over the first period (the same kernel and arithmetic per query, so any error in
    a piece's offsets shows as a mismatch);
  - the training-batch generator at its maximum size, 2^32 samples, against the FP64 oracle's
    samples at indices on both sides of every piece boundary (positions are FP32 uniforms, exact);
  - a photon map built from a trace with more record slots than one dispatch holds, against the
    map built from the same records compacted (one launch): equal cell offsets and, per cell,
    equal sums of the records' bit patterns.

They allocate up to about 112 GiB of device memory and free it at the end."""
import gc
import time

import numpy as np
import pytest

from gpu_common import gpu_context, say, scene_arrays, smooth_cache

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
G_BINS = [-0.5, 0.0, 0.6]


@pytest.fixture(autouse=True)
def _release_memory():
    yield
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def _repeat(tile, n):
    """The first n rows of tile repeated."""
    import torch
    T = tile.shape[0]
    out = torch.empty((n,) + tuple(tile.shape[1:]), dtype=tile.dtype, device=tile.device)
    k = n // T
    out[:k * T].view((k,) + tuple(tile.shape)).copy_(tile.unsqueeze(0).expand((k,) + tuple(tile.shape)))
    out[k * T:].copy_(tile[:n - k * T])
    return out


def _check_periodic(big, small, same=None):
    """big (n rows) against small (T rows) repeated; `same(a, b)` compares two equal-shaped
    blocks (default: bit-exact)."""
    import torch
    same = same or torch.equal
    T, n = small.shape[0], big.shape[0]
    k = n // T
    shape = tuple(small.shape)
    for j0 in range(0, k, 64):
        j1 = min(k, j0 + 64)
        blk = big[j0 * T:j1 * T].view((j1 - j0,) + shape)
        assert same(blk, small.unsqueeze(0).expand((j1 - j0,) + shape)), f"rows {j0 * T}.."
    assert same(big[k * T:], small[:n - k * T]), "tail"


def _unit_octant(rng, T):
    """Unit vectors with positive components: valid both as positions in [0,1]^3 and as
    directions, so one buffer serves as both inputs."""
    v = np.abs(rng.normal(size=(T, 3))) + 1e-3
    return (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("n, decode", [((1 << 30) + 4099, True), ((1 << 32) + 4099, False)])
def test_field_query_in_pieces(n, decode):
    import torch
    from paper_2304_07338_amd.pfn import Context, FieldConfig
    ctx = Context(0)
    ctx.field_init(FieldConfig(), seed=3)
    T = 1 << 20
    rng = np.random.default_rng(7)
    tile = torch.tensor(_unit_octant(rng, T), device=DEV)
    gtile = torch.tensor(rng.uniform(-0.9, 0.9, T).astype(np.float32), device=DEV)
    ref = ctx.field_query(tile, tile, gtile, "f16", decode=decode)
    buf, gb = _repeat(tile, n), _repeat(gtile, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.field_query(buf, buf, gb, "f16", decode=decode)
    torch.cuda.synchronize()
    say(f"  {n} queries (decode {decode}) in {time.perf_counter() - t0:.2f} s")
    del buf, gb
    if decode:
        _check_periodic(out[0], ref[0])
        _check_periodic(out[1], ref[1])
    else:
        _check_periodic(out, ref)
    ctx.close()


def test_train_batch_at_maximum_size(orc):
    """2^32 samples (positions only; the other outputs NULL) against the oracle."""
    import torch
    w, vol, tf, lights = scene_arrays("c0")
    ctx = gpu_context(vol, tf, lights)
    cache = smooth_cache(16, 3, seed=9)
    ctx.set_cache(torch.tensor(cache, dtype=torch.float32, device=DEV), [-0.5, 0.0, 0.5],
                  float(cache.max()))
    n = 1 << 32
    xyz = torch.empty((n, 3), dtype=torch.float32, device=DEV)
    t0 = time.perf_counter()
    ctx._ok(ctx.lib.pfn_train_batch(ctx.h, 42, 17, n, 0, xyz.data_ptr(), None, None, None, None))
    ctx.sync()
    say(f"  {n} samples in {time.perf_counter() - t0:.2f} s")
    P = 1 << 30
    idx = [0, 1, n - 2, n - 1]
    for b in (P, 2 * P, 3 * P):
        idx += [b - 2, b - 1, b, b + 1]
    idx += [int(i) for i in np.random.default_rng(2).integers(0, n, 48)]
    got = xyz[torch.tensor(idx, device=DEV)].cpu().numpy().astype(np.float64)
    del xyz
    oc = orc.OracleCache(cache, [-0.5, 0.0, 0.5], 16)
    for i, row in zip(idx, got):
        ox = orc.train_batch(42, 17, 1, oc, float(cache.max()), first=i)[0]
        np.testing.assert_array_equal(row, ox[0], err_msg=f"sample {i}")
    ctx.close()


def _cell_sums(m, n_start):
    """Per cell: the sums (wrapping in 64 bits) of the bit patterns of the records' nine values
    and of their squares, which do not depend on the records' order inside the cell."""
    import torch
    start = m["start"].long()
    counts = start[1:] - start[:-1]
    key = torch.repeat_interleave(torch.arange(n_start - 1, device=DEV), counts)
    cols = torch.cat([m["pos"], m["dir"], m["score"]], 1).contiguous().view(torch.int32).long()
    s1 = torch.zeros((n_start - 1, 9), dtype=torch.int64, device=DEV).index_add_(0, key, cols)
    s2 = torch.zeros((n_start - 1, 9), dtype=torch.int64, device=DEV).index_add_(0, key,
                                                                                  cols * cols)
    return start, s1, s2


def test_photon_map_build_in_pieces():
    """17.5 M photons with up to 63 records each: 1.1e9 record slots, two pieces."""
    import torch
    w, vol, tf, lights = scene_arrays("c0")
    ctx = gpu_context(vol, tf, lights)
    n_ph = 17_500_000
    st = ctx.trace_photon_cache(n_ph, G_BINS, cache_res=32, seed=3, max_collisions=64)
    n_rec = int(st["n_records"])
    assert n_ph * 63 > (1 << 30)
    G = 32
    n_start = len(G_BINS) * G ** 3 + 1
    t0 = time.perf_counter()
    ctx.photon_map_build(G)
    say(f"  map over {n_ph * 63} slots ({n_rec} records) in {time.perf_counter() - t0:.2f} s")
    a = ctx.photon_map_get(n_start, n_rec)
    assert a["n"] == n_rec
    sa = _cell_sums(a, n_start)
    del a
    r = ctx.get_records(n_rec)
    assert r["x"].shape[0] == n_rec
    ctx.photon_map_set(r["x"], r["w"], r["power"], r["bin"], G_BINS, G)
    del r
    b = ctx.photon_map_get(n_start, n_rec)
    assert b["n"] == n_rec
    sb = _cell_sums(b, n_start)
    del b
    for x, y, what in zip(sa, sb, ("cell offsets", "sums", "sums of squares")):
        assert torch.equal(x, y), what
    ctx.close()


@pytest.mark.parametrize("k", [0, 8])
def test_photon_estimate_in_pieces(k):
    """2^26 + 77 queries, one wavefront each: more than 2^32 work-items.  The K-nearest path
    fills its LDS ranking buffer through atomics, so its sums may differ in the last bit between
    launches; counts and radii stay exact."""
    import torch
    w, vol, tf, lights = scene_arrays("c0")
    vol = torch.full_like(vol, 0.5)
    ctx = gpu_context(vol, tf, lights)
    rng = np.random.default_rng(11)
    m = 20000
    T_ = lambda a: torch.tensor(a, device=DEV).contiguous()
    x = rng.uniform(0, 1, (m, 3)).astype(np.float32)
    d = rng.normal(size=(m, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    p = rng.uniform(0.01, 1.0, (m, 3)).astype(np.float32)
    b = rng.integers(0, 3, m).astype(np.int32)
    ctx.photon_map_set(T_(x), T_(d), T_(p), T_(b), G_BINS, grid_res=16)
    T = 1 << 16
    qx = T_(rng.uniform(0, 1, (T, 3)).astype(np.float32))
    qd = rng.normal(size=(T, 3))
    qd = T_((qd / np.linalg.norm(qd, axis=1, keepdims=True)).astype(np.float32))
    qb = rng.integers(-1, 3, T).astype(np.int32)
    qb = T_(qb)
    ref = ctx.photon_map_estimate(qx, qd, qb, 0.08, k)
    n = (1 << 26) + 77
    t0 = time.perf_counter()
    big = ctx.photon_map_estimate(_repeat(qx, n), _repeat(qd, n), _repeat(qb, n), 0.08, k)
    torch.cuda.synchronize()
    say(f"  {n} estimates (k {k}) in {time.perf_counter() - t0:.2f} s, counts of the first "
        f"period: mean {ref[2].float().mean().item():.1f}")
    close = None
    if k:
        close = lambda a, c: bool(torch.allclose(a, c, rtol=1e-6, atol=0.0))
    _check_periodic(big[0], ref[0], close)
    _check_periodic(big[1], ref[1])
    _check_periodic(big[2], ref[2])
    ctx.close()
