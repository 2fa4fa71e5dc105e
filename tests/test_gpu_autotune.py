"""gccd_autotune: the measured launch shape (targets per thread, source
chunks, tile size) is one of the candidates, keeps the field within the
Eq. (6) tolerance, and reproduces bit for bit when fixed again with
gccd_set_launch and gccd_set_tile in a fresh context.  gccd_set_tile: every
tile size meets the tolerance, and the automatic choice takes 64-source
tiles for a small cloud and 256 for a large one."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_11043_amd import gccd
    return gccd


@pytest.fixture(scope="module")
def W():
    from paper_2203_11043_amd import workloads
    return workloads


def gpu(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def test_autotune_single_cloud_and_batch(g, W, orc):
    w = W.single_cloud(30000, seed=12, depth_um=120.0)
    d = dict(W.DEVICE, event=4)
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        g.gccd_load(ctx, *gpu(w.x, w.y, w.z))
        tpt, chunks, ms = g.gccd_autotune(ctx)
        st = g.gccd_stats(ctx)
        tile = st["tile_sources"]
        print(f"[autotune] n=30000: tpt {tpt}, chunks {chunks}, tile {tile}, {ms:.3f} ms per "
              "launch", flush=True)
        assert tpt in (1, 2, 4) and chunks in (0, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 48, 56, 64) and ms > 0
        assert st["targets_per_thread"] == tpt
        assert tile in ((64, 128, 256) if tpt == 1 else (256,))
        E = g.gccd_field(ctx, w.n).cpu().numpy()
        g.gccd_run(ctx, 10.0, 20)
        p1, _ = g.gccd_positions(ctx, w.n)
        p1 = p1.cpu().numpy()
    finally:
        g.gccd_destroy(ctx)
    idx = np.random.default_rng(3).choice(w.n, 200, replace=False)
    Eo, A = orc.field([w.x[idx], w.y[idx], w.z[idx]], [w.x, w.y, w.z], with_magnitude=True)
    check_field(E[:, idx], Eo, A)
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        g.gccd_set_launch(ctx, tpt, chunks)
        g.gccd_set_tile(ctx, tile)
        g.gccd_load(ctx, *gpu(w.x, w.y, w.z))
        assert g.gccd_stats(ctx)["tile_sources"] == tile
        g.gccd_run(ctx, 10.0, 20)
        p2, _ = g.gccd_positions(ctx, w.n)
        assert np.array_equal(p1, p2.cpu().numpy())
    finally:
        g.gccd_destroy(ctx)

    # a batch of uneven events: chunks capped per event, results within tolerance
    sizes = [300, 5000, 40, 12000, 900]
    xs, ys, zs, off = [], [], [], [0]
    for e, n in enumerate(sizes):
        x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, 50.0 + 100 * e), 6,
                                   stream=800 + e)
        xs.append(x)
        ys.append(y)
        zs.append(z)
        off.append(off[-1] + n)
    x, y, z = np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        g.gccd_load_events(ctx, off, *gpu(x, y, z))
        tpt, chunks, ms = g.gccd_autotune(ctx)
        tile = g.gccd_stats(ctx)["tile_sources"]
        print(f"[autotune] batch: tpt {tpt}, chunks {chunks}, tile {tile}, {ms:.3f} ms",
              flush=True)
        E = g.gccd_field(ctx, len(x)).cpu().numpy()
    finally:
        g.gccd_destroy(ctx)
    for e in range(len(sizes)):
        sl = slice(off[e], off[e + 1])
        Eo, A = orc.field([x[sl], y[sl], z[sl]], with_magnitude=True)
        check_field(E[:, sl], Eo, A)
    # the batch again in the shape it chose, in a fresh context: bit for bit
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        g.gccd_set_launch(ctx, tpt, chunks)
        g.gccd_set_tile(ctx, tile)
        g.gccd_load_events(ctx, off, *gpu(x, y, z))
        assert np.array_equal(E, g.gccd_field(ctx, len(x)).cpu().numpy())
    finally:
        g.gccd_destroy(ctx)


def check_field(E, Eo, A):
    """Both criteria of the Eq. (6) field tests: 1e-5 of the sum of term
    magnitudes per carrier, and 1e-5 of the rms field normwise."""
    d = np.linalg.norm(E - Eo, axis=0)
    ok = A > 0
    rms = math.sqrt(float(np.mean(np.sum(Eo**2, axis=0))))
    assert np.max(d[ok] / A[ok]) <= 1e-5
    assert np.max(d) <= 1e-5 * rms


@pytest.mark.parametrize("n", [1000, 5003])
def test_every_tile_size(g, W, orc, n):
    """64-, 128- and 256-source tiles (and the automatic choice) against the
    oracle: every hole judged."""
    w = W.single_cloud(n, seed=21, depth_um=200.0)
    Eo, A = orc.field([w.x, w.y, w.z], with_magnitude=True)
    for tile in (64, 128, 256, 0):
        ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE)))
        try:
            g.gccd_set_tile(ctx, tile)
            g.gccd_load(ctx, *gpu(w.x, w.y, w.z))
            used = g.gccd_stats(ctx)["tile_sources"]
            E = g.gccd_field(ctx, n).cpu().numpy()
        finally:
            g.gccd_destroy(ctx)
        d = np.linalg.norm(E - Eo, axis=0)
        rms = math.sqrt(float(np.mean(np.sum(Eo**2, axis=0))))
        print(f"[tile] n={n} tile {tile} (used {used}): max|dE|/A = {np.max(d / A):.3e}, "
              f"max|dE|/rms|E| = {np.max(d) / rms:.3e}", flush=True)
        assert used == (tile or (64 if n == 1000 else used))
        check_field(E, Eo, A)


def test_automatic_tile_choice(g, W):
    """64-source tiles for a 1000-hole cloud (its items fit one round of
    workgroups), 256 for 1e5 holes; other shapes and precisions keep 256."""
    cases = [(1000, 0, 0, 64), (100000, 0, 0, 256), (1000, 2, 0, 256), (1000, 0, 4, 256)]
    for n, tpt, prec, want in cases:
        w = W.single_cloud(n, seed=22)
        ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE)))
        try:
            g.gccd_set_launch(ctx, tpt, 0)
            g.gccd_set_precision(ctx, prec)
            g.gccd_load(ctx, *gpu(w.x, w.y, w.z))
            assert g.gccd_stats(ctx)["tile_sources"] == want, (n, tpt, prec)
            if prec:
                g.gccd_set_tile(ctx, 64)  # accepted, not used by that precision
                assert g.gccd_stats(ctx)["tile_sources"] == 256
        finally:
            g.gccd_destroy(ctx)
    ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE)))
    try:
        for bad in (-1, 32, 100, 512):
            with pytest.raises(RuntimeError):
                g.gccd_set_tile(ctx, bad)
    finally:
        g.gccd_destroy(ctx)


def test_autotune_without_repulsion_keeps_shape(g, W):
    ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE, coulomb=0)))
    try:
        g.gccd_set_launch(ctx, 2, 8)
        g.gccd_load(ctx, *gpu(np.zeros(4), np.zeros(4), np.full(4, 5.0)))
        tpt, chunks, ms = g.gccd_autotune(ctx)
        assert (tpt, chunks) == (2, 8) and ms < 0
    finally:
        g.gccd_destroy(ctx)
