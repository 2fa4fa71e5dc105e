"""Loads above 2048 holes whose steps have less pair work than the
pipelined list needs (5e9 pairs) keep a serial list: after each step the
list is sorted again, on the critical path.  There the step kernel's
workgroups sort their 256 slots' new keys into runs, the sort only merges
those runs, and (every hole a source) one launch gathers the positions and
boxes and writes each event's travelling count, where a fresh load sorts
the keys from scratch and counts and gathers separately.  The keys are
unique, so both must give the same list.

As in the small-load list test, the list a run leaves is compared with the
one a fresh load of the same positions builds, through gccd_field, whose
rounding depends on the slot order, the counts and the tile boxes: the two
fields must agree bit for bit."""
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


def load(g, ctx, offsets, x, y, z):
    if offsets is None:
        g.gccd_load(ctx, *gpu(x, y, z))
    else:
        g.gccd_load_events(ctx, offsets, *gpu(x, y, z))


def run_then_compare(g, d, x, y, z, offsets=None, steps=0, until_active=None):
    n = len(x)
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        load(g, ctx, offsets, x, y, z)
        done, na = 0, n
        if steps:
            done, na = g.gccd_run(ctx, 10.0, steps)
        while until_active is not None and na > until_active and done < 3000:
            k, na = g.gccd_run(ctx, 10.0, 8)
            done += k
        pos, cs = g.gccd_positions(ctx, n)
        pos, cs = pos.cpu().numpy(), cs.cpu().numpy()
        E1 = g.gccd_field(ctx, n).cpu().numpy()
    finally:
        g.gccd_destroy(ctx)
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        load(g, ctx, offsets, pos[0], pos[1], pos[2])
        _, cs2 = g.gccd_positions(ctx, n)
        E2 = g.gccd_field(ctx, n).cpu().numpy()
    finally:
        g.gccd_destroy(ctx)
    assert np.array_equal(cs >= 0, cs2.cpu().numpy() >= 0)
    return E1, E2, done, int(np.sum(cs < 0))


@pytest.mark.parametrize("n,sources", [(3000, 1), (10000, 1), (3000, 0)])
def test_single_cloud_serial_list(g, W, n, sources):
    x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, 20.0), 93, stream=n)
    d = dict(W.DEVICE, collected_are_sources=sources)
    E1, E2, done, na = run_then_compare(g, d, x, y, z, until_active=n // 2)
    print(f"[serial list] n={n} sources={'all' if sources else 'travelling'}: {done} steps, "
          f"{na} travelling", flush=True)
    assert 0 < na <= n // 2
    assert np.array_equal(E1, E2)


def test_events_serial_list(g, W):
    """Five events of 1 to 2500 holes (5008 in all) at different depths:
    per-event counts written by the tile that holds each event's first
    collected key, or by its last tile."""
    sizes = [1, 2500, 7, 1800, 700]
    depths = [12.0, 20.0, 300.0, 25.0, 15.0]
    xs, ys, zs, off = [], [], [], [0]
    for e, (n, dz) in enumerate(zip(sizes, depths)):
        x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, dz), 94, stream=e)
        xs.append(x)
        ys.append(y)
        zs.append(z)
        off.append(off[-1] + n)
    x, y, z = np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)
    E1, E2, done, na = run_then_compare(g, dict(W.DEVICE), x, y, z, offsets=off, steps=150)
    print(f"[serial list] 5 events, {off[-1]} holes: {done} steps, {na} travelling", flush=True)
    assert 0 < na < off[-1]
    assert np.array_equal(E1, E2)
