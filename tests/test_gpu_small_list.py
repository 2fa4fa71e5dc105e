"""Loads of at most 2048 holes rebuild the sorted carrier list inside the
step kernel: each workgroup sorts its 256 slots' new keys into a run, and
the last one merges the runs in LDS (1024- and 2048-key merges below), finds
each event's travelling holes and gathers the positions and boxes of the
source tiles, where larger loads launch the sort, the count and the gather
separately.  The keys are unique, so both must give the same list.

After runs that collect part of the holes, the list the step kernel left is
compared with the one a fresh load of the same positions builds by the
separate launches, through gccd_field: it sums each target over the
list's source tiles in slot order, with origins and near/far choices taken
from the tile boxes and the travelling counts, so any difference in order,
counts or boxes changes its rounding.  The two fields must agree bit for
bit (every load here has at most 2048 holes, so both contexts split the
work alike)."""
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


def run_then_compare(g, d, x, y, z, offsets=None, steps=None, until_active=None):
    n = len(x)
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        load(g, ctx, offsets, x, y, z)
        done, na = 0, n
        if steps is not None:
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
    # the fresh load collects exactly the holes the run collected
    assert np.array_equal(cs >= 0, cs2.cpu().numpy() >= 0)
    return E1, E2, done, int(np.sum(cs < 0))


@pytest.mark.parametrize("n,sources", [(2000, 1), (2048, 1), (1500, 0), (700, 1), (1, 1)])
def test_single_cloud_list(g, W, n, sources):
    x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, 20.0), 91, stream=n)
    d = dict(W.DEVICE, collected_are_sources=sources)
    E1, E2, done, na = run_then_compare(g, d, x, y, z, until_active=max(n // 2, 0),
                                        steps=None if n > 1 else 5)
    print(f"[small list] n={n} sources={'all' if sources else 'travelling'}: {done} steps, "
          f"{na} travelling", flush=True)
    assert np.array_equal(E1, E2)


def test_events_list(g, W):
    """Six events of 1 to 900 holes at different depths, some collected,
    some not: per-event counts and tiles."""
    sizes = [300, 7, 1, 900, 250, 400]
    depths = [15.0, 300.0, 12.0, 25.0, 400.0, 18.0]
    xs, ys, zs, off = [], [], [], [0]
    for e, (n, dz) in enumerate(zip(sizes, depths)):
        x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, dz), 92, stream=e)
        xs.append(x)
        ys.append(y)
        zs.append(z)
        off.append(off[-1] + n)
    x, y, z = np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)
    E1, E2, done, na = run_then_compare(g, dict(W.DEVICE), x, y, z, offsets=off, steps=150)
    print(f"[small list] 6 events, {off[-1]} holes: {done} steps, {na} travelling", flush=True)
    assert 0 < na < off[-1]
    assert np.array_equal(E1, E2)
