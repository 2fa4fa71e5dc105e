"""The size limits of a load, at the limit and just past it.

  * rejected: no holes, more than 2^27 holes in one event, an event count
    times the largest event beyond the 27 bits of key payload;
  * the key-space boundary: 2^12 events with the largest of 2^15 holes fill
    every bit of the 64-bit list key (12 event bits, the collected bit, 36
    curve bits, 15 local bits); the large event's field matches the oracle and
    the one-hole events feel nothing;
  * the largest single event, 2^27 holes, without repulsion (an O(N) step):
    every hole's trajectory matches the oracle's over 3 steps (same Philox
    words; device-libm rounding only) and the charge is conserved.
"""
import ctypes

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


def test_rejected_sizes(g, W):
    ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE)))
    try:
        L = g.lib
        assert L.gccd_load(ctx, 0, None, None, None) == g.GCCD_E_INVALID
        assert L.gccd_load(ctx, (1 << 27) + 1, None, None, None) == g.GCCD_E_INVALID
        # 2^13 events with one of 2^15 holes: 13 + 15 > 27 key bits
        n_ev = 1 << 13
        off = (ctypes.c_int64 * (n_ev + 1))(*([0] + [k + (1 << 15) for k in range(1, n_ev + 1)]))
        x, y, z = gpu(np.zeros(4), np.zeros(4), np.zeros(4))
        st = L.gccd_load_events(ctx, n_ev, off, x.data_ptr(), y.data_ptr(), z.data_ptr())
        assert st == g.GCCD_E_INVALID
        assert b"2^27" in L.gccd_last_error(ctx)
    finally:
        g.gccd_destroy(ctx)


def test_key_space_boundary(g, W, orc):
    n_ev, big = 1 << 12, 1 << 15
    sizes = [big] + [1] * (n_ev - 1)
    rng = np.random.default_rng(31)
    bx, by, bz = W.gaussian_cloud(big, W.cloud_sigma(big), (480.0, 480.0, 200.0), 31, stream=5)
    x = np.concatenate([bx, rng.uniform(0, 960, n_ev - 1)])
    y = np.concatenate([by, rng.uniform(0, 960, n_ev - 1)])
    z = np.concatenate([bz, rng.uniform(1, 670, n_ev - 1)])
    off = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE)))
    try:
        g.gccd_load_events(ctx, off, *gpu(x, y, z))
        E = g.gccd_field(ctx, len(x)).cpu().numpy()
        g.gccd_run(ctx, 10.0, 3)
        st = g.gccd_stats(ctx)
    finally:
        g.gccd_destroy(ctx)
    assert st["n_events"] == n_ev and st["step"] == 3
    assert np.all(E[:, big:] == 0.0)                 # alone in their events
    idx = np.random.default_rng(2).choice(big, 256, replace=False)
    Eo, A = orc.field([bx[idx], by[idx], bz[idx]], [bx, by, bz], with_magnitude=True)
    err = np.max(np.linalg.norm(E[:, idx] - Eo, axis=0) / A)
    print(f"[limits] 4096 events, 64-bit keys: max|dE|/A = {err:.2e}", flush=True)
    assert err <= 1e-5


def test_largest_single_event_without_repulsion(g, W, orc):
    n = 1 << 27
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 960.0, n)
    y = rng.uniform(0.0, 960.0, n)
    z = rng.uniform(1.0, 674.0, n)
    d = dict(W.DEVICE, coulomb=0, event=3)
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        g.gccd_load(ctx, *gpu(x, y, z))
        done, na = g.gccd_run(ctx, 10.0, 3)
        pos, cs = g.gccd_positions(ctx, n)
        counts, nout = g.gccd_image(ctx, 0.0, 0.0, 15.0, 64, 64)
        pos = pos.cpu().numpy()
        collected = int(counts.sum().item()) + int(nout.item())
    finally:
        g.gccd_destroy(ctx)
    assert done == 3 and collected + na == n
    o = orc.Device()
    for k, v in d.items():
        setattr(o, k, v)
    st = orc.State(o, x, y, z)
    del x, y, z
    st.run(10.0, 3)
    diff = max(float(np.max(np.abs(pos[0] - st.x))), float(np.max(np.abs(pos[1] - st.y))),
               float(np.max(np.abs(pos[2] - st.z))))
    print(f"[limits] 2^27 holes, 3 steps without repulsion: max |dr| = {diff:.2e} um", flush=True)
    assert diff < 1e-10 and st.n_active == na
