"""The three ways gccd_run issues the steps of the exact path -- one
workgroup per work item (grid), a persistent launch over a work queue in
device memory (queue), and the queue launch captured once per 32-step
stretch as a HIP graph and replayed (graph) -- run the same kernels on the
same items, so every stretch must agree bit for bit.

Each gccd_run(32) call below is one graph replay; between replays the test
does eager work of its own (a field call, an image, position read-backs and
synchronisations), and every replay's result is compared with the grid
schedule's.  The loads collect holes as they go, so the work items are
rebuilt in place between replays.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SCHEDULES = ("grid", "queue", "graph")


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


def stretches(g, d, x, y, z, schedule, offsets=None, n_stretch=6, timing=False):
    n = len(x)
    ctx = g.gccd_init(g.Params.from_device(d))
    out = []
    try:
        g.gccd_set_schedule(ctx, schedule)
        g.gccd_set_timing(ctx, timing)
        if offsets is None:
            g.gccd_load(ctx, *gpu(x, y, z))
        else:
            g.gccd_load_events(ctx, offsets, *gpu(x, y, z))
        for k in range(n_stretch):
            done, na = g.gccd_run(ctx, 10.0, 32)
            pos, cs = g.gccd_positions(ctx, n)
            E = g.gccd_field(ctx, n)                      # eager work between replays
            if offsets is None:
                counts, nout = g.gccd_image(ctx, 0.0, 0.0, 15.0, 64, 64)
                img = counts.cpu().numpy().copy()
            else:
                img = None
            out.append((pos.cpu().numpy().copy(), cs.cpu().numpy().copy(),
                        E.cpu().numpy().copy(), img, done, na))
            if na == 0:
                break
        st = g.gccd_stats(ctx)
    finally:
        g.gccd_destroy(ctx)
    return out, st


def compare(runs, label):
    ref = runs["grid"][0]
    for s in ("queue", "graph"):
        got = runs[s][0]
        assert len(got) == len(ref), (label, s)
        for k, (a, b) in enumerate(zip(ref, got)):
            assert a[4] == b[4] and a[5] == b[5], (label, s, k)
            assert np.array_equal(a[0], b[0]), (label, s, k, "positions")
            assert np.array_equal(a[1], b[1]), (label, s, k, "collection steps")
            assert np.array_equal(a[2], b[2]), (label, s, k, "field")
            if a[3] is not None:
                assert np.array_equal(a[3], b[3]), (label, s, k, "image")


def test_single_cloud_schedules_agree(g, W):
    w = W.single_cloud(3000, seed=7, depth_um=30.0)
    d = dict(W.DEVICE, event=7)
    runs = {s: stretches(g, d, w.x, w.y, w.z, s) for s in SCHEDULES}
    compare(runs, "cloud")
    st = runs["graph"][1]
    calls = len(runs["graph"][0])   # every call started with holes travelling: one replay each
    print(f"[schedule] cloud n=3000: {calls} stretches, graph replays "
          f"{st['graph_replays']}, usable {st['graph_usable']}", flush=True)
    assert st["schedule"] == 2 and st["graph_usable"] == 1
    assert st["graph_replays"] == calls >= 3
    assert runs["grid"][1]["graph_replays"] == 0 and runs["queue"][1]["graph_replays"] == 0


def test_batch_schedules_agree(g, W):
    events = W.batch_of_clouds(48, seed=3)
    off = np.concatenate([[0], np.cumsum([len(e[0]) for e in events])]).astype(np.int64)
    x = np.concatenate([e[0] for e in events])
    y = np.concatenate([e[1] for e in events])
    z = np.concatenate([e[2] for e in events])
    d = dict(W.DEVICE, event=11)
    runs = {s: stretches(g, d, x, y, z, s, offsets=list(off), n_stretch=5) for s in SCHEDULES}
    compare(runs, "batch")
    st = runs["graph"][1]
    print(f"[schedule] batch of 48: graph replays {st['graph_replays']}, usable "
          f"{st['graph_usable']}", flush=True)
    assert st["graph_usable"] == 1 and st["graph_replays"] >= 3


def test_graph_timing(g, W):
    """With per-launch timing on, the graph schedule issues its steps one by
    one (events cannot be read back from replays): one field time per step,
    no replay, the same results."""
    w = W.single_cloud(3000, seed=8, depth_um=200.0)
    d = dict(W.DEVICE, event=8)
    runs = {s: stretches(g, d, w.x, w.y, w.z, s, n_stretch=3, timing=True)
            for s in ("grid", "graph")}
    for s in ("grid", "graph"):
        st = runs[s][1]
        assert st["field_launches"] == 96 and st["field_ms"] > 0, (s, st)
    assert runs["graph"][1]["graph_replays"] == 0
    for a, b in zip(runs["grid"][0], runs["graph"][0]):
        assert np.array_equal(a[0], b[0])


def test_schedule_validation(g, W):
    ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE)))
    try:
        assert g.lib.gccd_set_schedule(ctx, 3) == g.GCCD_E_INVALID
        assert g.lib.gccd_set_schedule(ctx, -1) == g.GCCD_E_INVALID
        assert g.gccd_stats(ctx)["schedule"] == 2          # the default: graph
    finally:
        g.gccd_destroy(ctx)


def test_graph_recaptured_after_closure_buffers_change(g, W):
    """Exact steps (captured), closure steps (which reallocate the work-item
    and partial-sum buffers the graph names), exact steps again: the graph
    is captured anew and every stretch matches the grid schedule."""
    import os
    from paper_2203_11043_amd import closure_eval
    if not os.path.exists(closure_eval.WEIGHTS):
        pytest.skip("no trained closure weights in the package")
    wts = closure_eval.load_weights()
    w = W.single_cloud(6000, seed=9, depth_um=250.0)
    d = dict(W.DEVICE, event=9)
    res = {}
    for s in ("grid", "graph"):
        ctx = g.gccd_init(g.Params.from_device(d))
        snaps = []
        try:
            g.gccd_set_schedule(ctx, s)
            # two source chunks: the closure's 7 groups and 144 items outgrow the
            # exact path's buffers, which are reallocated under the graph
            g.gccd_set_launch(ctx, 1, 2)
            g.gccd_load(ctx, *gpu(w.x, w.y, w.z))
            g.gccd_run(ctx, 10.0, 32)
            snaps.append(g.gccd_positions(ctx, w.n)[0].cpu().numpy().copy())
            g.gccd_set_closure(ctx, wts, 0)
            g.gccd_run(ctx, 10.0, 32)
            snaps.append(g.gccd_positions(ctx, w.n)[0].cpu().numpy().copy())
            g.gccd_set_closure(ctx, None, 0)
            for _ in range(2):
                g.gccd_run(ctx, 10.0, 32)
                snaps.append(g.gccd_positions(ctx, w.n)[0].cpu().numpy().copy())
            st = g.gccd_stats(ctx)
        finally:
            g.gccd_destroy(ctx)
        res[s] = (snaps, st)
    for k, (a, b) in enumerate(zip(res["grid"][0], res["graph"][0])):
        assert np.array_equal(a, b), k
    st = res["graph"][1]
    assert st["closure_steps"] == 32 and st["graph_replays"] == 3 and st["graph_usable"] == 1


def test_full_size_schedules_agree(g, W):
    """The 1e5-hole cloud of the benchmark, two 32-step stretches: the three
    schedules agree bit for bit at the size they are timed on."""
    w = W.single_cloud(100000, seed=1)
    d = dict(W.DEVICE)
    runs = {s: stretches(g, d, w.x, w.y, w.z, s, n_stretch=2) for s in SCHEDULES}
    compare(runs, "cloud 1e5")
    st = runs["graph"][1]
    print(f"[schedule] cloud n=100000: graph replays {st['graph_replays']}, usable "
          f"{st['graph_usable']}", flush=True)
    assert st["graph_usable"] == 1 and st["graph_replays"] == 2


def test_full_batch_schedules_agree(g, W):
    """The 4096-cloud batch (1.8e7 holes) under the three schedules, two
    32-step stretches: the graph is captured at this size (the per-step sort
    issues no memory-set command) and replayed, and every stretch is bit
    for bit the grid schedule's."""
    events = W.batch_of_clouds(4096, seed=1)
    off = np.concatenate([[0], np.cumsum([len(e[0]) for e in events])]).astype(np.int64)
    x = np.concatenate([e[0] for e in events])
    y = np.concatenate([e[1] for e in events])
    z = np.concatenate([e[2] for e in events])
    d = dict(W.DEVICE)
    runs = {s: stretches(g, d, x, y, z, s, offsets=list(off), n_stretch=2) for s in SCHEDULES}
    compare(runs, "batch 4096")
    st = runs["graph"][1]
    print(f"[schedule] batch of 4096 ({len(x)} holes): graph replays {st['graph_replays']}, "
          f"usable {st['graph_usable']}", flush=True)
    assert st["graph_usable"] == 1 and st["graph_replays"] == 2
