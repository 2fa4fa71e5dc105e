"""Precision modes of the Eq. (6) kernel against the FP64 oracle.

The FP64 mode runs the same work items, tiles, source dealing, chunk
partials and FP64 reduction as the fast path, with every pair in FP64; it
must agree with the oracle to 1e-12 of A_j = K sum_i |r_ij|/(r^2+eps^2)^{3/2}
(the partial sums travel as FP32 hi/lo pairs, exact to about 2^-48).  The
default and compensated modes carry the proven 1e-5 A bound.  The others
(no close-pair recomputation, one origin per event, absolute FP32
coordinates as the paper stores them) have no such bound: the study records
their errors and times beside the rest, for every workload.

Set PRECISION_STUDY_OUT to a file path to have the table written there.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5
FP64_TOL = 1e-12
MODES = ["default", "block", "event", "absolute", "compensated", "fp64"]


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


def oracle_device(orc, d, event=0):
    o = orc.Device()
    for k, v in d.items():
        setattr(o, k, v)
    o.event = event
    return o


def errors(E, Eo, A):
    """max |dE|/A, max |dE|/rms|E|, p99 of |dE|/|E| over carriers with
    |E| > 1e-3 rms."""
    d = np.linalg.norm(E - Eo, axis=0)
    mag = np.linalg.norm(Eo, axis=0)
    rms = math.sqrt(float(np.mean(mag**2)))
    ok = A > 0
    big = mag > 1e-3 * rms
    return (float(np.max(d[ok] / A[ok])) if ok.any() else 0.0,
            float(np.max(d) / rms) if rms > 0 else 0.0,
            float(np.percentile(d[big] / mag[big], 99)) if big.any() else 0.0)


def field_with_mode(g, d, x, y, z, mode, offsets=None, tpt=0, chunks=0, time_steps=0):
    ctx = g.gccd_init(g.Params.from_device(d))
    try:
        g.gccd_set_launch(ctx, tpt, chunks)
        g.gccd_set_precision(ctx, mode)
        if offsets is None:
            g.gccd_load(ctx, *gpu(x, y, z))
        else:
            g.gccd_load_events(ctx, offsets, *gpu(x, y, z))
        E = g.gccd_field(ctx, len(x)).cpu().numpy()
        ms = None
        if time_steps:
            # untimed warm-up: the first launches after a load run at a lower clock
            g.gccd_run(ctx, 10.0, 3 if mode == "fp64" else 10)
            g.gccd_set_timing(ctx, True)
            g.gccd_run(ctx, 10.0, time_steps)
            st = g.gccd_stats(ctx)
            ms = st["field_ms"] / max(st["field_launches"], 1)
        st = g.gccd_stats(ctx)
    finally:
        g.gccd_destroy(ctx)
    return E, st, ms


# ------------------------------------------------------------- FP64 mode

@pytest.mark.parametrize("tpt,chunks", [(1, 1), (2, 5), (4, 32), (1, 64), (0, 0)])
def test_fp64_mode_matches_oracle(g, W, orc, tpt, chunks):
    """Ragged 5003-hole cloud over launch shapes: the FP64 mode reproduces
    the oracle to rounding, which checks the list, tiles, chunking and the
    reduction independently of the FP32 pair arithmetic.  At most 32 chunks
    (each takes two partial groups) and at most one per 256-source tile."""
    w = W.single_cloud(5003, seed=4, depth_um=222.0)
    d = dict(W.DEVICE)
    E, st, _ = field_with_mode(g, d, w.x, w.y, w.z, "fp64", tpt=tpt, chunks=chunks)
    Eo, A = orc.field([w.x, w.y, w.z], with_magnitude=True)
    ea, er, _ = errors(E, Eo, A)
    print(f"[fp64] n=5003 tpt={st['targets_per_thread']} chunks={st['source_chunks']}: "
          f"max|dE|/A = {ea:.2e}", flush=True)
    assert ea <= FP64_TOL
    if chunks:   # FP64 takes at most 32 chunks, and no event more chunks than tiles
        assert st["source_chunks"] == min(chunks, 32, (5003 + 255) // 256)
    assert st["tile_sources"] == 256


def test_fp64_mode_track_and_batch(g, W, orc):
    """The mirrored muon track (sampled targets) and a batch of uneven events."""
    w = W.muon_track(seed=1)
    d = dict(W.DEVICE)
    E, _, _ = field_with_mode(g, d, w.x, w.y, w.z, "fp64")
    o = orc.State(oracle_device(orc, d), w.x, w.y, w.z)
    idx = np.random.default_rng(9).choice(w.n, 256, replace=False)
    Eo, A = orc.field([o.x[idx], o.y[idx], o.z[idx]], [o.x, o.y, o.z], with_magnitude=True)
    assert errors(E[:, idx], Eo, A)[0] <= FP64_TOL

    sizes = [200, 3000, 257, 1, 1024, 50]
    xs, ys, zs, off = [], [], [], [0]
    for e, n in enumerate(sizes):
        x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, 20.0 + 90 * e), 5,
                                   stream=700 + e)
        xs.append(x)
        ys.append(y)
        zs.append(z)
        off.append(off[-1] + n)
    x, y, z = np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)
    E, st, _ = field_with_mode(g, d, x, y, z, "fp64", offsets=off)
    assert st["n_events"] == len(sizes)
    for e in range(len(sizes)):
        sl = slice(off[e], off[e + 1])
        Eo, A = orc.field([x[sl], y[sl], z[sl]], with_magnitude=True)
        assert errors(E[:, sl], Eo, A)[0] <= FP64_TOL, e


def test_precision_mode_validation(g, W):
    ctx = g.gccd_init(g.Params.from_device(dict(W.DEVICE)))
    try:
        for bad in (-1, 6, 99):
            with pytest.raises(g.GccdError) as e:
                g.gccd_set_precision(ctx, bad)
            assert e.value.status == g.GCCD_E_INVALID
        g.gccd_set_precision(ctx, "fp64")
        g.gccd_load(ctx, *gpu(np.zeros(3), np.zeros(3), np.array([10.0, 11.0, 12.0])))
        g.gccd_set_precision(ctx, "default")   # re-splits the loaded state
        E = g.gccd_field(ctx, 3).cpu().numpy()
        assert np.all(np.isfinite(E))
    finally:
        g.gccd_destroy(ctx)


# ------------------------------------------------------------- the study

def study_workloads(W):
    """(name, workload, sampled targets or 0 for all) of every single-event
    workload; the batch is added in the test."""
    return [("cloud n=1000", W.x_ray_cloud(seed=1), 0),
            ("cloud n=10000", W.single_cloud(10000, seed=1), 0),
            ("cloud n=100000", W.single_cloud(100000, seed=1), 512),
            ("cloud n=300000", W.single_cloud(300000, seed=1), 512),
            ("muon track n=62354", W.muon_track(seed=1), 512)]


def test_precision_study(g, W, orc):
    d = dict(W.DEVICE)
    rows = []

    def add(name, E_by_mode, Eo, A, ms_by_mode):
        for m in MODES:
            ea, er, p99 = errors(E_by_mode[m], Eo, A)
            rows.append((name, m, ea, er, p99, ms_by_mode[m]))

    for name, w, sample in study_workloads(W):
        o = orc.State(oracle_device(orc, d), w.x, w.y, w.z)   # load-time mirror
        if sample:
            idx = np.random.default_rng(w.n).choice(w.n, sample, replace=False)
            Eo, A = orc.field([o.x[idx], o.y[idx], o.z[idx]], [o.x, o.y, o.z],
                              with_magnitude=True)
        else:
            idx = slice(None)
            Eo, A = orc.field([o.x, o.y, o.z], with_magnitude=True)
        Es, ms = {}, {}
        for m in MODES:
            E, _, t = field_with_mode(g, d, w.x, w.y, w.z, m, time_steps=5)
            Es[m], ms[m] = E[:, idx], t
        add(name, Es, Eo, A, ms)

    # 4096-event batch: 32 sampled events, all their targets
    events = W.batch_of_clouds(4096, seed=1)
    off = np.concatenate([[0], np.cumsum([len(e[0]) for e in events])]).astype(np.int64)
    x = np.concatenate([e[0] for e in events])
    y = np.concatenate([e[1] for e in events])
    z = np.concatenate([e[2] for e in events])
    pick = np.sort(np.random.default_rng(4096).choice(len(events), 32, replace=False))
    parts = []
    for e in pick:
        sl = slice(int(off[e]), int(off[e + 1]))
        o = orc.State(oracle_device(orc, d, e), x[sl], y[sl], z[sl])
        parts.append((sl, *orc.field([o.x, o.y, o.z], with_magnitude=True)))
    Eo = np.concatenate([p[1] for p in parts], axis=1)
    A = np.concatenate([p[2] for p in parts])
    Es, ms = {}, {}
    for m in MODES:
        E, _, t = field_with_mode(g, d, x, y, z, m, offsets=list(off), time_steps=5)
        Es[m], ms[m] = np.concatenate([E[:, p[0]] for p in parts], axis=1), t
    add("batch 4096 events (32 sampled)", Es, Eo, A, ms)

    lines = ["| workload | mode | max abs(dE)/A | max abs(dE)/rms abs(E) | p99 abs(dE)/abs(E) "
             "| ms per field launch |", "|---|---|---|---|---|---|"]
    for name, m, ea, er, p99, t in rows:
        lines.append(f"| {name} | {m} | {ea:.2e} | {er:.2e} | {p99:.2e} | {t:.3f} |")

    # the observable: second moments of the collected clouds after full runs
    lines += ["", "| run to completion | mode | steps | var_x rel. to oracle | var_y rel. to oracle |",
              "|---|---|---|---|---|"]
    for name, w in (("cloud n=1000, depth 300 um", W.x_ray_cloud(seed=1)),
                    ("cloud n=10000, depth 30 um", W.single_cloud(10000, seed=2, depth_um=30.0))):
        o = orc.State(oracle_device(orc, d), w.x, w.y, w.z)
        o.run(10.0, 5000)
        assert o.n_active == 0
        for m in MODES:
            ctx = g.gccd_init(g.Params.from_device(d))
            try:
                g.gccd_set_precision(ctx, m)
                g.gccd_load(ctx, *gpu(w.x, w.y, w.z))
                done, na = g.gccd_run(ctx, 10.0, 5000)
                pos, _ = g.gccd_positions(ctx, w.n)
                pos = pos.cpu().numpy()
            finally:
                g.gccd_destroy(ctx)
            assert na == 0
            rx = np.var(pos[0]) / np.var(o.x) - 1.0
            ry = np.var(pos[1]) / np.var(o.y) - 1.0
            lines.append(f"| {name} | {m} | {done} (oracle {o.step}) | {rx:+.2e} | {ry:+.2e} |")
            if m in ("default", "compensated", "fp64"):
                assert abs(rx) < 5e-3 and abs(ry) < 5e-3, (name, m, rx, ry)
    table = "\n".join(lines)
    print("\n" + table, flush=True)
    path = os.environ.get("PRECISION_STUDY_OUT")
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            f.write(table + "\n")

    for name, m, ea, er, p99, t in rows:
        if m in ("default", "compensated"):
            assert ea <= FIELD_TOL, (name, m, ea)
        if m == "fp64":
            assert ea <= FP64_TOL, (name, m, ea)
