"""GPU (HIP, gfx950) path against the FP64 oracle, through the C ABI.

Tolerances (derived from the arithmetic, see the design notes):
  * Eq. (6) field, two criteria, both asserted:
      - normwise: max_j |dE_j| / rms_k |E_k| <= 1e-5 (the per-step field
        criterion; the per-carrier relative error |dE|/|E| is ill-conditioned
        where the terms cancel, at the centre of a cloud);
      - per carrier: |dE_j| <= 1e-5 A_j, A_j = K sum_i |r_ij| /
        (r_ij^2 + eps^2)^{3/2} the sum of term magnitudes (the scale that
        bounds the rounding error of any ordering of the sum).
  * Coulomb-off runs: same Philox words on both sides, so positions agree to
    device-libm rounding (1e-10 um) and collection steps exactly.
  * Coulomb-on runs: trajectories drift apart through FP32 rounding, so cloud
    second moments are compared (0.5 %), not positions.
  * Images from identical positions: bit-exact.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5


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


def dev_params(g, W, **kw):
    d = dict(W.DEVICE)
    d.update(kw)
    return g.Params.from_device(d), d


def oracle_device(orc, d):
    o = orc.Device()
    for k, v in d.items():
        setattr(o, k, v)
    return o


def gpu_tensors(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def field_errors(E_gpu, E_ora, A):
    d = np.linalg.norm(E_gpu - E_ora, axis=0)
    rms = math.sqrt(float(np.mean(np.sum(E_ora**2, axis=0))))
    return float(np.max(d / A)), float(np.max(d) / rms)


def gpu_field(g, params, x, y, z, tpt=0, chunks=0):
    ctx = g.gccd_init(params)
    try:
        g.gccd_set_launch(ctx, tpt, chunks)
        g.gccd_load(ctx, *gpu_tensors(x, y, z))
        E = g.gccd_field(ctx, len(x)).cpu().numpy()
        st = g.gccd_stats(ctx)
    finally:
        g.gccd_destroy(ctx)
    return E, st


def report(tag, e_abs, e_rms):
    print(f"[field] {tag}: max|dE|/A = {e_abs:.3e}, max|dE|/rms|E| = {e_rms:.3e}", flush=True)


# ---------------------------------------------------------------- Eq. (6)

def test_field_cloud_1000_all_targets(g, W, orc):
    w = W.x_ray_cloud(seed=1)
    p, d = dev_params(g, W)
    E, st = gpu_field(g, p, w.x, w.y, w.z)
    Eo, A = orc.field([w.x, w.y, w.z], with_magnitude=True)
    ea, er = field_errors(E, Eo, A)
    report("cloud n=1000", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL


@pytest.mark.parametrize("tpt,chunks", [(1, 1), (2, 1), (4, 1), (1, 3), (2, 8), (4, 32), (1, 64), (0, 0)])
def test_field_ragged_launch_shapes(g, W, orc, tpt, chunks):
    """5003 carriers: several LDS tiles, a ragged last tile and target block,
    and source chunks of unequal length."""
    w = W.single_cloud(5003, seed=4, depth_um=222.0)
    p, d = dev_params(g, W)
    E, st = gpu_field(g, p, w.x, w.y, w.z, tpt, chunks)
    Eo, A = orc.field([w.x, w.y, w.z], with_magnitude=True)
    ea, er = field_errors(E, Eo, A)
    report(f"cloud n=5003 tpt={st['targets_per_thread']} chunks={st['source_chunks']}", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL
    if tpt:   # a fixed chunk count is capped at the event's tiles (of the size in force)
        unit = st["tile_sources"]
        assert st["targets_per_thread"] == tpt
        assert unit in ((64, 128, 256) if tpt == 1 else (256,))
        assert st["source_chunks"] == min(chunks, (5003 + unit - 1) // unit)


@pytest.mark.parametrize("n", [30000, 100000, 300000])
def test_field_full_size_sampled(g, W, orc, n):
    """The single-cloud sizes at the launch shape the benchmark uses; the
    oracle evaluates 256 sampled targets against all n sources."""
    w = W.single_cloud(n, seed=1)
    p, d = dev_params(g, W)
    E, st = gpu_field(g, p, w.x, w.y, w.z)
    idx = np.random.default_rng(n).choice(n, 256, replace=False)
    Eo, A = orc.field([w.x[idx], w.y[idx], w.z[idx]], [w.x, w.y, w.z], with_magnitude=True)
    ea, er = field_errors(E[:, idx], Eo, A)
    report(f"cloud n={n} (256 sampled) tpt={st['targets_per_thread']} "
           f"chunks={st['source_chunks']}", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL


def test_field_muon_track_sampled(g, W, orc):
    """A straight track through the whole thickness: some holes start beyond
    the back surface and are mirrored at load, on both sides."""
    w = W.muon_track(seed=1)
    p, d = dev_params(g, W)
    E, st = gpu_field(g, p, w.x, w.y, w.z)
    o = orc.State(oracle_device(orc, d), w.x, w.y, w.z)     # load-time mirror
    assert np.any(w.z > d["thickness_um"])
    idx = np.random.default_rng(9).choice(w.n, 256, replace=False)
    Eo, A = orc.field([o.x[idx], o.y[idx], o.z[idx]], [o.x, o.y, o.z], with_magnitude=True)
    ea, er = field_errors(E[:, idx], Eo, A)
    report(f"track n={w.n} (256 sampled)", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL


def test_field_collected_not_sources(g, W, orc):
    """collected_are_sources = 0: holes loaded at or below the well neither
    move nor repel."""
    w = W.single_cloud(3000, seed=5, depth_um=1.0)   # part of the cloud is at z <= 0
    p, d = dev_params(g, W, collected_are_sources=0)
    E, st = gpu_field(g, p, w.x, w.y, w.z)
    act = w.z > 0.0
    assert 0 < act.sum() < w.n
    src = [w.x[act], w.y[act], w.z[act]]
    Eo, A = orc.field([w.x, w.y, w.z], src, with_magnitude=True)
    ea, er = field_errors(E[:, act], Eo[:, act], A[act])
    report("cloud n=3000, active sources only", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL


def test_field_far_from_origin_across_key_wrap(g, W, orc):
    """A cloud 60 mm from the coordinate origin, centred on a multiple of the
    1024 um period of the sort key's cell index in x and y: its holes get keys
    from both ends of the curve, and the pair offsets are formed relative to
    each workgroup's origin, so the field must not depend on where it sits."""
    n = 20000
    cx, cy = 60 * 1024.0 + 0.3, 2 * 1024.0 - 0.2
    x, y, z = W.gaussian_cloud(n, W.cloud_sigma(n), (cx, cy, 300.0), 41, stream=6)
    assert np.any(x < 60 * 1024.0) and np.any(x > 60 * 1024.0)
    p, d = dev_params(g, W)
    E, st = gpu_field(g, p, x, y, z)
    Eo, A = orc.field([x, y, z], with_magnitude=True)
    ea, er = field_errors(E, Eo, A)
    report(f"cloud n={n} at x={cx:.1f} um, y={cy:.1f} um", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL
    # the same holes near the origin: the same field to rounding
    E0, _ = gpu_field(g, p, x - cx + 480.0, y - cy + 480.0, z)
    Eo0, A0 = orc.field([x - cx + 480.0, y - cy + 480.0, z], with_magnitude=True)
    assert max(field_errors(E0, Eo0, A0)) <= FIELD_TOL
    assert np.max(np.linalg.norm(E - E0, axis=0) / A) <= 2 * FIELD_TOL


def test_field_coincident_holes(g, W, orc):
    """Every position held by three holes: a coincident pair's softened term
    is zero (Eq. (6) at r = 0), and the three copies feel the same field."""
    u = 1700
    x, y, z = W.gaussian_cloud(u, W.cloud_sigma(3 * u), (480.0, 480.0, 250.0), 43, stream=7)
    x, y, z = np.tile(x, 3), np.tile(y, 3), np.tile(z, 3)
    p, d = dev_params(g, W)
    E, st = gpu_field(g, p, x, y, z)
    Eo, A = orc.field([x, y, z], with_magnitude=True)
    ea, er = field_errors(E, Eo, A)
    report(f"cloud n={3 * u}, each position held by 3 holes", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL
    for k in (1, 2):
        assert np.max(np.linalg.norm(E[:, k * u:(k + 1) * u] - E[:, :u], axis=0)
                      / A[:u]) <= 2 * FIELD_TOL


def test_field_two_distant_clusters(g, W, orc):
    """Two clusters 150 um apart: almost every source tile lies far from the
    target block, so the expanded-square form carries nearly all pairs; the
    clusters' mutual field is close to that of two point charges."""
    n = 6000
    a = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, 200.0), 47, stream=8)
    b = W.gaussian_cloud(n, W.cloud_sigma(n), (480.0, 480.0, 350.0), 47, stream=9)
    x, y, z = (np.concatenate([a[i], b[i]]) for i in range(3))
    p, d = dev_params(g, W)
    E, st = gpu_field(g, p, x, y, z)
    Eo, A = orc.field([x, y, z], with_magnitude=True)
    ea, er = field_errors(E, Eo, A)
    report(f"two clusters of {n}, 150 um apart", ea, er)
    assert ea <= FIELD_TOL and er <= FIELD_TOL
    # each cluster's own field sums to zero; the other one, 150 um away, pushes
    # the lower cluster down and the upper one up, as a point charge would
    point = orc.coulomb_constant(d["eps_r"]) * n / 150.0**2
    assert abs(np.mean(Eo[2, :n]) + point) < 0.01 * point
    assert abs(np.mean(Eo[2, n:]) - point) < 0.01 * point
    assert np.mean(E[2, :n]) < 0.0 < np.mean(E[2, n:])


def test_field_degenerate_sizes(g, W):
    p, d = dev_params(g, W)
    E, _ = gpu_field(g, p, [1.0], [2.0], [3.0])
    assert np.all(E == 0.0)                       # the self term vanishes
    E, _ = gpu_field(g, p, [-0.5, 0.5], [0.0, 0.0], [300.0, 300.0])
    assert np.array_equal(E[:, 0], -E[:, 1])      # Newton's third law, exactly
    assert E[0, 1] > 0 and E[1, 1] == 0 and E[2, 1] == 0


# ---------------------------------------------------------------- the time step

def run_both(g, W, orc, w, steps, **kw):
    p, d = dev_params(g, W, **kw)
    ctx = g.gccd_init(p)
    try:
        g.gccd_load(ctx, *gpu_tensors(w.x, w.y, w.z))
        done, na = g.gccd_run(ctx, w.dt_ps, steps)
        pos, cs = g.gccd_positions(ctx, w.n)
        st = g.gccd_stats(ctx)
        pos, cs = pos.cpu().numpy(), cs.cpu().numpy()
    finally:
        g.gccd_destroy(ctx)
    o = orc.State(oracle_device(orc, d), w.x, w.y, w.z)
    odone, ona = o.run(w.dt_ps, steps)
    return (done, na, pos, cs, st), (odone, ona, o)


def test_step_full_size_every_hole(g, W, orc, step_bound):
    """One whole step on the 1e5-hole cloud, in the launch configuration of
    the benchmark: every hole's new position agrees with the oracle's FP64
    step to the displacement that the field tolerance (1e-5 A_j) allows, plus
    device-libm rounding; no hole is collected in that step on either side."""
    w = W.single_cloud(100000, seed=1)
    p, d = dev_params(g, W)
    ctx = g.gccd_init(p)
    try:
        g.gccd_load(ctx, *gpu_tensors(w.x, w.y, w.z))
        done, na = g.gccd_run(ctx, w.dt_ps, 1)
        pos, cs = g.gccd_positions(ctx, w.n)
        pos, cs = pos.cpu().numpy(), cs.cpu().numpy()
    finally:
        g.gccd_destroy(ctx)
    _, A = orc.field([w.x, w.y, w.z], with_magnitude=True)
    o = orc.State(oracle_device(orc, d), w.x, w.y, w.z)
    odone, ona = o.run(w.dt_ps, 1)
    assert (done, na) == (odone, ona) == (1, w.n)
    assert np.array_equal(cs, o.cstep)
    dr = np.linalg.norm(pos - np.stack([o.x, o.y, o.z]), axis=0)
    bound = step_bound(d, w.dt_ps) * FIELD_TOL * A + 1e-9
    print(f"[step] n={w.n}, one step: max |dr| = {dr.max():.3e} um, "
          f"max |dr|/bound = {np.max(dr / bound):.3e}", flush=True)
    assert np.all(dr <= bound)


def test_run_coulomb_off_matches_oracle(g, W, orc):
    """Drift + diffusion: identical Philox words; positions equal to rounding
    of the device math library; identical collection steps."""
    w = W.x_ray_cloud(seed=3)
    (done, na, pos, cs, st), (odone, ona, o) = run_both(g, W, orc, w, 2000, coulomb=0)
    assert (done, na) == (odone, ona)
    assert np.array_equal(cs, o.cstep)
    dmax = np.max(np.abs(pos - np.stack([o.x, o.y, o.z])))
    print(f"[run] coulomb off: max |dr| = {dmax:.3e} um over {done} steps", flush=True)
    assert dmax < 1e-10
    assert st["pair_interactions"] == 0
    assert st["carrier_steps"] == int(np.sum(np.where(cs > 0, cs, 0)))


def moments(x, y):
    vx, vy = np.var(x), np.var(y)
    rho = np.cov(x, y)[0, 1] / math.sqrt(vx * vy)
    return vx, vy, rho


def test_run_cloud_1000_moments_and_image(g, W, orc):
    """The 1000-hole cloud run to completion with Coulomb repulsion: second
    moments of the collected cloud within 0.5 %, charge conserved, and the
    GPU image equal to the oracle's histogram of the same final positions."""
    w = W.x_ray_cloud(seed=1)
    (done, na, pos, cs, st), (odone, ona, o) = run_both(g, W, orc, w, 20000)
    assert na == 0 and ona == 0
    assert abs(done - odone) <= 3
    m_g, m_o = moments(pos[0], pos[1]), moments(o.x, o.y)
    print(f"[run] n=1000: steps gpu {done} oracle {odone}; var_x {m_g[0]:.5f} vs {m_o[0]:.5f}; "
          f"var_y {m_g[1]:.5f} vs {m_o[1]:.5f}; rho {m_g[2]:.4f} vs {m_o[2]:.4f}", flush=True)
    assert abs(m_g[0] / m_o[0] - 1) < 5e-3 and abs(m_g[1] / m_o[1] - 1) < 5e-3
    assert abs(m_g[2] - m_o[2]) < 5e-3
    assert st["pair_interactions"] == st["carrier_steps"] * w.n
    assert st["carrier_steps"] == int(cs.sum())
    # image of the GPU's own final positions, binned on both sides
    p, d = dev_params(g, W)
    ctx = g.gccd_init(p)
    try:
        xg, yg, zg = gpu_tensors(pos[0], pos[1], np.minimum(pos[2], 0.0))
        g.gccd_load(ctx, xg, yg, zg)                # every hole collected at load
        counts, nout = g.gccd_image(ctx, 0.0, 0.0, w.pitch_um, w.nx, w.ny)
        counts, nout = counts.cpu().numpy(), int(nout.cpu().numpy()[0])
    finally:
        g.gccd_destroy(ctx)
    oc, onout = orc.image(pos[0], pos[1], np.zeros(w.n, np.int32), 0.0, 0.0, w.pitch_um,
                          w.nx, w.ny)
    assert np.array_equal(counts, oc) and nout == onout
    assert int(counts.sum()) + nout == w.n


def test_run_cloud_10000_moments(g, W, orc):
    """1e4-hole cloud (the smallest single-cloud size), 150 steps with
    Coulomb repulsion: variances of the travelling cloud within 0.5 %."""
    w = W.single_cloud(10000, seed=1)
    (done, na, pos, cs, st), (odone, ona, o) = run_both(g, W, orc, w, 150)
    assert done == odone == 150 and na == ona == w.n
    for k, (a, b) in enumerate(zip(pos, (o.x, o.y, o.z))):
        rel = np.var(a) / np.var(b) - 1.0
        print(f"[run] n=10000 axis {k}: var gpu {np.var(a):.5f} oracle {np.var(b):.5f} "
              f"rel {rel:.2e}", flush=True)
        assert abs(rel) < 5e-3


def test_run_shallow_cloud_10000_to_completion(g, W, orc):
    w = W.single_cloud(10000, seed=2, depth_um=30.0)
    (done, na, pos, cs, st), (odone, ona, o) = run_both(g, W, orc, w, 5000)
    assert na == 0 and ona == 0
    m_g, m_o = moments(pos[0], pos[1]), moments(o.x, o.y)
    print(f"[run] n=10000 d=30: steps {done}/{odone} var_x {m_g[0]:.5f}/{m_o[0]:.5f} "
          f"var_y {m_g[1]:.5f}/{m_o[1]:.5f}", flush=True)
    assert abs(m_g[0] / m_o[0] - 1) < 5e-3 and abs(m_g[1] / m_o[1] - 1) < 5e-3


def test_run_two_body_mirror(g, W):
    """Two holes, Coulomb only: the GPU keeps them exact mirror images."""
    p, d = dev_params(g, W, diffusion=0, a1=0.0, a2=0.0, mobility_model=1)
    ctx = g.gccd_init(p)
    try:
        g.gccd_load(ctx, *gpu_tensors([-0.5, 0.5], [0.0, 0.0], [300.0, 300.0]))
        g.gccd_run(ctx, 10.0, 1000)
        pos, _ = g.gccd_positions(ctx, 2)
        pos = pos.cpu().numpy()
    finally:
        g.gccd_destroy(ctx)
    assert pos[0, 0] == -pos[0, 1] and pos[2, 0] == 300.0
    mu0 = 1.31e8 * 140.0 ** -2.2
    K = 1.602176634e-19 / (4 * math.pi * 8.8541878128e-12 * 11.7) * 1e10
    want = (1.0 + 6.0 * mu0 * K * 1e4 * 1000 * 10e-12) ** (1.0 / 3.0)
    assert abs((pos[0, 1] - pos[0, 0]) / want - 1.0) < 3e-4


def test_run_is_resumable_and_deterministic(g, W):
    w = W.single_cloud(4000, seed=7, depth_um=20.0)
    p, d = dev_params(g, W)
    outs = []
    for plan in ([45, 70, 5000], [115, 5000], [115, 5000]):
        ctx = g.gccd_init(p)
        try:
            g.gccd_load(ctx, *gpu_tensors(w.x, w.y, w.z))
            tot = 0
            for k in plan:
                tot += g.gccd_run(ctx, w.dt_ps, k)[0]
            pos, cs = g.gccd_positions(ctx, w.n)
            outs.append((tot, pos.cpu().numpy(), cs.cpu().numpy(), g.gccd_stats(ctx)))
        finally:
            g.gccd_destroy(ctx)
    for tot, pos, cs, st in outs[1:]:
        assert tot == outs[0][0]
        assert np.array_equal(pos, outs[0][1]) and np.array_equal(cs, outs[0][2])
        assert st["pair_interactions"] == outs[0][3]["pair_interactions"]


def test_load_boundary_handling(g, W, orc):
    x = np.arange(6, dtype=np.float64)
    z = np.array([680.0, 0.0, -1.0, 10.0, 675.0, 1e-9])
    p, d = dev_params(g, W)
    ctx = g.gccd_init(p)
    try:
        g.gccd_load(ctx, *gpu_tensors(x, x, z))
        pos, cs = g.gccd_positions(ctx, 6)
        st = g.gccd_stats(ctx)
    finally:
        g.gccd_destroy(ctx)
    o = orc.State(oracle_device(orc, d), x, x, z)
    assert np.array_equal(pos.cpu().numpy()[2], o.z)
    assert np.array_equal(cs.cpu().numpy(), o.cstep)
    assert st["n_active"] == o.n_active == 4     # 670 (mirrored), 10, 675, 1e-9


def test_everything_collected_at_load(g, W):
    p, d = dev_params(g, W)
    ctx = g.gccd_init(p)
    try:
        g.gccd_load(ctx, *gpu_tensors([1.0, 2.0], [1.0, 2.0], [0.0, -3.0]))
        assert g.gccd_run(ctx, 10.0, 100) == (0, 0)
        counts, nout = g.gccd_image(ctx, 0.0, 0.0, 15.0, 4, 4)
        assert int(counts.sum().item()) == 2 and int(nout.item()) == 0
    finally:
        g.gccd_destroy(ctx)


def test_image_edges_bit_exact(g, W, orc):
    """Bin edges, negative offsets, far-away and non-finite positions."""
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.uniform(-20, 1000, 5000), [0.0, 15.0, 960.0, 959.9999999999,
                                                      -1e-300, np.nan, np.inf, 1e300]])
    y = np.concatenate([rng.uniform(-20, 1000, 5000), [0.0, 30.0, 0.0, 945.0, 5.0, 1.0, 1.0,
                                                      1.0]])
    z = np.zeros_like(x)
    p, d = dev_params(g, W)
    for (x0, y0, pitch, nx, ny) in [(0.0, 0.0, 15.0, 64, 64), (-7.5, 3.0, 2.5, 401, 7),
                                    (100.0, 100.0, 15.0, 1, 1)]:
        ctx = g.gccd_init(p)
        try:
            g.gccd_load(ctx, *gpu_tensors(x, y, z))
            counts, nout = g.gccd_image(ctx, x0, y0, pitch, nx, ny)
            counts, nout = counts.cpu().numpy(), int(nout.cpu().numpy()[0])
        finally:
            g.gccd_destroy(ctx)
        oc, onout = orc.image(x, y, np.zeros(x.size, np.int32), x0, y0, pitch, nx, ny)
        assert np.array_equal(counts, oc) and nout == onout
        assert int(counts.sum()) + nout == x.size


def test_image_full_size_concentrated(g, W, orc):
    """2^24 collected holes, most of them within a few pixels (millions of
    increments of one counter) and 2 % sprayed over an area four times the
    grid's width: the histogram and the outside count are bit-exact."""
    n = 1 << 24
    rng = np.random.default_rng(23)
    wide = rng.random(n) < 0.02
    x = np.where(wide, rng.uniform(-1440.0, 2400.0, n), rng.normal(480.0, 6.0, n))
    y = np.where(wide, rng.uniform(-1440.0, 2400.0, n), rng.normal(480.0, 6.0, n))
    z = np.zeros(n)
    p, d = dev_params(g, W)
    ctx = g.gccd_init(p)
    try:
        g.gccd_load(ctx, *gpu_tensors(x, y, z))
        counts, nout = g.gccd_image(ctx, 0.0, 0.0, 15.0, 64, 64)
        counts, nout = counts.cpu().numpy(), int(nout.cpu().numpy()[0])
    finally:
        g.gccd_destroy(ctx)
    oc, onout = orc.image(x, y, np.zeros(n, np.int32), 0.0, 0.0, 15.0, 64, 64)
    print(f"[image] n=2^24: fullest pixel {int(oc.max())}, outside {onout}", flush=True)
    assert oc.max() > 1 << 20 and onout > 0
    assert np.array_equal(counts, oc) and nout == onout
    assert int(counts.sum()) + nout == n


def test_nonfinite_position_is_reported(g, W):
    p, d = dev_params(g, W)
    ctx = g.gccd_init(p)
    try:
        g.gccd_load(ctx, *gpu_tensors([1.0, np.nan], [0.0, 0.0], [100.0, 100.0]))
        with pytest.raises(g.GccdError) as e:
            g.gccd_run(ctx, 10.0, 5)
        assert e.value.status == g.GCCD_E_NONFINITE
    finally:
        g.gccd_destroy(ctx)


def test_call_order_and_arguments_on_gpu(g, W):
    p, d = dev_params(g, W)
    ctx = g.gccd_init(p)
    try:
        with pytest.raises(g.GccdError) as e:
            g.gccd_run(ctx, 10.0, 5)
        assert e.value.status == g.GCCD_E_STATE
        with pytest.raises(g.GccdError) as e:
            g.gccd_field(ctx, 4)
        assert e.value.status == g.GCCD_E_STATE
        with pytest.raises(g.GccdError) as e:
            g.gccd_set_launch(ctx, 3, 0)
        assert e.value.status == g.GCCD_E_INVALID
        g.gccd_load(ctx, *gpu_tensors([1.0], [1.0], [5.0]))
        with pytest.raises(g.GccdError) as e:
            g.gccd_run(ctx, -1.0, 5)
        assert e.value.status == g.GCCD_E_INVALID
        with pytest.raises(g.GccdError) as e:
            g.gccd_image(ctx, 0.0, 0.0, 0.0, 4, 4)
        assert e.value.status == g.GCCD_E_INVALID
        assert g.gccd_run(ctx, 10.0, 0) == (0, 1)
    finally:
        g.gccd_destroy(ctx)
