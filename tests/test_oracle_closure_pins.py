"""Pins of the closure oracle (oracle/closure.py) and of the windowed pair
sum, each against a fact from outside the code under test: brute force,
exactness properties of the interpolation and deposit schemes, symmetries of
the construction, and the exact far field itself."""
import importlib.util
import math
import os

import numpy as np
import pytest

if os.environ.get("ORACLE_CLOSURE"):
    # the mutation check points the pins at a deliberately broken copy
    _spec = importlib.util.spec_from_file_location("closure_under_test",
                                                   os.environ["ORACLE_CLOSURE"])
    C = importlib.util.module_from_spec(_spec)
    _spec.loader.exec_module(C)
else:
    from oracle import closure as C


@pytest.fixture(scope="module")
def Kc(orc):
    return orc.coulomb_constant(11.7)


def gauss(n, sigma, seed, center=(480.0, 480.0, 300.0)):
    g = np.random.default_rng(seed)
    p = g.normal(0.0, sigma, size=(3, n))
    return [p[d] + center[d] for d in range(3)]


# ---------------------------------------------------------------- windowed sum

def test_window_brute_force(orc, Kc):
    """Tiny case against a direct double loop with an explicit distance test."""
    g = np.random.default_rng(3)
    t = g.uniform(-1, 1, size=(3, 7))
    s = g.uniform(-1, 1, size=(3, 40))
    lo, hi, eps = 0.3, 0.9, 1e-3
    E = orc.field_window(t, s, lo, hi, eps)
    ref = np.zeros((3, 7))
    for j in range(7):
        for i in range(40):
            r = t[:, j] - s[:, i]
            d = math.sqrt(float(r @ r))
            if lo <= d < hi:
                ref[:, j] += Kc * r / (d * d + eps * eps) ** 1.5
    assert np.allclose(E, ref, rtol=1e-13, atol=1e-12)


def test_window_split_adds_to_full_field(orc):
    x, y, z = gauss(3000, 1.2, 5)
    full, A = orc.field([x, y, z], with_magnitude=True)
    near = orc.field_window([x, y, z], [x, y, z], 0.0, 0.7)
    far = orc.field_window([x, y, z], [x, y, z], 0.7, np.inf)
    assert np.max(np.linalg.norm(near + far - full, axis=0) / A) < 1e-13
    assert np.max(np.abs(orc.field_window([x, y, z], [x, y, z], 0.0, np.inf) - full)) \
        <= 1e-13 * np.max(A)
    assert np.all(orc.field_window([x, y, z], [x, y, z], 0.0, 0.0) == 0.0)


# ---------------------------------------------------------------- placement

def test_placement_keeps_every_charge_inside(orc):
    x, y, z = gauss(20000, 2.0, 7)
    origin, h = C.placement(x, y, z)
    assert h == pytest.approx(0.5 * 2.0, rel=0.02)       # s = sigma for a Gaussian
    u = [(v - origin[d]) / h for d, v in enumerate((x, y, z))]
    assert all(np.all((v >= 1.0) & (v < C.NG - 2)) for v in u)
    # an outlier widens the grid instead of leaving it
    x2 = np.append(x, x.mean() + 100.0)
    y2, z2 = np.append(y, y.mean()), np.append(z, z.mean())
    origin, h = C.placement(x2, y2, z2)
    u = (x2 - origin[0]) / h
    assert np.all((u >= 1.0) & (u < C.NG - 2)) and h > 5.0
    # the grid is centred on the centroid
    c = (origin + 0.5 * (C.NG - 1) * h)
    assert np.allclose(c, [x2.mean(), y2.mean(), z2.mean()], rtol=0, atol=1e-9)


# ---------------------------------------------------------------- deposit

def test_deposit_conserves_charge_and_centroid(orc):
    x, y, z = gauss(5000, 1.0, 9)
    origin, h = C.placement(x, y, z)
    rho = C.deposit(x, y, z, origin, h)
    assert rho.sum() == pytest.approx(5000.0, rel=1e-13)
    k = np.arange(C.NG)
    # linear weights reproduce linear functions: the node-weighted mean
    # position equals the charges' mean position
    for d, (v, axis) in enumerate(((x, (0, 1)), (y, (0, 2)), (z, (1, 2)))):
        prof = rho.sum(axis=axis)
        assert origin[d] + h * (prof @ k) / prof.sum() == pytest.approx(v.mean(), abs=1e-9)


def test_deposit_single_charges():
    origin, h = np.zeros(3), 1.0
    rho = C.deposit([3.0], [4.0], [5.0], origin, h)
    assert rho[5, 4, 3] == 1.0 and rho.sum() == 1.0
    rho = C.deposit([3.5], [4.5], [5.5], origin, h)
    assert np.allclose(rho[5:7, 4:6, 3:5], 0.125) and rho.sum() == pytest.approx(1.0)
    rho = C.deposit([3.25], [4.0], [5.0], origin, h)
    assert rho[5, 4, 3] == 0.75 and rho[5, 4, 4] == 0.25


# ---------------------------------------------------------------- network parts

def test_conv3d_against_loops():
    g = np.random.default_rng(11)
    a = g.normal(size=(2, 5, 5, 5))
    w = g.normal(size=(3, 2, 3, 3, 3))
    out = C.conv3d(a, w)
    ref = np.zeros((3, 5, 5, 5))
    pad = np.zeros((2, 7, 7, 7))
    pad[:, 1:6, 1:6, 1:6] = a
    for o in range(3):
        for z in range(5):
            for y in range(5):
                for x in range(5):
                    ref[o, z, y, x] = np.sum(w[o] * pad[:, z:z + 3, y:y + 3, x:x + 3])
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-12)
    w1 = g.normal(size=(3, 2, 1, 1, 1))
    assert np.allclose(C.conv3d(a, w1), np.einsum("oi,izyx->ozyx", w1[:, :, 0, 0, 0], a))


def test_pool_and_upsample():
    a = np.arange(8.0).reshape(1, 2, 2, 2)
    assert C.avgpool2(a).item() == 3.5
    # a linear function of the coarse cell centres comes back as the same
    # linear function at the fine cell centres (coarse i + 1/4 per fine half
    # cell), away from the clamped edges
    n = 6
    i = np.arange(n, dtype=float)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    coarse = (2.0 * X - 3.0 * Y + 0.5 * Z + 1.0)[None]
    fine = C.upsample2(coarse)
    f = (np.arange(2 * n) - 0.5) / 2.0
    FZ, FY, FX = np.meshgrid(f, f, f, indexing="ij")
    want = 2.0 * FX - 3.0 * FY + 0.5 * FZ + 1.0
    sl = slice(1, 2 * n - 1)
    assert np.allclose(fine[0, sl, sl, sl], want[sl, sl, sl], atol=1e-12)
    # and averaging the upsampled field gives back the coarse one in the interior
    assert np.allclose(C.avgpool2(fine)[0, 1:-1, 1:-1, 1:-1], coarse[0, 1:-1, 1:-1, 1:-1])


def test_bf16_rounding():
    # bfloat16 keeps 7 fraction bits: neighbours of 1 are 1 + k 2^-7
    v = np.array([1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-9, -2.5, 3.0e38, 1.0 + 3 * 2.0**-8,
                  1.0 + 2.0**-9])
    out = C.bf16(v)
    assert out[0] == 1.0 and out[3] == -2.5
    assert out[1] == 1.0                      # halfway, ties to the even neighbour 1
    assert out[2] == 1.0 + 2.0**-7            # above halfway rounds up
    assert out[5] == 1.0 + 2.0**-6            # halfway from the odd 1 + 2^-7: up to even
    assert out[6] == 1.0
    assert np.isfinite(out[4])


# ---------------------------------------------------------------- interpolation

def test_catmull_rom_reproduces_quadratics():
    """Cubic convolution with a = -1/2 is exact for polynomials of degree <= 2
    and is a partition of unity; at a node it returns the node value."""
    g = np.random.default_rng(13)
    k = np.arange(C.NG, dtype=float)
    Z, Y, X = np.meshgrid(k, k, k, indexing="ij")
    q = lambda x, y, z: 1.5 + 0.2 * x - 0.7 * y + 0.01 * x * x - 0.03 * y * z + 0.02 * z * z
    F = np.stack([q(X, Y, Z), np.ones_like(X)])
    pts = g.uniform(1.0, C.NG - 2.0, size=(3, 500))
    out = C.interpolate(F, *pts, np.zeros(3), 1.0)
    assert np.allclose(out[0], q(*pts), rtol=1e-12, atol=1e-12)
    assert np.allclose(out[1], 1.0, atol=1e-13)
    w = C.catmull_rom(np.array(0.0))
    assert [float(v) for v in w] == [0.0, 1.0, 0.0, 0.0]


# ---------------------------------------------------------------- assembly

def test_closure_with_exact_far_nodes_matches_exact_field(orc):
    """With the exact far field at the nodes in place of the network, the
    closure's far part reproduces the exact field of the sources beyond a, and
    near plus far the exact Eq. (6) field, up to interpolation and the
    discreteness of the far charges.  Errors are measured against the rms of
    the exact far field: the total field's rms is set by a few close pairs.
    This checks the node convention, the K / h^2 unit and the split radius
    (a half-cell shift, a wrong power of h or a different split fails)."""
    x, y, z = gauss(30000, 1.5, 17)
    idx = np.random.default_rng(1).choice(30000, 400, replace=False)
    t = [x[idx], y[idx], z[idx]]
    src = [x, y, z]
    near, far, (origin, h) = C.closure_field(
        orc, t, src, parts=True,
        far_nodes=lambda rho, o, hh: C.exact_far_nodes(orc, src, o, hh))
    a = 0.8 * h  # the split radius of the construction
    far_exact = orc.field_window(t, src, a, np.inf)
    total = orc.field(t, src)
    rms = lambda E: np.sqrt(np.mean(np.sum(E**2, axis=0)))
    scale = rms(far_exact)
    assert rms(far - far_exact) / scale < 0.03
    assert rms(near + far - total) / scale < 0.03
    assert np.allclose(near + far_exact, total, rtol=0, atol=1e-9 * np.abs(total).max())


def test_closure_is_translation_invariant_and_scale_covariant(orc):
    """Any linear network: shifting the cloud leaves the field unchanged;
    stretching it about its centroid by 2 divides the field by 4 (up to the
    softening, taken negligible here)."""
    g = np.random.default_rng(19)
    W = g.normal(0.0, 0.05, size=C.n_weights())
    x, y, z = gauss(1500, 0.8, 23)
    src = [x, y, z]
    tgt = [v[:50] for v in src]
    eps = 1e-9
    E = C.closure_field(orc, tgt, src, W, softening_um=eps)
    sh = [v + d for v, d in zip(src, (3.25, -7.5, 11.0))]
    Es = C.closure_field(orc, [v[:50] for v in sh], sh, W, softening_um=eps)
    assert np.allclose(Es, E, rtol=1e-9, atol=1e-9 * np.abs(E).max())
    c = [v.mean() for v in src]
    st = [cc + 2.0 * (v - cc) for v, cc in zip(src, c)]
    E2 = C.closure_field(orc, [v[:50] for v in st], st, W, softening_um=eps)
    assert np.allclose(E2, E / 4.0, rtol=1e-8, atol=1e-8 * np.abs(E).max())
