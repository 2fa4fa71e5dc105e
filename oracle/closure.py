"""FP64 CPU oracle of the far-field closure -- TEST INFRASTRUCTURE ONLY.

The closure replaces the far part of the Eq. (6) sum.  The near part stays an
exact pair sum over the sources closer than a; the far part is read from a
coarse grid:

    E_j = K sum_{i: |r_ij| < a} r_ij / (|r_ij|^2 + eps^2)^{3/2}  +  (K / h^2) I[F](r_j)

  * grid: NG^3 nodes of spacing h around the charge centroid c, node k at
    c + (k - (NG-1)/2) h on every axis; h = max(SIGMA_CELLS * s, d_max / MAX_DEV_CELLS),
    s = rms distance of the charges from c per axis (population), d_max the
    largest |x - c| over charges and axes, so every charge lies at least one
    node inside the grid;
  * density rho: every charge (travelling or collected) deposits weight 1
    with trilinear (cloud-in-cell) weights on the 8 nodes around it;
  * F = U(rho): a fixed linear U-Net of 3x3x3 convolutions without bias,
    2x2x2 average pooling and x2 linear upsampling, its weights learned
    elsewhere; F is the far field in units of K / h^2 at the nodes;
  * I[F]: Catmull-Rom (cubic convolution, a = -1/2) interpolation, separable
    over the 4x4x4 nodes around the point;
  * a = NEAR_CELLS * h.

Every quantity here is the plain definition, in float64.  Only tests may
import this module.
"""
from __future__ import annotations

import numpy as np

NG = 32                 # nodes per axis
SIGMA_CELLS = 0.5       # h = 0.5 s: sixteen rms widths across the grid
MAX_DEV_CELLS = 14.0    # and no charge farther than 14 h from the centroid
NEAR_CELLS = 0.8        # exact pair sum within a = 0.8 h

# the network: (name, kind, c_in, c_out, level); level l has NG / 2^l nodes
LAYERS = [
    ("e0a", "conv3", 1, 16, 0), ("e0b", "conv3", 16, 16, 0),
    ("e1a", "conv3", 16, 32, 1), ("e1b", "conv3", 32, 32, 1),
    ("e2a", "conv3", 32, 32, 2), ("e2b", "conv3", 32, 32, 2),
    ("b3a", "conv3", 32, 32, 3), ("b3b", "conv3", 32, 32, 3),
    ("d2", "conv3", 64, 32, 2), ("d1", "conv3", 64, 32, 1), ("d0", "conv3", 48, 16, 0),
    ("head", "conv1", 16, 3, 0),
]


def weight_shapes():
    """PyTorch Conv3d layout (c_out, c_in, kz, ky, kx) of every layer, in order."""
    out = []
    for name, kind, ci, co, _ in LAYERS:
        k = 3 if kind == "conv3" else 1
        out.append((name, (co, ci, k, k, k)))
    return out


def n_weights() -> int:
    return int(sum(np.prod(s) for _, s in weight_shapes()))


def split_weights(flat):
    """Flat float array -> {name: array of the layer's shape}."""
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == n_weights(), (flat.size, n_weights())
    out, k = {}, 0
    for name, shape in weight_shapes():
        m = int(np.prod(shape))
        out[name] = flat[k:k + m].reshape(shape)
        k += m
    return out


# ---------------------------------------------------------------- placement

def placement(x, y, z):
    """(origin, h): node k of axis d sits at origin[d] + k h."""
    p = np.stack([np.asarray(v, dtype=np.float64) for v in (x, y, z)])
    n = p.shape[1]
    c = p.sum(axis=1) / n
    dev = p - c[:, None]
    s = np.sqrt((dev * dev).sum() / (3.0 * n))
    dmax = np.abs(dev).max()
    h = max(SIGMA_CELLS * s, dmax / MAX_DEV_CELLS)
    origin = c - 0.5 * (NG - 1) * h
    return origin, h


# ---------------------------------------------------------------- deposit

def deposit(x, y, z, origin, h):
    """Cloud-in-cell charge per node, array [z][y][x] of NG^3 float64."""
    rho = np.zeros((NG, NG, NG), dtype=np.float64)
    u = [(np.asarray(v, dtype=np.float64) - origin[d]) / h for d, v in enumerate((x, y, z))]
    i = [np.floor(v).astype(np.int64) for v in u]
    f = [v - iv for v, iv in zip(u, i)]
    for dz in (0, 1):
        wz = f[2] if dz else 1.0 - f[2]
        for dy in (0, 1):
            wy = f[1] if dy else 1.0 - f[1]
            for dx in (0, 1):
                wx = f[0] if dx else 1.0 - f[0]
                np.add.at(rho, (i[2] + dz, i[1] + dy, i[0] + dx), wx * wy * wz)
    return rho


# ---------------------------------------------------------------- network

def conv3d(a, w):
    """a: [c_in, n, n, n]; w: [c_out, c_in, k, k, k]; zero padding k // 2;
    output [c_out, n, n, n].  Uses torch's CPU convolution in float64."""
    import torch
    import torch.nn.functional as F
    k = w.shape[-1]
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))[None]
    wt = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64))
    return F.conv3d(t, wt, padding=k // 2)[0].numpy()


def avgpool2(a):
    """Mean over 2x2x2 blocks: [c, n, n, n] -> [c, n/2, n/2, n/2]."""
    c, n = a.shape[0], a.shape[1]
    m = n // 2
    return a.reshape(c, m, 2, m, 2, m, 2).mean(axis=(2, 4, 6))


def upsample2(a):
    """x2 linear upsampling per axis, fine node 2i -> 3/4 a[i] + 1/4 a[i-1],
    fine node 2i+1 -> 3/4 a[i] + 1/4 a[i+1], the neighbour clamped at the
    edges: [c, n, n, n] -> [c, 2n, 2n, 2n]."""
    def one_axis(v, ax):
        n = v.shape[ax]
        idx = np.arange(n)
        lo = np.take(v, np.maximum(idx - 1, 0), axis=ax)
        hi = np.take(v, np.minimum(idx + 1, n - 1), axis=ax)
        even = 0.75 * v + 0.25 * lo
        odd = 0.75 * v + 0.25 * hi
        out = np.stack([even, odd], axis=ax + 1)
        shape = list(v.shape)
        shape[ax] = 2 * n
        return out.reshape(shape)
    for ax in (1, 2, 3):
        a = one_axis(a, ax)
    return a


def bf16(a):
    """Round float64 values to bfloat16 (nearest, ties to even), through float32."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def network(rho, weights, quantize=None):
    """F = U(rho), rho [NG, NG, NG] -> F [3, NG, NG, NG].  quantize (a
    function or None) is applied to the input, to every intermediate tensor
    the network stores and to the weights: the points where the GPU rounds
    to bfloat16.  The output stays unrounded."""
    W = split_weights(weights) if not isinstance(weights, dict) else weights
    q = quantize or (lambda v: v)

    def conv(name, a, last=False):
        out = conv3d(a, q(W[name]))
        return out if last else q(out)

    x0 = q(rho[None])
    s0 = conv("e0b", conv("e0a", x0))
    s1 = conv("e1b", conv("e1a", q(avgpool2(s0))))
    s2 = conv("e2b", conv("e2a", q(avgpool2(s1))))
    b = conv("b3b", conv("b3a", q(avgpool2(s2))))
    d2 = conv("d2", np.concatenate([q(upsample2(b)), s2]))
    d1 = conv("d1", np.concatenate([q(upsample2(d2)), s1]))
    d0 = conv("d0", np.concatenate([q(upsample2(d1)), s0]))
    return conv("head", d0, last=True)


# ---------------------------------------------------------------- interpolation

def catmull_rom(f):
    """Weights of nodes i-1, i, i+1, i+2 for a point at i + f, 0 <= f < 1."""
    f2, f3 = f * f, f * f * f
    return (0.5 * (-f3 + 2.0 * f2 - f), 0.5 * (3.0 * f3 - 5.0 * f2 + 2.0),
            0.5 * (-3.0 * f3 + 4.0 * f2 + f), 0.5 * (f3 - f2))


def interpolate(F, x, y, z, origin, h):
    """I[F] at the points: F [c, NG, NG, NG] -> [c, n]."""
    u = [(np.asarray(v, dtype=np.float64) - origin[d]) / h for d, v in enumerate((x, y, z))]
    i = [np.floor(v).astype(np.int64) for v in u]
    w = [catmull_rom(v - iv) for v, iv in zip(u, i)]
    out = np.zeros((F.shape[0], u[0].size), dtype=np.float64)
    for a in range(4):
        for b in range(4):
            for c in range(4):
                wt = w[2][a] * w[1][b] * w[0][c]
                out += wt * F[:, i[2] + a - 1, i[1] + b - 1, i[0] + c - 1]
    return out


# ---------------------------------------------------------------- assembly

def exact_far_nodes(orc, sources, origin, h, softening_um=1e-3, eps_r=11.7):
    """The exact far field (sources at distance >= a) at every node, in units
    of K / h^2: what the network is trained to reproduce.  [3, NG, NG, NG]."""
    k = np.arange(NG, dtype=np.float64)
    Z, Y, X = np.meshgrid(k, k, k, indexing="ij")
    nodes = [origin[0] + X.ravel() * h, origin[1] + Y.ravel() * h, origin[2] + Z.ravel() * h]
    E = orc.field_window(nodes, sources, NEAR_CELLS * h, np.inf, softening_um, eps_r)
    return (E * (h * h) / orc.coulomb_constant(eps_r)).reshape(3, NG, NG, NG)


def closure_field(orc, targets, sources, weights=None, softening_um=1e-3, eps_r=11.7,
                  quantize=None, parts=False, far_nodes=None):
    """The closure's field at the targets from the sources (V/cm, [3, nt]).
    far_nodes(rho, origin, h), if given, replaces the network."""
    origin, h = placement(*sources)
    a = NEAR_CELLS * h
    near = orc.field_window(targets, sources, 0.0, a, softening_um, eps_r)
    rho = deposit(*sources, origin, h)
    F = far_nodes(rho, origin, h) if far_nodes else network(rho, weights, quantize)
    far = orc.coulomb_constant(eps_r) / (h * h) * interpolate(F, *targets, origin, h)
    if parts:
        return near, far, (origin, h)
    return near + far
