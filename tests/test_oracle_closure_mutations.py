"""The closure oracle's pins must catch a plausible mistake anywhere in it.

Each case plants one mistake in a copy of oracle/closure.py (on the CPU) and
runs tests/test_oracle_closure_pins.py against the copy in a subprocess; the
pins must fail.  The unmodified copy must pass.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "closure.py")

MUTATIONS = {
    "placement centred off the centroid": ("origin = c - 0.5 * (NG - 1) * h", "origin = c - 0.5 * NG * h"),
    "placement width from the variance": ("s = np.sqrt((dev * dev).sum() / (3.0 * n))",
                                          "s = (dev * dev).sum() / (3.0 * n)"),
    "placement misses outliers": ("h = max(SIGMA_CELLS * s, dmax / MAX_DEV_CELLS)", "h = SIGMA_CELLS * s"),
    "deposit weights swapped": ("wx = f[0] if dx else 1.0 - f[0]", "wx = 1.0 - f[0] if dx else f[0]"),
    "deposit to the wrong node": ("np.add.at(rho, (i[2] + dz, i[1] + dy, i[0] + dx), wx * wy * wz)",
                                  "np.add.at(rho, (i[2] + dz, i[1] + dx, i[0] + dy), wx * wy * wz)"),
    "convolution padding": ("return F.conv3d(t, wt, padding=k // 2)[0].numpy()",
                            "return F.conv3d(t, wt, padding=k // 2)[0].flip(-1).numpy()"),
    "pooling as a sum": ("return a.reshape(c, m, 2, m, 2, m, 2).mean(axis=(2, 4, 6))",
                         "return a.reshape(c, m, 2, m, 2, m, 2).sum(axis=(2, 4, 6))"),
    "upsampling weights swapped": ("even = 0.75 * v + 0.25 * lo", "even = 0.25 * v + 0.75 * lo"),
    "bf16 rounding truncates": ("b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16", "b = b >> 16 << 16"),
    "Catmull-Rom weight": ("0.5 * (3.0 * f3 - 5.0 * f2 + 2.0)", "0.5 * (3.0 * f3 - 5.0 * f2 + 2.5)"),
    "interpolation stencil shifted": ("out += wt * F[:, i[2] + a - 1, i[1] + b - 1, i[0] + c - 1]",
                                      "out += wt * F[:, i[2] + a - 1, i[1] + b - 1, i[0] + c]"),
    "far field unit K / h": ("far = orc.coulomb_constant(eps_r) / (h * h) * interpolate(",
                             "far = orc.coulomb_constant(eps_r) / h * interpolate("),
    "near radius": ("a = NEAR_CELLS * h\n    near", "a = 0.5 * NEAR_CELLS * h\n    near"),
    "exact far nodes in the wrong unit": ("return (E * (h * h) / orc.coulomb_constant(eps_r))",
                                          "return (E * h / orc.coulomb_constant(eps_r))"),
}


def pins_pass(path):
    env = dict(os.environ, ORACLE_CLOSURE=path)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_closure_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode == 0, r.stdout[-2000:]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def write(tmp_path, text):
    p = tmp_path / "closure_copy.py"
    p.write_text(text)
    return str(p)


def test_unmodified_closure_oracle_passes(source, tmp_path):
    ok, out = pins_pass(write(tmp_path, source))
    assert ok, out


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_closure_mutation_is_caught(source, tmp_path, name):
    old, new = MUTATIONS[name]
    assert source.count(old) == 1, f"mutation site not found once: {old}"
    ok, out = pins_pass(write(tmp_path, source.replace(old, new)))
    assert not ok, f"the pins did not catch: {name}\n{out}"
