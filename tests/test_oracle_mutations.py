"""The pins must catch a plausible mistake anywhere in the oracle.

Each case plants one mistake in a copy of the oracle source (on the CPU),
builds it, and runs the pin suite against it in a subprocess; the suite must
fail.  The unmodified source must pass.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gccd_oracle.c")

MUTATIONS = {
    "field r^-2 instead of r^-3": ("double w = 1.0 / (q * sqrt(q));", "double w = 1.0 / q;"),
    "field sign": ("double dx = tx[j] - sx[i];", "double dx = sx[i] - tx[j];"),
    "Coulomb prefactor": ("* 1e12 * 1e-2;", "* 1e12 * 1e-3;"),
    "softening dropped": ("double q = r2 + e2;", "double q = r2 + 1e-30;"),
    "mobility T exponent": ("pow(T, -2.2)", "pow(T, -2.0)"),
    "mobility beta exponent": ("0.46 * pow(T, 0.17)", "0.46 * pow(T, 0.27)"),
    "Philox multiplier": ("0xD2511F53u", "0xD2511F55u"),
    "Box-Muller pair": ("n[1] = r01 * sin(2.0 * ORC_PI * u1);",
                        "n[1] = r01 * cos(2.0 * ORC_PI * u1);"),
    "diffusion variance": ("sqrt(2.0 * D * dt_s)", "sqrt(D * dt_s)"),
    "static field sign": ("p->a1 * z[j] - p->a2", "p->a2 - p->a1 * z[j]"),
    "mirror at the back": ("if (zn > p->thickness_um) zn = 2.0 * p->thickness_um - zn;",
                           "if (zn > p->thickness_um) zn = p->thickness_um;"),
    "collection test": ("if (zn <= p->z_well_um) cstep[j]", "if (zn < p->z_well_um - 0.5) cstep[j]"),
    "pixel rounding": ("double fx = floor((x[j] - x0) / pitch);",
                       "double fx = round((x[j] - x0) / pitch);"),
}


def build(src_text, out_dir, name):
    c = os.path.join(out_dir, f"{name}.c")
    with open(c, "w") as f:
        f.write(src_text)
    so = os.path.join(out_dir, f"lib{name}.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I", os.path.join(ROOT, "oracle"), "-o", so, c, "-lm"], check=True)
    return so


def pins_pass(lib_path):
    env = dict(os.environ, ORACLE_LIB=lib_path, OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "8"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode == 0, r.stdout[-2000:]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_unmodified_oracle_passes(source, tmp_path):
    ok, out = pins_pass(build(source, str(tmp_path), "clean"))
    assert ok, out


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(source, tmp_path, name):
    old, new = MUTATIONS[name]
    assert source.count(old) == 1, f"mutation site not found once: {old}"
    ok, out = pins_pass(build(source.replace(old, new), str(tmp_path), "mutant"))
    assert not ok, f"the pins did not catch: {name}\n{out}"
