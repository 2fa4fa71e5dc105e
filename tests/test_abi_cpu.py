"""The C ABI without a GPU: exports, struct layout, argument validation.

No compute call is made here; calls that would need the device either fail
validation first or report GCCD_E_DEVICE on a machine without a GPU.
"""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gccd.h")


@pytest.fixture(scope="module")
def g():
    from paper_2203_11043_amd import gccd
    return gccd


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gccd_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(g):
    names = declared_functions()
    assert len(names) == 21
    for name in names:
        assert hasattr(g.lib, name), name
    assert sorted(g.EXPORTS) == names


def test_struct_layout_matches_header(g, tmp_path):
    """The binding's ctypes structs must match the C compiler's layout."""
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "gccd.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(gccd_params),'
        " offsetof(gccd_params, thickness_um), offsetof(gccd_params, coulomb),"
        " offsetof(gccd_params, seed), offsetof(gccd_params, event), sizeof(gccd_stats_t));\n"
        'printf("%zu %zu %zu %zu %zu %zu %d\\n", offsetof(gccd_stats_t, field_ms),'
        " offsetof(gccd_stats_t, source_chunks), offsetof(gccd_stats_t, max_source_chunks),"
        " offsetof(gccd_stats_t, near_chunks), offsetof(gccd_stats_t, graph_replays),"
        " offsetof(gccd_stats_t, graph_usable), GCCD_CLOSURE_WEIGHTS);"
        'printf("%zu\\n", offsetof(gccd_stats_t, tile_sources));'
        'printf("%d\\n", GCCD_NOALLOC_MAX_CARRIERS);'
        "\nreturn 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    P, S = g.CParams, g.CStats
    want = [ctypes.sizeof(P), P.thickness_um.offset, P.coulomb.offset, P.seed.offset,
            P.event.offset, ctypes.sizeof(S), S.field_ms.offset, S.source_chunks.offset,
            S.max_source_chunks.offset, S.near_chunks.offset, S.graph_replays.offset,
            S.graph_usable.offset, g.CLOSURE_WEIGHTS, S.tile_sources.offset,
            g.GCCD_NOALLOC_MAX_CARRIERS]
    assert list(map(int, out)) == want


def _init_status(g, **changes):
    p = g.Params().c()
    for k, v in changes.items():
        setattr(p, k, v)
    out = ctypes.c_void_p()
    st = g.lib.gccd_init(ctypes.byref(p), None, ctypes.byref(out))
    if st == g.GCCD_OK:
        g.lib.gccd_destroy(out)
    return st


@pytest.mark.parametrize("changes", [
    dict(abi_version=0), dict(reserved0=1), dict(reserved1=7),
    dict(thickness_um=0.0), dict(thickness_um=-5.0), dict(thickness_um=math.nan),
    dict(a1_Vcm_per_um=math.inf), dict(a2_Vcm=math.nan),
    dict(well_z_um=675.0), dict(well_z_um=math.nan),
    dict(temperature_K=0.0), dict(eps_r=-11.7), dict(softening_um=0.0),
    dict(softening_um=math.nan), dict(coulomb=2), dict(diffusion=-1),
    dict(mobility_model=3), dict(collected_are_sources=5),
])
def test_init_rejects_bad_params(g, changes):
    assert _init_status(g, **changes) == g.GCCD_E_INVALID


def test_init_without_gpu_reports_device_error(g):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _init_status(g) == g.GCCD_E_DEVICE


def test_null_arguments(g):
    L = g.lib
    assert L.gccd_init(None, None, None) == g.GCCD_E_INVALID
    out = ctypes.c_void_p()
    assert L.gccd_init(None, None, ctypes.byref(out)) == g.GCCD_E_INVALID
    assert L.gccd_load(None, 10, None, None, None) == g.GCCD_E_INVALID
    assert L.gccd_load_events(None, 1, None, None, None, None) == g.GCCD_E_INVALID
    assert L.gccd_image_events(None, 0.0, 0.0, 15.0, 4, 4, None, None) == g.GCCD_E_INVALID
    assert L.gccd_run(None, 10.0, 1, None, None) == g.GCCD_E_INVALID
    assert L.gccd_image(None, 0.0, 0.0, 15.0, 4, 4, None, None) == g.GCCD_E_INVALID
    assert L.gccd_field(None, None, None, None) == g.GCCD_E_INVALID
    assert L.gccd_positions(None, None, None, None, None) == g.GCCD_E_INVALID
    assert L.gccd_stats(None, None) == g.GCCD_E_INVALID
    assert L.gccd_set_launch(None, 0, 0) == g.GCCD_E_INVALID
    assert L.gccd_set_tile(None, 0) == g.GCCD_E_INVALID
    assert L.gccd_set_timing(None, 1) == g.GCCD_E_INVALID
    assert L.gccd_set_precision(None, 0) == g.GCCD_E_INVALID
    assert L.gccd_set_schedule(None, 2) == g.GCCD_E_INVALID
    assert L.gccd_set_closure(None, None, 0, 0) == g.GCCD_E_INVALID
    assert L.gccd_autotune(None, None, None, None) == g.GCCD_E_INVALID
    assert L.gccd_closure_parts(None, None, None, None, None, None, None, None, None) == \
        g.GCCD_E_INVALID
    L.gccd_destroy(None)
    assert L.gccd_last_error(None) == b""


def test_strerror_names_every_status(g):
    seen = set()
    for st in (0, -1, -2, -3, -4, -5):
        s = g.lib.gccd_strerror(st).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 6
    assert g.lib.gccd_strerror(-99) == b"unknown status"
