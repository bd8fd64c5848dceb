"""The C-ABI library loads and exports every entry point include/gsmi.h
declares; host-side argument checks return errors without launching work
(no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(gs_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def G():
    from paper_2605_13794_amd import gsmi
    if not os.path.exists(gsmi.LIB_PATH):
        from paper_2605_13794_amd import build
        build.build()
    gsmi.lib()
    return gsmi


def test_every_declared_symbol_is_exported(G):
    names = declared_functions()
    assert len(names) >= 12
    L = G.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(G.EXPORTED)


def test_sizes_and_tiles(G):
    assert G.gs_num_tiles(1920, 1080) == 120 * 68
    assert G.gs_num_tiles(128, 128) == 64
    assert G.gs_num_tiles(0, 5) == 0
    a = G.gs_workspace_size(G.GS_OP_BIN_SORT, 4096, 20000, 64, 1)
    b = G.gs_workspace_size(G.GS_OP_BIN_SORT, 4096, 40000, 64, 1)
    assert 0 < a < b and a % 256 == 0
    assert G.gs_workspace_size(G.GS_OP_RENDER_BWD, 1000, 0, 0, 2) >= 2 * 9 * 1000 * 4
    assert G.gs_workspace_size(99, 10, 10, 10, 1) == 0


def test_host_side_errors(G):
    from paper_2605_13794_amd import scenes as S
    L = G.lib()
    assert L.gs_project(None, None, 0, None, None, 0, None, None, 0, None) == G.GS_ERR_INVALID_ARG
    assert "scene" in G.gs_last_error()
    cams = G.camera_array([S.cube_camera()])
    assert L.gs_bin_sort(None, cams, 1, 10, None, None, 0, None, None, None, 0, None) == G.GS_ERR_INVALID_ARG
    bad = G.camera_array([S.cube_camera(0, 10)])
    dummy = (G.GsProjected * 1)()
    assert L.gs_render_fwd(dummy, bad, 1, None, None, None, None, None, None, None, None, None) == G.GS_ERR_INVALID_ARG
    assert L.gs_adam_step(None, None, None, None, None, 0, None, 0.9, 0.999, 1e-8, 1, None, 0, None) == G.GS_ERR_INVALID_ARG
    assert L.gs_score_keep_bits(None, 10, 3, None, None, 0, None) == G.GS_ERR_INVALID_ARG
    # workspace too small is reported before any launch
    sc = G.GsScene()
    sc.n = 10
    for f in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
        setattr(sc, f, 256)
    p = G.lod_params(G.GS_LOD_RADIUS)
    out = ctypes.c_void_p(256)
    rc = L.gs_lod_mask(ctypes.byref(sc), ctypes.byref(cams[0]), ctypes.byref(p), None, out, out, out, 16, None)
    assert rc == G.GS_ERR_WORKSPACE


def test_compact_host_side_errors(G):
    """gs_compact checks its arguments before any launch (no device pointer is
    dereferenced on these paths)."""
    L = G.lib()
    P = ctypes.c_void_p
    src, dst = (P * 1)(256), (P * 1)(512)
    rows, eb = (ctypes.c_int32 * 1)(3), (ctypes.c_int32 * 1)(4)
    ws, keep, big = P(256), P(1024), 1 << 20
    inval = G.GS_ERR_INVALID_ARG
    assert L.gs_compact(src, dst, rows, eb, 1, 10, 5, None, ws, big, None) == inval  # no keep bits for n > 0
    assert L.gs_compact(src, dst, rows, eb, 1, 10, 11, keep, ws, big, None) == inval  # n_keep > n
    assert L.gs_compact(src, dst, rows, eb, 1, -1, 0, keep, ws, big, None) == inval  # negative n
    assert L.gs_compact(src, dst, rows, eb, 0, 10, 5, keep, ws, big, None) == inval  # no arrays
    assert L.gs_compact(src, dst, rows, eb, 17, 10, 5, keep, ws, big, None) == inval  # more than 16 arrays
    assert L.gs_compact(src, dst, rows, (ctypes.c_int32 * 1)(2), 1, 10, 5, keep, ws, big, None) == inval
    assert L.gs_compact(src, dst, (ctypes.c_int32 * 1)(0), eb, 1, 10, 5, keep, ws, big, None) == inval
    assert L.gs_compact(src, dst, rows, eb, 1, 10, 5, keep, ws, 16, None) == G.GS_ERR_WORKSPACE
    assert L.gs_compact(src, dst, rows, eb, 1, 10, 5, keep, P(260), big, None) == G.GS_ERR_WORKSPACE  # unaligned


def test_noalloc_gate_refuses_oversized_input_on_the_host(G):
    """The allocation-free gate rejects more Gaussians than its fixed scratch
    holds before touching the device."""
    from paper_2605_13794_amd import scenes as S
    scn = G.GsScene()
    scn.n = (1 << 24) + 1
    cam = G.camera(S.cube_camera())
    prm = G.lod_params(G.GS_LOD_NONE)
    dummy = ctypes.c_void_p(256)
    rc = G.lib().gs_lod_mask_noalloc(ctypes.byref(scn), ctypes.byref(cam), ctypes.byref(prm), None, dummy, dummy,
                                     None)
    assert rc == G.GS_ERR_INVALID_ARG
    assert "exceeds the fixed scratch" in G.lib().gs_last_error().decode()


def test_level_ceiling_matches_reference(G):
    """L_max(t) of the library (host arithmetic) against the reference
    schedule: geometric unlock times between t0 and t1."""
    from oracle import levels as LV
    for t0, t1, K in ((2000, 32000, 5), (1000, 128000, 8), (500, 90000, 12), (5, 50, 1), (24000, 32000, 3)):
        for t in list(range(0, t1 + 2000, max(1, (t1 + 2000) // 997))) + [t0, t1, t0 - 1, t1 - 1, t1 + 1]:
            assert G.gs_lod_level_ceiling(t, t0, t1, K) == LV.level_ceiling(t, t0, t1, K), (t, t0, t1, K)
