"""The C-ABI library loads and exports every entry point include/lddmm.h
declares; host-side validation and workspace sizing (no GPU needed)."""

import ctypes
import os
import re

import pytest

from paper_1807_11560_amd import lddmm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lddmm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lddmm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "lddmm_hessvec" in names and "lddmm_register" in names and len(names) >= 10
    lib = L.raw()
    for n in names:
        assert hasattr(lib, n), n


def test_params_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors have the C compiler's size and offsets."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "lddmm.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu", sizeof(lddmm_params),'
        ' offsetof(lddmm_params, alpha), offsetof(lddmm_params, hessian),'
        ' offsetof(lddmm_params, state), offsetof(lddmm_params, integrator),'
        ' sizeof(lddmm_stats), offsetof(lddmm_stats, trials)); return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [ctypes.sizeof(L.LddmmParams), L.LddmmParams.alpha.offset,
                   L.LddmmParams.hessian.offset, L.LddmmParams.state.offset, L.LddmmParams.integrator.offset,
                   ctypes.sizeof(L.LddmmStats),
                   L.LddmmStats.trials.offset]


def test_workspace_bytes_scales_with_problem():
    small = L.Problem(grid=(32, 32, 32), band=(8, 8, 8)).workspace_bytes()
    big = L.Problem(grid=(128, 128, 128), band=(32, 32, 32), s=3).workspace_bytes()
    assert 0 < small < big
    assert big < 2 * 1024 ** 3  # fits comfortably in one MI355X


@pytest.mark.parametrize("kw,code", [
    (dict(band=(15, 16, 16)), L.E_SHAPE),            # odd band
    (dict(band=(16, 16, 80)), L.E_SHAPE),            # band larger than 64
    (dict(grid=(12, 64, 64)), L.E_SHAPE),            # band > grid
    (dict(spectral=(20, 0, 0)), L.E_SHAPE),          # alias-free bound 3K/2 - 2 = 22
    (dict(alpha=0.0), L.E_INVALID_ARG),
    (dict(sigma=-1.0), L.E_INVALID_ARG),
    (dict(s=0), L.E_INVALID_ARG),
    (dict(time_steps=0), L.E_INVALID_ARG),
    (dict(hessian=7), L.E_INVALID_ARG),
    (dict(state=2), L.E_INVALID_ARG),
    (dict(integrator=2), L.E_INVALID_ARG),
    (dict(integrator=1, state=1), L.E_INVALID_ARG),   # RK4 integrates the image state only
])
def test_validation_rejects(kw, code):
    base = dict(grid=(64, 64, 64), band=(16, 16, 16))
    base.update(kw)
    with pytest.raises(L.LddmmError) as e:
        L.Problem(**base).workspace_bytes()
    assert e.value.code == code


def test_planar_problems_size_their_workspace_and_validate():
    """A planar problem runs as the volume problem of depth 8 with band depth
    4 plus staging for two images of that depth and two band fields: its
    workspace is at least that volume problem's; the planar bounds are the
    volume ones; the batch, the static entry and the tile table take volumes
    only; ndim other than 2 or 3 is rejected."""
    planar = L.Problem(grid=(64, 64), band=(16, 16))
    assert planar.band_shape == (2, 16, 16)
    vol = L.Problem(grid=(8, 64, 64), band=(4, 16, 16))
    stage = 2 * 8 * 64 * 64 * 4 + 2 * 3 * 4 * 16 * 16 * 8
    assert planar.workspace_bytes() >= vol.workspace_bytes() + stage
    assert planar.workspace_bytes() < vol.workspace_bytes() + stage + 4096
    with pytest.raises(L.LddmmError) as ei:
        L.Problem(grid=(64, 64), band=(15, 16)).workspace_bytes()
    assert ei.value.code == L.E_SHAPE
    with pytest.raises(L.LddmmError) as ei:
        L.Problem(grid=(64, 300), band=(16, 16)).workspace_bytes()
    assert ei.value.code == L.E_SHAPE
    with pytest.raises(L.LddmmError) as ei:
        L.batch_workspace_bytes([planar])
    assert ei.value.code == L.E_SHAPE
    with pytest.raises(L.LddmmError) as ei:
        L.tiles_set(planar, {"sl_threads": 64}, arch="gfx950")
    assert ei.value.code == L.E_SHAPE
    p = L.Problem(grid=(64, 64, 64), band=(16, 16, 16)).c_params()
    n = ctypes.c_size_t(0)
    for nd in (1, 4):
        p.ndim = nd
        assert L.raw().lddmm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == L.E_SHAPE


def test_entry_points_validate_before_touching_the_device():
    """Null pointers and short workspaces are rejected on the host."""
    lib = L.raw()
    p = L.Problem(grid=(32, 32, 32), band=(8, 8, 8)).c_params()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.lddmm_shoot(ctypes.byref(p), null, fake, fake, null, fake, 1 << 40, null) == L.E_INVALID_ARG
    assert lib.lddmm_shoot(ctypes.byref(p), fake, fake, fake, null, fake, 16, null) == L.E_WORKSPACE
    assert lib.lddmm_hessvec(ctypes.byref(p), fake, fake, fake, 1 << 40, null) == L.E_INVALID_ARG
    assert lib.lddmm_hessvec(ctypes.byref(p), fake, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000),
                             1 << 40, null) == L.E_NOT_PREPARED
    assert lib.lddmm_register(ctypes.byref(p), fake, fake, fake, 1, 0, None, 0, fake, 1 << 40,
                              null) == L.E_INVALID_ARG
    assert b"grid" in lib.lddmm_status_string(L.E_SHAPE) or lib.lddmm_status_string(L.E_SHAPE)
    # the entry point without a workspace: null pointers, and problems larger than its fixed array
    assert lib.lddmm_shoot_static(ctypes.byref(p), null, fake, fake, null, null) == L.E_INVALID_ARG
    big = L.Problem(grid=(128, 128, 128), band=(32, 32, 32)).c_params()
    assert lib.lddmm_shoot_static(ctypes.byref(big), fake, fake, fake, null, null) == L.E_WORKSPACE
    assert b"lddmm_shoot_static" in lib.lddmm_last_error()


def test_switches_reject_bad_values():
    """lddmm_use_graphs and lddmm_kernel_timer validate their argument on the host."""
    lib = L.raw()
    assert lib.lddmm_use_graphs(2) == L.E_INVALID_ARG
    assert lib.lddmm_use_graphs(-1) == L.E_INVALID_ARG
    assert lib.lddmm_kernel_timer(11, 1) == L.E_INVALID_ARG
    assert lib.lddmm_kernel_timer(-1, 1) == L.E_INVALID_ARG
    assert lib.lddmm_kernel_timer(5, 0) == L.E_INVALID_ARG
    assert lib.lddmm_kernel_timer(5, 1001) == L.E_INVALID_ARG
    assert lib.lddmm_use_graphs(1) == L.OK
    assert lib.lddmm_use_graphs(0) == L.OK
    assert lib.lddmm_kernel_timer(L.KF_SRC, 4) == L.OK
    assert lib.lddmm_kernel_timer(0, 1) == L.OK


def test_deformation_state_needs_less_workspace():
    """No per-step image, grid velocity or image-grid stage-0 buffer is kept
    for the deformation state (paper §3.3: the lower-memory variant)."""
    kw = dict(grid=(128, 128, 128), band=(32, 32, 32), s=3)
    img = L.Problem(**kw).workspace_bytes()
    dfm = L.Problem(state=L.STATE_DEFORMATION, **kw).workspace_bytes()
    assert dfm < 0.8 * img


def test_batch_workspace_is_the_sum_of_aligned_slices():
    probs = [L.Problem(grid=(32, 32, 32), band=(8, 8, 8)),
             L.Problem(grid=(40, 36, 32), band=(12, 16, 8), state=L.STATE_DEFORMATION),
             L.Problem(grid=(64, 64, 64), band=(16, 16, 16), hessian=L.NEWTON)]
    want = sum((q.workspace_bytes() + 255) // 256 * 256 for q in probs)
    assert L.batch_workspace_bytes(probs) == want
    bad = probs + [L.Problem(grid=(32, 32, 32), band=(9, 8, 8))]
    with pytest.raises(L.LddmmError) as e:
        L.batch_workspace_bytes(bad)
    assert e.value.code == L.E_SHAPE and "pair 3" in str(e.value)


def test_batch_validates_before_touching_the_device():
    lib = L.raw()
    probs = [L.Problem(grid=(32, 32, 32), band=(8, 8, 8))] * 2
    arr = (L.LddmmParams * 2)(*[q.c_params() for q in probs])
    fake = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    nulls = (ctypes.c_void_p * 2)(0x1000, 0)
    ws = ctypes.c_void_p(0x3000)
    null = ctypes.c_void_p(0)
    call = lib.lddmm_register_batch
    assert call(0, arr, fake, fake, fake, 1, 1, 0, None, 0, None, None, ws, 1 << 40, null) == L.E_INVALID_ARG
    assert call(2, arr, fake, nulls, fake, 1, 1, 0, None, 0, None, None, ws, 1 << 40, null) == L.E_INVALID_ARG
    assert call(2, arr, fake, fake, fake, 1, 0, 0, None, 0, None, None, ws, 1 << 40, null) == L.E_INVALID_ARG
    assert call(2, arr, fake, fake, fake, 1, 1, 65, None, 0, None, None, ws, 1 << 40, null) == L.E_INVALID_ARG
    assert call(2, arr, fake, fake, fake, 1, 1, 0, None, 0, None, None, ws, 64, null) == L.E_WORKSPACE


def test_rk4_is_for_shooting_only():
    """The adjoint sweeps are transposes of Euler steps: gradient, hessvec,
    register and the batch reject LDDMM_RK4 on the host; the workspace query
    and the shooting entry points accept it."""
    lib = L.raw()
    prob = L.Problem(grid=(32, 32, 32), band=(8, 8, 8), integrator=L.RK4)
    assert prob.workspace_bytes() > 0
    p = prob.c_params()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    big = 1 << 40
    assert lib.lddmm_gradient(ctypes.byref(p), fake, fake, fake, fake, null, fake, big, null) == L.E_INVALID_ARG
    assert lib.lddmm_hessvec(ctypes.byref(p), fake, ctypes.c_void_p(0x2000), fake, big, null) == L.E_INVALID_ARG
    assert lib.lddmm_register(ctypes.byref(p), fake, fake, fake, 1, 1, None, 0, fake, big, null) == L.E_INVALID_ARG
    assert "lddmm_shoot" in lib.lddmm_last_error().decode()
    arr = (L.LddmmParams * 1)(p)
    ptrs = (ctypes.c_void_p * 1)(0x1000)
    assert lib.lddmm_register_batch(1, arr, ptrs, ptrs, ptrs, 1, 1, 0, None, 0, None, None, fake, big,
                                    null) == L.E_INVALID_ARG
    assert lib.lddmm_geodesic_energy(ctypes.byref(p), null, fake, fake, big, null) == L.E_INVALID_ARG


def test_tile_table_set_get_save_load_round_trip(tmp_path):
    """Host-only: entries keyed by (grid, band, spectral grid, precision,
    arch), JSON written and read back exactly, and a malformed or invalid
    file rejected without changing the table."""
    import json
    L.tiles_clear()
    try:
        a = L.Problem(grid=(128, 128, 128), band=(32, 32, 32), s=3)
        b = L.Problem(grid=(96, 96, 96), band=(24, 24, 24), s=3, precision=L.FP32_BF16X3)
        assert L.tiles_get(a, arch="gfx950") is None
        L.tiles_set(a, {"prod_rows": 2, "col_split": 3, "sl_threads": 128}, arch="gfx950")
        L.tiles_set(b, {"prod_rows": 1, "col_split": 1, "sl_threads": 64}, arch="gfx950")
        assert L.tiles_get(a, arch="gfx950") == {"prod_rows": 2, "col_split": 3, "sl_threads": 128}
        assert L.tiles_get(a, arch="gfx942") is None
        # the key is the shape and precision, not the other parameters
        a2 = L.Problem(grid=(128, 128, 128), band=(32, 32, 32), s=2, time_steps=20, alpha=0.01)
        assert L.tiles_get(a2, arch="gfx950") == L.tiles_get(a, arch="gfx950")
        assert L.tiles_get(L.Problem(grid=(96, 96, 96), band=(24, 24, 24), s=3), arch="gfx950") is None
        path = tmp_path / "tiles.json"
        L.tiles_save(str(path))
        doc = json.loads(path.read_text())
        assert doc["format"] == "lddmm-tiles-1" and len(doc["entries"]) == 2
        e = [x for x in doc["entries"] if x["grid"] == [128, 128, 128]][0]
        assert e == {"arch": "gfx950", "grid": [128, 128, 128], "band": [32, 32, 32], "spectral": [48, 48, 48],
                     "precision": "fp32", "prod_rows": 2, "col_split": 3, "sl_threads": 128, "ms_per_hvp": 0.0}
        L.tiles_clear()
        assert L.tiles_get(a, arch="gfx950") is None
        L.tiles_load(str(path))
        assert L.tiles_get(a, arch="gfx950") == {"prod_rows": 2, "col_split": 3, "sl_threads": 128}
        assert L.tiles_get(b, arch="gfx950") == {"prod_rows": 1, "col_split": 1, "sl_threads": 64}
        # every entry is checked before any is taken
        bad = dict(doc)
        bad["entries"] = [dict(e, grid=[64, 64, 64], band=[16, 16, 16], spectral=[24, 24, 24]),
                          dict(e, sl_threads=100)]
        (tmp_path / "bad.json").write_text(json.dumps(bad))
        with pytest.raises(L.LddmmError) as ei:
            L.tiles_load(str(tmp_path / "bad.json"))
        assert ei.value.code == L.E_INVALID_ARG and "entry 1" in str(ei.value)
        assert L.tiles_get(L.Problem(grid=(64, 64, 64), band=(16, 16, 16)), arch="gfx950") is None
        for text in ["", "{", "[]", '{"format": "other", "entries": []}', '{"format": "lddmm-tiles-1"}',
                     path.read_text()[:-5], path.read_text() + "x"]:
            (tmp_path / "m.json").write_text(text)
            with pytest.raises(L.LddmmError):
                L.tiles_load(str(tmp_path / "m.json"))
        with pytest.raises(L.LddmmError):
            L.tiles_load(str(tmp_path / "missing.json"))
    finally:
        L.tiles_clear()


@pytest.mark.parametrize("tiles", [dict(prod_rows=6), dict(prod_rows=-1), dict(col_split=4), dict(sl_threads=32),
                                   dict(sl_threads=512)])
def test_tile_fields_out_of_range_are_rejected(tiles):
    a = L.Problem(grid=(128, 128, 128), band=(32, 32, 32), s=3)  # M2 = 48: at most 5 rows
    with pytest.raises(L.LddmmError) as ei:
        L.tiles_set(a, tiles, arch="gfx950")
    assert ei.value.code == L.E_INVALID_ARG
    assert L.tiles_get(a, arch="gfx950") is None
