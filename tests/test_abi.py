"""Host-side checks of the C ABI (no GPU needed).

* libspinpic.so loads and exports every function declared in include/spinpic.h;
* pic_init rejects bad configurations before touching the GPU (T16):
  dimensions, cell counts and sizes, the Courant limit, species, precision,
  tiles, non-unit spins and non-finite input; calls on a NULL context return
  PIC_ESTATE.
"""

import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2002_02211_amd import spinpic as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(S.LIB_PATH):
        pytest.fail("libspinpic.so is not built: run __graft_entry__.build()")
    return S.load_library()


def test_exports_every_declared_function(lib):
    header = open(os.path.join(ROOT, "include", "spinpic.h")).read()
    declared = set(re.findall(r"\b(pic_[a-z_]+)\s*\(", header))
    assert declared == set(S.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name
    # ctypes mirrors of the structs: the C side reads fields out to the last one
    assert ctypes.sizeof(S.Config) == 4 + 12 + 24 + 8 + 4 + 4 + 4 * 24 + 12 + 4 + 8 + 4 + 4
    assert ctypes.sizeof(S.State) == 8 * 4 + 8 * 4 + 8
    assert ctypes.sizeof(S.WindowConfig) == 8 + 4 + 4 + 3 * 8 + 3 * 8
    assert S.WindowConfig.s0.offset == 40 and S.WindowConfig.n0.offset == 16


def _good_cfg(**kw):
    cfg = S.make_config(2, (32, 16, 1), (0.3, 0.3, 1.0), 0.2,
                        [{"Z": -1.0, "mu": 1.0, "a": 0.00116}, {"Z": 1.0, "mu": 1836.15, "a": 1.793}])
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


def _init_status(lib, cfg, parts=None, fields=None):
    st = S.State()
    keep = []
    for s in range(S.MAX_SPECIES):
        st.count[s] = 0
        st.particles[s] = None
    for s, p in enumerate(parts or []):
        arr = np.ascontiguousarray(p, dtype=np.float64)
        keep.append(arr)
        st.count[s] = arr.shape[0]
        st.particles[s] = arr.ctypes.data
    if fields is not None:
        F = np.ascontiguousarray(fields, dtype=np.float64)
        keep.append(F)
        st.fields = F.ctypes.data
    ctx = ctypes.c_void_p()
    code = lib.pic_init(ctypes.byref(cfg), ctypes.byref(st), None, None, ctypes.byref(ctx))
    msg = lib.pic_last_error(None).decode()
    return code, msg, ctx


def _set(cfg, field, idx, value):
    getattr(cfg, field)[idx] = value
    return cfg


@pytest.mark.parametrize("mutate,code,needle", [
    (lambda c: setattr(c, "ndim", 4), S.PIC_EINVAL, "ndim"),
    (lambda c: _set(c, "n", 0, 0), S.PIC_EINVAL, "n[0]"),
    (lambda c: _set(c, "n", 1, 70000), S.PIC_EINVAL, "n[1]"),
    (lambda c: _set(c, "d", 0, -1.0), S.PIC_EINVAL, "d[0]"),
    (lambda c: _set(c, "d", 1, math.nan), S.PIC_EINVAL, "d[1]"),
    (lambda c: setattr(c, "dt", 0.0), S.PIC_EINVAL, "dt"),
    (lambda c: setattr(c, "dt", 0.3 / math.sqrt(2) * 1.0001), S.PIC_ECFL, "Courant"),
    (lambda c: setattr(c, "dt", 1.0), S.PIC_ECFL, "Courant"),
    (lambda c: setattr(c, "precision", 7), S.PIC_EINVAL, "precision"),
    (lambda c: setattr(c, "nspecies", 0), S.PIC_EINVAL, "nspecies"),
    (lambda c: setattr(c, "nspecies", 5), S.PIC_EINVAL, "nspecies"),
    (lambda c: setattr(c.sp[1], "mu", 0.0), S.PIC_EINVAL, "species 1"),
    (lambda c: setattr(c.sp[0], "a", math.inf), S.PIC_EINVAL, "species 0"),
    (lambda c: _set(c, "tile", 0, 100), S.PIC_EINVAL, "tile[0]"),
    (lambda c: _set(c, "tile", 1, -2), S.PIC_EINVAL, "tile[1]"),
    (lambda c: setattr(c, "slack", -0.5), S.PIC_EINVAL, "slack"),
    (lambda c: setattr(c, "flags", 8), S.PIC_EINVAL, "flags"),
    (lambda c: setattr(c, "deposit_acc", 3), S.PIC_EINVAL, "deposit_acc"),
])
def test_T16_init_rejects_bad_config(lib, mutate, code, needle):
    cfg = _good_cfg()
    mutate(cfg)
    got, msg, ctx = _init_status(lib, cfg)
    assert got == code, msg
    assert needle in msg
    assert not ctx.value


def test_T16_3d_limits_and_shared_memory(lib):
    cfg = S.make_config(3, (4096, 16, 16), (0.3, 0.3, 0.3), 0.1, [{"Z": -1, "mu": 1, "a": 0}])
    got, msg, _ = _init_status(lib, cfg)
    assert got == S.PIC_EINVAL and "n[0]" in msg
    cfg = S.make_config(3, (64, 64, 64), (0.3, 0.3, 0.3), 0.1, [{"Z": -1, "mu": 1, "a": 0}],
                        precision=S.PIC_FP64, tile=(16, 16, 16))
    got, msg, _ = _init_status(lib, cfg)
    assert got == S.PIC_EINVAL and "shared memory" in msg


def _one_particle(**cols):
    p = np.zeros((1, 10))
    p[0, :] = [1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.01]
    names = ("x", "y", "z", "ux", "uy", "uz", "sx", "sy", "sz", "w")
    for k, v in cols.items():
        p[0, names.index(k)] = v
    return p


@pytest.mark.parametrize("cols,needle", [
    ({"sy": 0.9}, "|s|"),
    ({"sx": 1.0}, "|s|"),
    ({"ux": math.nan}, "non-finite"),
    ({"x": math.inf}, "non-finite"),
    ({"w": math.nan}, "non-finite"),
])
def test_T16_init_rejects_bad_particles(lib, cols, needle):
    got, msg, _ = _init_status(lib, _good_cfg(), [_one_particle(**cols)])
    assert got == S.PIC_EINVAL, msg
    assert needle in msg


def test_T16_init_rejects_missing_particle_pointer(lib):
    cfg = _good_cfg()
    st = S.State()
    st.count[0] = 5
    st.particles[0] = None
    ctx = ctypes.c_void_p()
    assert lib.pic_init(ctypes.byref(cfg), ctypes.byref(st), None, None, ctypes.byref(ctx)) == S.PIC_EINVAL
    assert "NULL" in lib.pic_last_error(None).decode()
    assert lib.pic_init(None, None, None, None, ctypes.byref(ctx)) == S.PIC_EINVAL
    assert lib.pic_init(ctypes.byref(cfg), None, None, None, None) == S.PIC_EINVAL


def test_T16_calls_on_null_context(lib):
    P = np.zeros(3)
    N = ctypes.c_int64()
    assert lib.pic_step(None, 1) == S.PIC_ESTATE
    assert lib.pic_polarization(None, -1, 0.0, 1.0, P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.byref(N)) == S.PIC_ESTATE
    assert lib.pic_fields(None, 1, None, 0) == S.PIC_ESTATE
    assert lib.pic_energy(None, None, 0) == S.PIC_ESTATE
    assert lib.pic_stats(None, None, 0) == S.PIC_ESTATE
    assert lib.pic_spectrum(None, 0, 0.0, 1.0, 4, None, None, None) == S.PIC_ESTATE
    assert lib.pic_phase_space(None, 0, 0, 0.0, 1.0, 4, 0, -1.0, 1.0, 4, None) == S.PIC_ESTATE
    assert lib.pic_density(None, 0, None, 0) == S.PIC_ESTATE
    assert lib.pic_window(None, ctypes.byref(S.window_config())) == S.PIC_ESTATE
    n = ctypes.c_int32(7)
    assert lib.pic_polarization_record(None, -1, 0.0, 1.0, 16) == S.PIC_ESTATE
    assert lib.pic_polarization_history(None, None, None, 0, ctypes.byref(n)) == S.PIC_ESTATE
    lib.pic_free(None)


def test_binding_raises_when_library_missing(tmp_path):
    saved = S._lib
    try:
        S._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            S.load_library(str(tmp_path / "nope.so"))
    finally:
        S._lib = saved


def test_track_calls_validate_without_a_gpu(lib):
    P = ctypes.c_void_p()
    good = S.TrackConfig(1.0, 1836.15267343, 1.793, 0.5, 100, 10, S.PIC_FP32_MIXED)
    assert lib.pic_track_create(ctypes.byref(good), 10, None, None, None) == S.PIC_EINVAL
    assert lib.pic_track_create(None, 10, None, None, ctypes.byref(P)) == S.PIC_EINVAL
    bad = [
        (S.TrackConfig(1.0, 1836.15, 1.793, 0.5, 100, 10, S.PIC_FP32_MIXED), 0, "outside 1.."),
        (S.TrackConfig(1.0, 0.0, 1.793, 0.5, 100, 10, S.PIC_FP32_MIXED), 10, "mass"),
        (S.TrackConfig(1.0, 1836.15, 1.793, -0.5, 100, 10, S.PIC_FP32_MIXED), 10, "dt"),
        (S.TrackConfig(1.0, 1836.15, 1.793, 0.5, -1, 10, S.PIC_FP32_MIXED), 10, "nsteps"),
        (S.TrackConfig(1.0, 1836.15, 1.793, 0.5, 100, 0, S.PIC_FP32_MIXED), 10, "checkpoint"),
        (S.TrackConfig(1.0, 1836.15, 1.793, 0.5, 100, 10, 7), 10, "precision"),
    ]
    for cfg, n, needle in bad:
        assert lib.pic_track_create(ctypes.byref(cfg), n, None, None, ctypes.byref(P)) == S.PIC_EINVAL
        assert needle in lib.pic_track_last_error(None).decode()
    assert lib.pic_track_forward(None, 0.1, 0.1, None, None, None, None, None, None, None) == S.PIC_ESTATE
    assert lib.pic_track_backward(None, None, None, None, None, None, None) == S.PIC_ESTATE
    assert lib.pic_track_timing(None, None) == S.PIC_ESTATE
    lib.pic_track_free(None)


def _cell_row(**cols):
    p = np.zeros((1, 13))
    p[0, :] = [3.0, 2.0, 0.0, 0.25, 0.5, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.01]
    names = ("cx", "cy", "cz", "ox", "oy", "oz", "ux", "uy", "uz", "sx", "sy", "sz", "w")
    for k, v in cols.items():
        p[0, names.index(k)] = v
    return p


@pytest.mark.parametrize("cols,needle", [
    ({"cx": 32.0}, "cell outside"),      # the grid has 32 x 16 cells
    ({"cy": -1.0}, "cell outside"),
    ({"cx": 2.5}, "cell outside"),       # not a whole number
    ({"ox": 1.0}, "offset outside"),
    ({"oy": -0.1}, "offset outside"),
    ({"sy": 0.5}, "|s|"),
    ({"w": math.nan}, "non-finite"),
])
def test_T16_init_rejects_bad_cell_rows(lib, cols, needle):
    """Rows in cell form (PIC_FLAG_CELL_ROWS) are checked before the GPU is touched."""
    cfg = _good_cfg(flags=S.PIC_FLAG_CELL_ROWS | S.PIC_FLAG_DETERMINISTIC)
    got, msg, _ = _init_status(lib, cfg, [_cell_row(**cols)])
    assert got == S.PIC_EINVAL, msg
    assert needle in msg


def test_deterministic_and_cell_rows_not_in_batches(lib):
    cfg = _good_cfg(flags=S.PIC_FLAG_DETERMINISTIC)
    st = S.State()
    for s in range(S.MAX_SPECIES):
        st.count[s] = 0
        st.particles[s] = None
    b = ctypes.c_void_p()
    assert lib.pic_batch_init(1, ctypes.byref(cfg), ctypes.byref(st), 0, None, None, ctypes.byref(b)) == S.PIC_EINVAL
    assert "deterministic" in lib.pic_batch_last_error(None).decode()


def test_new_hooks_on_null_context(lib):
    N = ctypes.c_int64()
    assert lib.pic_particles_cells(None, 0, None, 0, ctypes.byref(N)) == S.PIC_ESTATE
    assert lib.pic_test_poison(None, 0) == S.PIC_ESTATE
    assert lib.pic_spectrum_noalloc(None, 0, 0.0, 1.0, 4, None, None, None) == S.PIC_ESTATE
