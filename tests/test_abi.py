"""The C-ABI library loads and exports what include/fe.h declares; host-side
validation rejects bad arguments before any device work (runs without a GPU)."""

import ctypes
import math
import os
import re

import pytest

from paper_2103_04856_amd import fe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fe.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fe.LIB_PATH):
        pytest.fail("libfe.so is not built: run python -m paper_2103_04856_amd.build")
    return fe.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert "fe_create" in names and "fe_step" in names and "fe_energy_grad" in names
    for n in names:
        assert hasattr(L, n), n
    # and the binding covers exactly the declared set
    assert sorted(fe.SIGNATURES) == names


def test_header_entry_points_have_documented_errors():
    text = open(HEADER).read()
    for code in ("FE_OK", "FE_EINVAL", "FE_EHIP", "FE_ENOMEM", "FE_ENONFINITE"):
        assert code in text


def test_variant_table(L):
    vs = fe.variants()
    assert len(vs) >= 4
    assert any(m & 1 for *_, m in vs) and any(m & 2 for *_, m in vs)
    for tx, ty, nt, m in vs:
        assert nt % 64 == 0 and nt <= 1024 and tx * ty >= nt // 2
    bad = ctypes.c_int()
    assert L.fe_variant_info(len(vs), ctypes.byref(bad), None, None, None) == fe.FE_EINVAL


def _create(L, grid, eps, coeffs):
    out = ctypes.c_void_p()
    rc = L.fe_create(ctypes.byref(grid) if grid is not None else None,
                     fe._dbl(eps) if eps is not None else None,
                     fe._dbl(coeffs) if coeffs is not None else None, None, ctypes.byref(out))
    return rc, out, L.fe_last_error().decode()


GOOD = dict(nx=8, ny=8, nz=8, batch=1, h=0.125, dtype=0)


@pytest.mark.parametrize("field,value,msg", [
    ("nx", 0, "grid sizes"), ("nz", -3, "grid sizes"), ("batch", 0, "batch"),
    ("h", 0.0, "h must"), ("h", float("nan"), "h must"), ("dtype", 7, "dtype"),
])
def test_create_rejects_bad_grid(L, field, value, msg):
    g = dict(GOOD)
    g[field] = value
    rc, out, err = _create(L, fe.FeGrid(**g), [0.25], [1, 2, 1, 0, 0, 0])
    assert rc == fe.FE_EINVAL and not out.value and msg in err


@pytest.mark.parametrize("nx,ny,dtype", [(40000, 30000, 0), (30000, 20000, 1)])
def test_create_rejects_planes_of_4_gib(L, nx, ny, dtype):
    rc, out, err = _create(L, fe.FeGrid(nx=nx, ny=ny, nz=1, batch=1, h=0.125, dtype=dtype), [0.25],
                           [1, 2, 1, 0, 0, 0])
    assert rc == fe.FE_EINVAL and not out.value and "too large" in err


@pytest.mark.parametrize("eps,coeffs,msg", [
    ([0.0], [1, 2, 1, 0, 0, 0], "eps[0]"),
    ([-1.0], [1, 2, 1, 0, 0, 0], "eps[0]"),
    ([math.inf], [1, 2, 1, 0, 0, 0], "eps[0]"),
    ([0.25], [1, 2, math.nan, 0, 0, 0], "p_coeffs[0][2]"),
    ([0.25], [1, 2, 1, 0, 0, math.inf], "p_coeffs[0][5]"),
])
def test_create_rejects_bad_params(L, eps, coeffs, msg):
    rc, out, err = _create(L, fe.FeGrid(**GOOD), eps, coeffs)
    assert rc == fe.FE_EINVAL and msg in err


def test_create_rejects_null_pointers(L):
    rc, _, err = _create(L, None, [0.25], [1, 2, 1, 0, 0, 0])
    assert rc == fe.FE_EINVAL and "grid" in err
    rc, _, err = _create(L, fe.FeGrid(**GOOD), None, None)
    assert rc == fe.FE_EINVAL and "NULL" in err
    assert L.fe_create(ctypes.byref(fe.FeGrid(**GOOD)), fe._dbl([0.25]), fe._dbl([0] * 6), None, None) == fe.FE_EINVAL


def test_calls_on_null_context_fail_cleanly(L):
    assert L.fe_energy_grad(None, None, None, None) == fe.FE_EINVAL
    assert L.fe_grad_scaled_async(None, None, None, None) == fe.FE_EINVAL
    assert L.fe_step(None, None, None, 1e-3, 1, None) == fe.FE_EINVAL
    assert L.fe_set_launch(None, 0, 0) == fe.FE_EINVAL
    assert L.fe_hminus_step(None, None, None, 2.0, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == fe.FE_EINVAL
    assert L.fe_hminus_reset(None) == fe.FE_EINVAL
    assert L.fe_diagnostics(None, None, None, None, 8, 10.0, None) == fe.FE_EINVAL
    L.fe_destroy(None)   # no-op


@pytest.mark.parametrize("grid,sigma_k,msg", [
    (dict(GOOD, batch=2), 1.0, "batch 1"),
    (GOOD, -1.0, "sigma_k"),
    (GOOD, 4.5, "sigma_k"),
    (dict(GOOD, nx=40000, ny=40000, nz=1), 0.0, "too large"),   # padded planes of 6.4 GB
    (dict(GOOD, nx=4, ny=70000, nz=4), 0.0, "too large"),       # padded ny beyond a grid dimension
])
def test_l2_create_rejects_before_device_work(L, grid, sigma_k, msg):
    out = ctypes.c_void_p()
    rc = L.fe_l2_create(ctypes.byref(fe.FeGrid(**grid)), 0.25, fe._dbl([1, 2, 1, 0, 0, 0]), sigma_k, None,
                        ctypes.byref(out))
    assert rc == fe.FE_EINVAL and not out.value and msg in L.fe_last_error().decode()


@pytest.mark.parametrize("grid,msg", [
    (dict(GOOD, batch=17), "16"),
    (dict(GOOD, nx=8192, ny=8192, nz=1), "partials"),   # 256 x 256 tile columns
    (dict(GOOD, nx=0), "grid sizes"),
])
def test_noalloc_rejects_before_device_work(L, grid, msg):
    """The allocation-free entry point checks its limits (batch <= 16, the block partials
    its static array holds) on the host, before it looks up the array or launches."""
    B = grid["batch"]
    rc = L.fe_energy_grad_noalloc(ctypes.byref(fe.FeGrid(**grid)), fe._dbl([0.25] * B),
                                  fe._dbl([1, 2, 1, 0, 0, 0] * B), ctypes.c_void_p(8), ctypes.c_void_p(16),
                                  None, None)
    assert rc == fe.FE_EINVAL and msg in L.fe_last_error().decode()


def test_tune_cache_file_round_trip(L, tmp_path):
    """The autotuner's cache file: a saved record loads back unchanged; a malformed line or
    an unknown variant is rejected and nothing is merged (host only, no device work)."""
    L.fe_tune_cache_clear()
    good = tmp_path / "good.txt"
    good.write_text("64x64x64x1:f32:step:nos:-:gfx950 0 32 12.500000\n")
    assert L.fe_tune_cache_load(str(good).encode()) == fe.FE_OK
    out = tmp_path / "out.txt"
    assert L.fe_tune_cache_save(str(out).encode()) == fe.FE_OK
    assert out.read_text() == good.read_text()
    for bad in ("not a record\n", f"k 0 1 2.0\nk2 {L.fe_num_variants()} 4 1.0\n", "k -1 4 1.0\n"):
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        assert L.fe_tune_cache_load(str(p).encode()) == fe.FE_EINVAL
    L.fe_tune_cache_clear()
    assert L.fe_tune_cache_save(str(out).encode()) == fe.FE_OK and out.read_text() == ""
    assert L.fe_tune_cache_load(str(tmp_path / "missing.txt").encode()) == fe.FE_EINVAL
