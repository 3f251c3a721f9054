"""The C-ABI library loads and exports every entry point include/ppe.h declares.

CPU only: no compute call is made (no device here); descriptor validation in
ppe_plan_workspace_bytes is host logic and is exercised directly.
"""
import ctypes
import math
import os
import re

import pytest

from paper_2103_01874_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppe.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(ppe_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libppe.so not built")
    return binding.load()


def test_header_lists_the_api():
    names = declared_functions()
    for n in ("ppe_plan", "ppe_solve", "ppe_correct", "ppe_residual", "ppe_plan_destroy",
              "ppe_plan_workspace_bytes"):
        assert n in names
    assert sorted(binding.EXPORTS) == names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert lib.ppe_version().decode().startswith("ppe-mi355x")


def test_struct_layouts():
    assert ctypes.sizeof(binding.Desc) == 72
    assert binding.INFO_DTYPE.itemsize == 64


def ws(**kw):
    base = dict(nx=32, ny=32, nz=32)
    base.update(kw)
    return binding.workspace_bytes(binding.make_desc(**base))


def test_descriptor_validation(lib):
    assert ws() > 0
    assert ws(nx=5) == 0          # FFT length with a factor 5
    assert ws(nz=14) == 0         # factor 7
    assert ws(ny=1) == 0          # y needs two cells
    assert ws(nx=4096) == 0       # beyond the supported length
    assert ws(lx=0.0) == 0
    assert ws(lx=-1.0) == 0
    assert ws(ly=math.nan) == 0
    assert ws(precision=7) == 0
    assert ws(batch=0) == 0
    assert ws(batch=binding.MAX_BATCH + 1) == 0
    assert ws(max_refine=-1) == 0
    assert ws(tol=-1.0) == 0
    for n in (1, 2, 3, 6, 9, 12, 96, 192, 512, 2048):
        assert ws(nx=n, nz=n if n <= 512 else 8, ny=4) > 0, n


def test_workspace_accounts_for_precision_and_batch(lib):
    a = ws(nx=64, ny=32, nz=64)
    b = ws(nx=64, ny=32, nz=64, batch=4)
    m = ws(nx=64, ny=32, nz=64, precision=binding.PPE_PREC_MIXED)
    # half spectrum in 128-byte kx tiles: 33 columns -> 5 tiles of 8 (FP64) or 3 tiles of 16 (FP32)
    spec64 = 64 * 32 * 40 * 16
    spec32 = 64 * 32 * 48 * 8
    assert b > 3 * a
    # mixed: FP32 spectrum plus the refinement residual, stored in FP32
    assert m - a == spec32 - spec64 + 64 * 32 * 64 * 4


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No CPU fallback: without the built library every entry point raises."""
    from paper_2103_01874_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.PPEError, match="not built"):
        binding.load(str(tmp_path / "libppe.so"))


def test_y_refine_flag_adds_the_block_tables(lib):
    """PPE_FLAG_Y_REFINE: the plan also holds a byte per y-solve block and the
    list of blocks to refine; above 256 rows refinement is on regardless."""
    plain = ws(nx=64, ny=32, nz=64)
    flagged = ws(nx=64, ny=32, nz=64, flags=binding.PPE_FLAG_Y_REFINE)
    assert flagged > plain
    assert ws(nx=64, ny=512, nz=64, flags=binding.PPE_FLAG_Y_REFINE) == ws(nx=64, ny=512, nz=64)
    assert ws(flags=4) == 0 and ws(flags=binding.PPE_FLAG_VARCOEF | binding.PPE_FLAG_Y_REFINE) > 0


def test_residual_buffer_sizes(lib):
    """FP64 residual (8 B per cell) for the fixed-point iteration; a mixed plan
    without PPE_FLAG_VARCOEF holds only the FP32 residual of its refinement."""
    n = 32 * 32 * 32
    fp64 = ws()
    assert ws(flags=binding.PPE_FLAG_VARCOEF) - fp64 == 8 * n
    mixed = ws(precision=binding.PPE_PREC_MIXED)
    assert ws(precision=binding.PPE_PREC_MIXED, flags=binding.PPE_FLAG_VARCOEF) - mixed == 4 * n
    # FP32 spectra (half of FP64's, in 128-byte tiles) plus the 4-byte residual
    spec64 = 32 * 32 * 24 * 16   # 17 kx columns in tiles of 8
    spec32 = 32 * 32 * 32 * 8    # 17 kx columns in tiles of 16
    assert mixed - fp64 == spec32 - spec64 + 4 * n
