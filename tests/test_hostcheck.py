"""CPU checks of the kernels' stage code (FFT stages, y-tridiagonal chunks).

libppe_hostcheck.so drives the same __host__ __device__ stage functions the
HIP kernels execute, thread by thread with the kernels' barrier placement.
Expected values come from numpy's FFT and a dense numpy solve.
"""
import ctypes
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_2103_01874_amd", "libppe_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIB):
        pytest.skip("libppe_hostcheck.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.hc_fft.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    lib.hc_tri.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp]
    lib.hc_tri_refined.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp]
    lib.hc_fft_plan.argtypes = [ctypes.c_int, ip, ip, ip, ip]
    lib.hc_twiddles.argtypes = [ctypes.c_int, dp]
    lib.hc_fft_ct.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    lib.hc_ct_plan_check.argtypes = [ctypes.c_int]
    lib.hc_fftz_pair_map.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


SIZES = [1, 2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 27, 32, 36, 48, 64, 96, 128, 192, 256, 384, 512, 1024, 2048]


@pytest.mark.parametrize("n", SIZES)
def test_fft_stages_match_numpy(hc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xin = np.ascontiguousarray(np.stack([x.real, x.imag], -1).ravel())
    out = np.zeros(2 * n)
    assert hc.hc_fft(n, -1, _p(xin), _p(out)) == 0
    y = out[0::2] + 1j * out[1::2]
    assert np.abs(y - np.fft.fft(x)).max() < 1e-14 * np.sqrt(n) * np.abs(x).sum() / np.sqrt(n) + 1e-15
    assert hc.hc_fft(n, +1, _p(xin), _p(out)) == 0
    y = out[0::2] + 1j * out[1::2]
    assert np.abs(y - n * np.fft.ifft(x)).max() < 1e-14 * np.abs(x).sum() + 1e-15


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 96, 192, 384])
def test_compile_time_plans_equal_the_host_plans(hc, n):
    """Power-of-two lengths and 96, 192, 384 run with compile-time stage
    tables: the same stages as the host factorisation, and bit for bit the
    same transform."""
    assert hc.hc_ct_plan_check(n) == 0
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xin = np.ascontiguousarray(np.stack([x.real, x.imag], -1).ravel())
    for d in (-1, +1):
        a, b = np.zeros(2 * n), np.zeros(2 * n)
        assert hc.hc_fft(n, d, _p(xin), _p(a)) == 0
        assert hc.hc_fft_ct(n, d, _p(xin), _p(b)) == 0
        assert np.array_equal(a, b)
    y = b[0::2] + 1j * b[1::2]
    assert np.abs(y - n * np.fft.ifft(x)).max() < 1e-14 * np.abs(x).sum() + 1e-15
    assert hc.hc_fft_ct(48, -1, _p(xin), _p(b)) != 0 and hc.hc_ct_plan_check(48) != 0


def test_fft_rejects_other_primes(hc):
    e, tc, nst = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rad = (ctypes.c_int * 16)()
    for n in (5, 7, 10, 14, 25, 4096):
        assert hc.hc_fft_plan(n, ctypes.byref(e), ctypes.byref(tc), ctypes.byref(nst), rad) != 0
    assert hc.hc_fft_plan(192, ctypes.byref(e), ctypes.byref(tc), ctypes.byref(nst), rad) == 0
    assert (e.value, tc.value, list(rad)[: nst.value]) == (12, 16, [3, 4, 4, 4])


def test_twiddles_accurate(hc):
    for n in (6, 96, 512):
        w = np.zeros(2 * n)
        hc.hc_twiddles(n, _p(w))
        # reference in extended precision (x87 long double), rounded once
        pi_ld = np.arctan(np.longdouble(1)) * 4
        a = 2 * pi_ld * np.arange(n, dtype=np.longdouble) / n
        assert np.abs(w[0::2] - np.cos(a).astype(np.float64)).max() <= 1.2e-16
        assert np.abs(w[1::2] + np.sin(a).astype(np.float64)).max() <= 1.2e-16


def _dense(ny, s):
    A = np.diag(np.full(ny, -2.0 - s)) + np.diag(np.ones(ny - 1), 1) + np.diag(np.ones(ny - 1), -1)
    A[0, 0] = A[-1, -1] = -1.0 - s
    return A


@pytest.mark.parametrize("ny,P", [(2, 1), (3, 1), (5, 2), (8, 1), (8, 4), (32, 4), (64, 8), (96, 12),
                                  (128, 16), (256, 32), (255, 32), (100, 7), (16, 1)])
@pytest.mark.parametrize("s", [1e-6, 0.37, 25.0])
def test_tri_chunks_match_dense(hc, ny, P, s):
    rng = np.random.default_rng(ny * 31 + P)
    rhs = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    rin = np.ascontiguousarray(np.stack([rhs.real, rhs.imag], -1).ravel())
    out = np.zeros(2 * ny)
    assert hc.hc_tri(ny, P, s, 0, _p(rin), _p(out)) == 0
    x = out[0::2] + 1j * out[1::2]
    want = np.linalg.solve(_dense(ny, s), rhs)
    cond = np.linalg.cond(_dense(ny, s))
    assert np.abs(x - want).max() <= 1e-15 * cond * np.abs(want).max() * 10


@pytest.mark.parametrize("ny,P", [(4, 2), (32, 4), (96, 12), (256, 32)])
def test_tri_zero_mode_pin_and_gauge(hc, ny, P):
    rng = np.random.default_rng(ny)
    rhs = rng.standard_normal(ny)
    rhs -= rhs.mean()
    rin = np.ascontiguousarray(np.stack([rhs, 0 * rhs], -1).ravel())
    out = np.zeros(2 * ny)
    assert hc.hc_tri(ny, P, 0.0, 1, _p(rin), _p(out)) == 0
    x = out[0::2]
    A = _dense(ny, 0.0)
    assert abs(x.mean()) < 1e-12 * np.abs(x).max()
    assert np.abs(A @ x - rhs).max() < 1e-14 * np.abs(A).max() * np.abs(x).max()
    ls = np.linalg.lstsq(A, rhs, rcond=None)[0]
    assert np.abs(x - (ls - ls.mean())).max() < 1e-9 * np.abs(x).max()


@pytest.mark.parametrize("ny,P", [(2, 1), (3, 1), (5, 2), (8, 4), (64, 8), (128, 16), (255, 32), (100, 7)])
@pytest.mark.parametrize("s", [0.0, 1e-6, 0.37, 25.0])
def test_tri_outflow_top_matches_dense(hc, ny, P, s):
    """Outflow top row: p = 0 on the top face, ghost -x_{ny-1}, so the last
    diagonal entry is -3 - s; the system is regular even at s = 0."""
    rng = np.random.default_rng(ny * 37 + P)
    rhs = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    rin = np.ascontiguousarray(np.stack([rhs.real, rhs.imag], -1).ravel())
    out = np.zeros(2 * ny)
    assert hc.hc_tri(ny, P, s, 2, _p(rin), _p(out)) == 0
    x = out[0::2] + 1j * out[1::2]
    A = _dense(ny, s)
    A[-1, -1] = -3.0 - s
    want = np.linalg.solve(A, rhs)
    cond = np.linalg.cond(A)
    assert np.abs(x - want).max() <= 1e-15 * cond * np.abs(want).max() * 10


def test_tri_rejects_pin_with_outflow(hc):
    rin = np.zeros(16)
    out = np.zeros(16)
    assert hc.hc_tri(8, 2, 0.0, 3, _p(rin), _p(out)) == -1


def _eigen_solve(rhs, s, outflow):
    """x_{j-1} - (2 + s) x_j + x_{j+1} = rhs with the scaled end rows, by its
    eigenvectors: cosines of (j + 1/2) k pi / ny (DCT-II, zero-flux ends,
    eigenvalues -4 sin^2(k pi / 2 ny) - s) or of (j + 1/2)(k + 1/2) pi / ny
    (DCT-IV, p = 0 on the top face, eigenvalues -4 sin^2((2k + 1) pi / 4 ny) - s).
    Accurate to a few eps for every mode, the smoothest included."""
    import scipy.fft as sf
    ny = len(rhs)
    t = 4 if outflow else 2
    k = np.arange(ny)
    lam = -4 * np.sin(np.pi * ((2 * k + 1) / (4 * ny) if outflow else k / (2 * ny))) ** 2 - s
    return sf.idct(sf.dct(rhs, type=t, norm="ortho") / lam, type=t, norm="ortho")


@pytest.mark.parametrize("ny,P", [(2048, 128), (2047, 128), (1000, 125), (256, 32), (64, 8)])
@pytest.mark.parametrize("s,outflow", [(0.0, 1), (1e-7, 0), (1e-7, 1), (1e-3, 0), (0.37, 1)])
@pytest.mark.parametrize("smooth", [False, True])
def test_tri_refinement_reaches_eps_on_near_singular_systems(hc, ny, P, s, outflow, smooth):
    """The elimination alone leaves ~4 eps / lambda_min on the smooth modes
    (lambda_min = s, or s + 4 sin^2(pi / 4 ny) with the outflow top): up to
    1e-10 here.  One correction solve of the difference-form residual brings
    every case to a few eps against the eigenvector solve."""
    rng = np.random.default_rng(ny + P)
    if smooth:
        yv = (np.arange(ny) + 0.5) / ny
        rhs = (np.cos(np.pi * yv) + 0.3 * np.sin(5 * np.pi * yv) + 0.2) * (1 + 0.5j)
    else:
        rhs = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    rin = np.ascontiguousarray(np.stack([rhs.real, rhs.imag], -1).ravel())
    want = _eigen_solve(rhs.real, s, outflow) + 1j * _eigen_solve(rhs.imag, s, outflow)
    plain, ref = np.zeros(2 * ny), np.zeros(2 * ny)
    assert hc.hc_tri(ny, P, s, 2 * outflow, _p(rin), _p(plain)) == 0
    assert hc.hc_tri_refined(ny, P, s, 2 * outflow, _p(rin), _p(ref)) == 0
    err = lambda o: np.linalg.norm(o[0::2] + 1j * o[1::2] - want) / np.linalg.norm(want)
    print(f"ny={ny} s={s} outflow={outflow}: plain {err(plain):.2e} refined {err(ref):.2e}")
    assert err(ref) <= 2e-15
    assert err(plain) <= 1e-15 + 50 * 2.2e-16 / (s + 4 * np.sin(np.pi / (4 * ny)) ** 2 * outflow)


def test_tri_refinement_rejects_the_pinned_system(hc):
    rin = np.zeros(16)
    out = np.zeros(16)
    assert hc.hc_tri_refined(8, 2, 0.0, 1, _p(rin), _p(out)) == -1


@pytest.mark.parametrize("gx", [8, 16, 64, 96, 256])
@pytest.mark.parametrize("gy", [1, 2, 3, 17, 18, 33])
def test_fftz_pair_order_is_a_permutation_with_paired_halves(hc, gx, gy):
    """The z transform's FP32 block order visits every (j, by) once, and the
    two halves of each tile row sit 8 linear indices apart (one XCD)."""
    n = gx * gy
    j = np.zeros(n, dtype=np.int32)
    by = np.zeros(n, dtype=np.int32)
    hc.hc_fftz_pair_map(gx, gy, j.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                        by.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    assert np.all((j >= 0) & (j < gx) & (by >= 0) & (by < gy))
    key = by.astype(np.int64) * gx + j
    assert np.array_equal(np.sort(key), np.arange(n))
    where = np.empty(n, dtype=np.int64)
    where[key] = np.arange(n)
    for t in range(gy // 2):
        a, b = where[(2 * t) * gx + np.arange(gx)], where[(2 * t + 1) * gx + np.arange(gx)]
        assert np.array_equal(b, a + 8)
