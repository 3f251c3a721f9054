"""The benchmark's compulsory-traffic model, against counts by hand.

Each figure is the bytes one launch must move: every input array read once,
every output written once (8 B per FP64 value, cs per spectral value)."""
import bench

NX, NY, NZ = 8, 4, 6
N = NX * NY * NZ
NV = NX * (NY + 1) * NZ
NS = (NX // 2 + 1) * NY * NZ


def ab(k, prec=0, **kw):
    return bench.algorithmic_bytes(k, NX, NY, NZ, prec, **kw)


def test_right_hand_side_with_and_without_the_split_term():
    # u*, v* (faces), w*, rho, p^n, p^{n-1}, S read; b written
    assert ab("k_rhs") == 8 * (N + NV + N + N + N + N + N) + 8 * N
    # the constant part c of the Eq. (25) iteration: u*, v*, w*, S
    assert ab("k_rhs", ctx={"split": False}) == 8 * (N + NV + N + N) + 8 * N


def test_spectral_passes_per_precision():
    for prec, cs in ((0, 16), (1, 8)):
        assert ab("k_r2c", prec) == 8 * N + cs * NS
        assert ab("k_tri", prec) == ab("k_fft_z_fwd", prec) == ab("k_fft_z_inv", prec) == 2 * cs * NS
        assert ab("k_c2r", prec) == cs * NS + 8 * N
        assert ab("k_c2r", prec, mode_update=True) == cs * NS + 16 * N  # p read back
        # the refinement's row transform reads the residual in the spectrum's precision
        assert ab("k_r2c", prec, mode_update=True) == (cs // 2) * N + cs * NS


def test_refinement_residual_is_stored_in_the_spectrum_precision():
    # b, p read in FP64; r written in FP32 for FP32 spectra
    assert ab("k_resid", 1) == 16 * N + 4 * N
    assert ab("k_resid", 0) == 24 * N


def test_fixed_point_residual_first_and_later_sweeps():
    # c, rho, p -> r
    assert ab("k_resid_var") == 8 * 4 * N
    # c, rho, p^n, p^{n-1} -> r, p_0
    assert ab("k_resid_var", ctx={"first_frac": 1.0}) == 8 * 6 * N
    assert ab("k_resid_var", ctx={"first_frac": 0.25}) == 0.75 * 32 * N + 0.25 * 48 * N


def test_correction_with_separate_or_shared_pressures():
    out = 8 * (N + NV + N)
    assert ab("k_correct") == 8 * (N + NV + N + N + N + N + N + N) + out
    assert ab("k_correct", ctx={"p_aliased": True}) == 8 * (N + NV + N + N + N + N) + out


def test_predictor_components():
    reads = 8 * (N + NV + N + 6 * N)  # u, v, w, rho^n, rho^{n+1}, mu, C, sigma, kappa
    assert ab("k_predict_u") == ab("k_predict_w") == reads + 8 * N
    assert ab("k_predict_v") == reads + 8 * NV
    assert ab("k_predict") == ab("k_predict_u") + ab("k_predict_v") + ab("k_predict_w")
    extra = 8 * (N + NV + N)          # viscous-term velocities given separately
    assert ab("k_predict_u", ctx={"viscous_separate": True}) == reads + extra + 8 * N


def test_unknown_kernel_has_no_model():
    assert ab("k_finish") == 0.0
