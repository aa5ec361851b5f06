"""Pins for the oracle's FP8-E4M3 reading (CPU only).

The FP8 path quantises each GEMM input with a static per-tensor scale s: the
operand is stored as round_e4m3(x / s) and its value is s * that code, with s
the smallest power of two that brings the tensor's largest magnitude inside
the E4M3 range (448).  The checks below hold the oracle's pieces to that
definition by other means: the scale against a brute-force search over powers
of two (no logarithms), the quantiser against torch's float8_e4m3fn cast,
exact round trips of powers of two, the relative error bound of a 4-bit
significand (which a scale applied on the wrong side or an exponent rounded
the wrong way would break by orders of magnitude), and the calibration script
against the same search over the oracle's own activations.
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import calibrate_fp8, encoder
from oracle.numerics import round_e4m3
from synth.configs import TINY

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def smallest_pow2_scale(amax: float) -> float:
    """Brute force: walk k upward from far below and return the first 2**k
    with amax / 2**k <= 448 (exact comparisons, no log2)."""
    if amax <= 0.0:
        return 1.0
    for k in range(-300, 300):
        s = 2.0 ** k
        if amax / s <= 448.0:
            return s
    raise AssertionError("no scale found")


def _amax_cases():
    rng = np.random.default_rng(3)
    vals = list(np.exp(rng.uniform(-30, 30, 400)))
    for k in range(-20, 21):
        t = 448.0 * 2.0 ** k
        vals += [t, np.nextafter(t, 0.0), np.nextafter(t, np.inf), 2.0 ** k, 3.0 * 2.0 ** k]
    return vals


def test_power_of_two_scale_is_the_smallest_that_fits():
    for amax in _amax_cases():
        s = encoder.power_of_two_scale(float(amax))
        m, _ = np.frexp(s)
        assert m == 0.5, (amax, s)                      # a power of two
        assert amax / s <= 448.0, (amax, s)              # fits the E4M3 range
        assert amax / (s / 2.0) > 448.0, (amax, s)       # and no smaller one does
        assert s == smallest_pow2_scale(float(amax)), amax
    assert encoder.power_of_two_scale(0.0) == 1.0


def test_gemm_input_equals_scaled_torch_cast():
    rng = np.random.default_rng(4)
    u32 = np.concatenate([rng.uniform(-448, 448, 4000), rng.normal(0, 0.05, 2000),
                          [0.0, 448.0, -448.0, 2.0 ** -9, 3 * 2.0 ** -10]]).astype(np.float32)
    code = torch.from_numpy(u32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    for s in (2.0 ** -7, 2.0 ** -3, 1.0, 2.0 ** 5):
        x = u32.astype(np.float64) * s                    # exact: s is a power of two
        prec = encoder.Precision("fp8", act_scales=[[s, 2 * s, 4 * s, 8 * s]])
        np.testing.assert_array_equal(prec.gemm_in(x, 0, 0), s * code)
        np.testing.assert_array_equal(prec.gemm_in(2 * x, 0, 1), 2 * s * code)


def test_gemm_weight_uses_its_own_amax_and_the_torch_cast():
    rng = np.random.default_rng(5)
    prec = encoder.Precision("fp8")
    for sd in (0.02, 0.3, 7.0):
        w = rng.normal(0, sd, (64, 96))
        s = smallest_pow2_scale(float(np.abs(w).max()))
        code = torch.from_numpy(w / s).to(torch.float8_e4m3fn).to(torch.float64).numpy()
        got = prec.gemm_w(w)
        np.testing.assert_array_equal(got, s * code)
        # the scale puts the largest weight in the top binade of the range
        assert 224.0 < np.abs(w).max() / s <= 448.0


def test_quantisation_error_is_that_of_a_four_bit_significand():
    """|q(x) - x| <= 2**-4 |x| on normal codes: a scale on the wrong side, or a
    scale that is off by a power of two, breaks this on every tensor."""
    rng = np.random.default_rng(6)
    for sd in (1e-3, 0.1, 1.0, 50.0):
        x = rng.normal(0, sd, 5000)
        s = smallest_pow2_scale(float(np.abs(x).max()))
        prec = encoder.Precision("fp8", act_scales=[[s] * 4])
        q = prec.gemm_in(x, 0, 2)
        normal = np.abs(x / s) >= 2.0 ** -6
        assert (np.abs(q - x)[normal] <= 2.0 ** -4 * np.abs(x)[normal]).all()
        qw = prec.gemm_w(x.reshape(50, 100)).reshape(-1)
        assert (np.abs(qw - x)[normal] <= 2.0 ** -4 * np.abs(x)[normal]).all()


def test_powers_of_two_round_trip_exactly():
    ks = np.arange(-6, 4)
    w = np.array([sg * 2.0 ** k for k in ks for sg in (1.0, -1.0)]).reshape(4, 5)
    # amax 8: s = 2**-5, w/s spans 2**-1 .. 2**8, all E4M3 codes
    assert encoder.power_of_two_scale(8.0) == 2.0 ** -5
    np.testing.assert_array_equal(encoder.Precision("fp8").gemm_w(w), w)
    prec = encoder.Precision("fp8", act_scales=[[2.0 ** -5] * 4])
    np.testing.assert_array_equal(prec.gemm_in(w, 0, 3), w)
    np.testing.assert_array_equal(round_e4m3(w / 2.0 ** -5) * 2.0 ** -5, w)


def test_scaled_product_is_the_product_of_codes_times_both_scales():
    """The GPU multiplies E4M3 codes and scales the FP32 sum by sa * sw; the
    oracle multiplies the dequantised operands.  Both are the same number."""
    rng = np.random.default_rng(9)
    x, w = rng.normal(0, 2.0, (8, 64)), rng.normal(0, 0.02, (64, 16))
    sa = smallest_pow2_scale(float(np.abs(x).max()))
    sw = smallest_pow2_scale(float(np.abs(w).max()))
    prec = encoder.Precision("fp8", act_scales=[[sa] * 4])
    qa = torch.from_numpy(x / sa).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    qw = torch.from_numpy(w / sw).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_allclose(prec.gemm_in(x, 0, 0) @ prec.gemm_w(w), sa * sw * (qa @ qw), rtol=1e-13, atol=0)


def test_calibration_takes_the_smallest_fitting_scale_of_each_gemm_input():
    W = synth.make_weights(TINY, 0)
    scales, _ = calibrate_fp8.calibrate(TINY, W, ("uniform", 16, 128), n_records=8, seed=calibrate_fp8.CAL_SEED)
    rb = synth.generate_records(8, ("uniform", 16, 128), TINY.n_types, TINY.vocab, calibrate_fp8.CAL_SEED)
    taps: dict = {}
    encoder.hidden_states(W, TINY, rb.ids, rb.cu_seqlens, encoder.Precision("pure"), taps=taps)
    for l in range(TINY.n_layers):
        t = taps[l]
        want = [smallest_pow2_scale(float(np.abs(t[k]).max())) for k in ("x_in", "attn", "x_mid", "ffn1")]
        assert scales[l] == want


@pytest.mark.parametrize("name", ["tiny_fp8", "large_fp8"])
def test_committed_scales_are_powers_of_two_in_layer_order(name):
    with open(os.path.join(GOLDEN, f"fp8_scales_{name}.json")) as f:
        sc = json.load(f)
    wl = synth.workload(name)
    arr = np.asarray(sc["scales"], np.float64)
    assert arr.shape == (wl.model.n_layers, 4)
    m, _ = np.frexp(arr)
    assert (m == 0.5).all()
    assert "oracle/calibrate_fp8.py" in sc["source"]
