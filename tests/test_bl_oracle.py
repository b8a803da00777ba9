"""Pins of the FP64 BeamLearning oracle (paper section II.B) against what the
paper prints and what the mathematics fixes, independent of the oracle's own code."""
import json
import os

import numpy as np
import pytest
from scipy import integrate, signal

from oracle import beamlearning as bl
from paper_2104_13347_amd import bl_data

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "beamlearning_architecture.json")))


def _g(key):
    return GOLD[key]["value"]


def test_architecture_matches_printed_figures():
    # 3 x 768 cascaded filters: 18 layers of N_f outputs (overview of section II.B)
    n_mod, per_mod = _g("cascaded_filters")
    assert len(bl.layer_dilations()) * bl.N_F == n_mod * per_mod
    assert bl.N_MODULES == n_mod and len(bl.DILATIONS) * bl.N_F == per_mod
    assert list(bl.DILATIONS) == _g("dilations")
    assert bl.N_F == _g("n_f") and bl.MULT == _g("channel_multiplier")


def test_time_scales_match_receptive_field():
    # fs from a 1024-sample frame lasting 23.2 ms; the shortest time scale is one
    # kernel (3 samples), the longest the whole cascade's receptive field.
    fs = _g("n_t") / (_g("frame_ms") * 1e-3)
    lo, hi = _g("time_scales_s")
    rf = 2 * bl.valid_margin() + 1
    assert abs(bl.TAPS / fs - lo) < 0.5e-6 * 2      # 68 us printed to 2 digits
    assert abs(rf / fs - hi) < 0.05e-3              # 8.6 ms printed to 2 digits
    assert rf == 379 and _g("kernel_size") == bl.TAPS


def test_variable_count_near_printed():
    # about 1.1e6 variables (section V.D); the flat layout holds the same order.
    n = bl_data.param_count(_g("n_c"), 2)
    assert 1.05e6 <= n < 1.2e6, n


@pytest.mark.parametrize("dilation", [1, 2, 8, 32])
def test_depthwise_is_channelwise_correlation(dilation):
    # Special case reducing to a library routine: each (channel, multiplier)
    # output is the 'same' cross-correlation with the dilated (zero-stuffed) kernel.
    rng = np.random.default_rng(dilation)
    T, C = 97, 3
    x = rng.standard_normal((T, C))
    w = rng.standard_normal((C, bl.MULT, 3))
    z = bl.depthwise_conv(x, w, dilation)
    for c in range(C):
        for j in range(bl.MULT):
            k = np.zeros(2 * dilation + 1)
            k[0], k[dilation], k[2 * dilation] = w[c, j]
            ref = signal.correlate(x[:, c], k, mode="same", method="direct")
            np.testing.assert_allclose(z[:, c * bl.MULT + j], ref, rtol=0, atol=1e-12)


def test_separable_equals_rank_structured_dense_conv():
    # Brute force on a tiny case: a depthwise-separable layer is a dense
    # convolution whose kernel is K[o, c, k] = sum_j P[c*m + j, o] w[c, j, k].
    rng = np.random.default_rng(5)
    T, C, O, D = 23, 2, 5, 4
    x = rng.standard_normal((T, C))
    w = rng.standard_normal((C, bl.MULT, 3))
    P = rng.standard_normal((C * bl.MULT, O))
    b = rng.standard_normal(O)
    got = bl.pointwise_conv(bl.depthwise_conv(x, w, D), P, b)
    ref = np.zeros((T, O))
    for t in range(T):
        for o in range(O):
            s = b[o]
            for c in range(C):
                for k in range(3):
                    tt = t + (k - 1) * D
                    if 0 <= tt < T:
                        s += x[tt, c] * sum(P[c * bl.MULT + j, o] * w[c, j, k] for j in range(bl.MULT))
            ref[t, o] = s
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_layer_norm_invariants():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((50, 8)) * 3 + 1.5
    y = bl.layer_norm(a, np.ones(8), np.zeros(8), 0.0)
    assert abs(y.mean()) < 1e-13 and abs(y.var() - 1.0) < 1e-12
    # invariant to a positive scale and a common shift of its input
    np.testing.assert_allclose(bl.layer_norm(4.0 * a - 2.0, np.ones(8), np.zeros(8), 0.0), y, atol=1e-12)


def test_selu_fixed_point():
    # The SELU constants make N(0, 1) inputs map to zero mean, unit variance.
    phi = lambda z: np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)
    m = integrate.quad(lambda z: float(bl.selu(z)) * phi(z), -np.inf, np.inf, epsabs=1e-13)[0]
    v = integrate.quad(lambda z: float(bl.selu(z)) ** 2 * phi(z), -np.inf, np.inf, epsabs=1e-13)[0]
    assert abs(m) < 1e-9 and abs(v - 1.0) < 1e-9


def _small_params(seed, c_in=3, n_out=4, unit_gain=True):
    return bl_data.make_params(seed, c_in=c_in, n_out=n_out, unit_gain=unit_gain)


def test_receptive_field_and_centering():
    # With the layer norms bypassed and zero biases, zero maps to zero, so the
    # response to one impulse is nonzero exactly within +-189 samples of it:
    # kernel 3, dilations 1..32, three modules, non-causal centring.
    p = _small_params(11)
    for l in range(18):
        p[f"b{l}"] = np.zeros_like(p[f"b{l}"])
    T, t0 = 600, 300
    x = np.zeros((3, T))
    x[1, t0] = 1.0
    S = bl.filterbank(x, p, 1e-6, normalise=False)
    nz = np.nonzero(np.abs(S).max(axis=1) > 0)[0]
    assert nz.min() == t0 - 189 and nz.max() == t0 + 189


def test_time_reversal_symmetry():
    # The convolutions are centred ('same' padding): reversing the frame in time
    # and every kernel's taps reverses S, and the valid crop is symmetric, so the
    # features and outputs are unchanged.
    p = _small_params(12)
    q = dict(p)
    for l in range(18):
        q[f"dw{l}"] = p[f"dw{l}"][:, :, ::-1].copy()
    x = bl_data.frames(3, 1, c_in=3, n_t=420)[0]
    S1 = bl.filterbank(x, p, 1e-6)
    S2 = bl.filterbank(x[:, ::-1], q, 1e-6)
    np.testing.assert_allclose(S2[::-1], S1, atol=1e-12)
    f1, o1 = bl.forward(x[None], p)
    f2, o2 = bl.forward(x[None, :, ::-1], q)
    np.testing.assert_allclose(f2, f1, atol=1e-12)
    np.testing.assert_allclose(o2, o1, atol=1e-12)


def test_layer_scale_invariance():
    # Every layer is followed by a layer norm: scaling a layer's pointwise
    # weights and bias by a positive constant leaves the network unchanged (up
    # to the eps of the norm, taken as zero here).
    p = _small_params(13)
    q = dict(p)
    for l in (0, 7, 17):
        q[f"pw{l}"] = p[f"pw{l}"].astype(np.float64) * 3.0
        q[f"b{l}"] = p[f"b{l}"].astype(np.float64) * 3.0
    x = bl_data.frames(4, 2, c_in=3, n_t=400)
    f1, o1 = bl.forward(x, p, eps=0.0)
    f2, o2 = bl.forward(x, q, eps=0.0)
    np.testing.assert_allclose(f2, f1, atol=1e-11)
    np.testing.assert_allclose(o2, o1, atol=1e-11)


def test_pseudo_energy_crop_and_mean():
    # A filterbank output that is c on the valid samples and huge outside gives
    # pseudo-energy c^2 per channel: the crop keeps exactly [189, T - 189).
    T = 1024
    S = np.full((T, bl.N_F), 1e6)
    S[189:T - 189] = np.arange(bl.N_F)[None, :] * 0.5
    np.testing.assert_array_equal(bl.pseudo_energy(S), (np.arange(bl.N_F) * 0.5) ** 2)
    assert T - 2 * bl.valid_margin() == 646
    with pytest.raises(ValueError):
        bl.pseudo_energy(np.zeros((378, bl.N_F)))


def test_classification_output_is_distribution():
    p = _small_params(14, n_out=16)
    x = bl_data.frames(5, 3, c_in=3, n_t=400)
    _, o = bl.forward(x, p, mode=bl.MODE_CLASSIFICATION)
    assert np.all(o > 0)
    np.testing.assert_allclose(o.sum(axis=1), 1.0, atol=1e-14)
    # the regression head is the same affine map before the softmax
    _, r = bl.forward(x, p, mode=bl.MODE_REGRESSION)
    sm = np.exp(r - r.max(axis=1, keepdims=True))
    np.testing.assert_allclose(sm / sm.sum(axis=1, keepdims=True), o, atol=1e-14)
