"""FP64 CPU oracle for the BeamLearning forward pass (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product library never loads it and
shares no code with it.  Plain numpy in FP64, written from paper section II.B:

* II.B.1 and the filterbank figure: three stacked modules of six layers; each
  layer is a non-causal depthwise convolution (kernel 3, dilation D = 1, 2, 4,
  8, 16, 32, channel multiplier 4), a pointwise (1x1) convolution onto
  N_f = 128 channels, a layer norm and a tanh; residual connections join the
  successive layers of all three modules.
* II.B.2: the filterbank output S[i, n] is squared, cropped to the time
  samples that are valid for every atrous layer, averaged over time, layer
  normalised and passed through a SELU.
* II.B.3: a fully connected layer maps the N_f pseudo-energies to the output
  (a unit-vector projection for regression; class probabilities, here a
  softmax, for classification).

Readings where the paper leaves a choice (each also listed with the design
notes): convolutions use zero padding to the input length ('same'); the
layer norm of a filterbank layer takes its statistics over the whole
N_t x N_f map of one frame, with a gain and an offset per filter channel; the
residual adds a layer's input to its activated output (x_{l+1} = x_l +
tanh(LN(a_l))) for every layer whose input has N_f channels, i.e. all but
the first; the pointwise convolution carries the layer's only bias; the
average pool spans every valid time sample.
"""
from __future__ import annotations

import numpy as np

N_F = 128
MULT = 4
TAPS = 3
DILATIONS = (1, 2, 4, 8, 16, 32)   # one filterbank module (filterbank figure)
N_MODULES = 3

# SELU constants (Klambauer et al., self-normalising networks): the unique
# (alpha, lambda) for which a standard normal input keeps zero mean, unit variance.
SELU_ALPHA = 1.6732632423543772848170429916717
SELU_LAMBDA = 1.0507009873554804934193349852946

MODE_REGRESSION = 0
MODE_CLASSIFICATION = 1


def layer_dilations():
    """Dilation of each of the 18 layers, modules in cascade."""
    return [d for _ in range(N_MODULES) for d in DILATIONS]


def valid_margin():
    """Samples lost at each end by the valid crop (II.B.2): the sum of the
    one-sided reach (k - 1) * D over all layers."""
    return sum((TAPS - 1) // 2 * d for d in layer_dilations())


def depthwise_conv(x, w, dilation):
    """Non-causal depthwise atrous convolution (II.B.1).

    x: [T, C]; w: [C, MULT, TAPS].  z[t, c*MULT + j] = sum_k w[c, j, k] *
    x[t + (k - 1) * dilation, c], with x = 0 outside [0, T).
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    T, C = x.shape
    half = (TAPS - 1) // 2 * dilation
    xp = np.zeros((T + 2 * half, C))
    xp[half:half + T] = x
    z = np.zeros((T, C, w.shape[1]))
    for k in range(TAPS):
        s = k * dilation
        z += xp[s:s + T, :, None] * w[None, :, :, k]
    return z.reshape(T, C * w.shape[1])


def pointwise_conv(z, p, b):
    """1x1 convolution onto N_f channels (II.B.1): a[t, o] = sum_i z[t, i] p[i, o] + b[o]."""
    return np.asarray(z, np.float64) @ np.asarray(p, np.float64) + np.asarray(b, np.float64)


def layer_norm(a, gain, offset, eps):
    """Layer norm (Ba et al.): statistics over every element of `a`, then a per-
    last-axis gain and offset."""
    a = np.asarray(a, np.float64)
    mu = a.mean()
    var = ((a - mu) ** 2).mean()
    return (a - mu) / np.sqrt(var + eps) * np.asarray(gain, np.float64) + np.asarray(offset, np.float64)


def selu(v):
    v = np.asarray(v, np.float64)
    return SELU_LAMBDA * np.where(v > 0, v, SELU_ALPHA * np.expm1(np.minimum(v, 0.0)))


def filterbank(x, params, eps, normalise=True):
    """The three cascaded filterbank modules (II.B.1) on one frame.

    x: [c_in, T] raw multichannel waveform.  Returns S as [T, N_f].
    normalise=False replaces each layer norm by the identity (only used to
    expose the network's receptive field in tests).
    """
    h = np.asarray(x, np.float64).T
    for l, d in enumerate(layer_dilations()):
        a = pointwise_conv(depthwise_conv(h, params[f"dw{l}"], d), params[f"pw{l}"], params[f"b{l}"])
        if normalise:
            a = layer_norm(a, params[f"g{l}"], params[f"be{l}"], eps)
        y = np.tanh(a)
        h = y if l == 0 else h + y
    return h


def pseudo_energy(S):
    """II.B.2 before its layer norm: square, keep the valid time samples, average over time."""
    m = valid_margin()
    T = S.shape[0]
    if T - 2 * m < 1:
        raise ValueError("frame shorter than the network's receptive field")
    return (np.asarray(S, np.float64)[m:T - m] ** 2).mean(axis=0)


def head(e, params, eps, mode):
    """Layer norm + SELU of the pseudo-energies (II.B.2), then the fully
    connected output (II.B.3).  Returns (features, output)."""
    f = selu(layer_norm(e, params["g_e"], params["be_e"], eps))
    o = f @ np.asarray(params["fc_w"], np.float64) + np.asarray(params["fc_b"], np.float64)
    if mode == MODE_CLASSIFICATION:
        o = np.exp(o - o.max())
        o = o / o.sum()
    return f, o


def forward(frames, params, eps=1e-6, mode=MODE_REGRESSION):
    """Forward pass over a batch of frames [B, c_in, T].

    Returns (features [B, N_f], outputs [B, n_out]) in FP64.
    """
    frames = np.asarray(frames)
    feats, outs = [], []
    for x in frames:
        f, o = head(pseudo_energy(filterbank(x, params, eps)), params, eps, mode)
        feats.append(f)
        outs.append(o)
    n_out = np.asarray(params["fc_b"]).shape[0]
    return (np.array(feats).reshape(len(frames), N_F), np.array(outs).reshape(len(frames), n_out))
