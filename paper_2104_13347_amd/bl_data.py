"""Seeded synthetic inputs for the BeamLearning forward pass (inputs only).

The network of paper section II.B has no published weights, so its variables
are drawn the way the paper initialises them before training (section II.B,
training procedure: a centred normal truncated at two standard deviations,
standard deviation 0.1).  Input frames are raw multichannel waveforms of
N_t samples.  This module holds shapes, the flat parameter layout and random
draws only; none of the network's arithmetic.  Both the GPU library and the
FP64 oracle receive what it returns.

Flat parameter layout (FP32, in this order; the layout the C-ABI reads):
for each layer l = 0 .. 17 (C = c_in for l = 0, else N_f = 128):
    dw{l}  [C][4][3]    depthwise taps: channel, multiplier, tap (tap k at
                        time offset (k - 1) * D)
    pw{l}  [4C][128]    pointwise weights, depthwise output c*4 + j first
    b{l}   [128]        pointwise bias
    g{l}   [128]        layer-norm gain (per filter channel)
    be{l}  [128]        layer-norm offset
then the head:
    g_e    [128], be_e [128]   layer norm of the pseudo-energies
    fc_w   [128][n_out], fc_b [n_out]   fully connected output layer
"""
from __future__ import annotations

import numpy as np

N_F = 128          # filter channels per layer (section II.B.1)
MULT = 4           # depthwise channel multiplier
N_LAYERS = 18      # three filterbank modules of six layers
TAPS = 3           # kernel size of every atrous convolution


def layer_cin(layer: int, c_in: int) -> int:
    return c_in if layer == 0 else N_F


def param_shapes(c_in: int, n_out: int):
    """Ordered (name, shape) list of the flat parameter blob."""
    out = []
    for l in range(N_LAYERS):
        ci = layer_cin(l, c_in)
        out += [(f"dw{l}", (ci, MULT, TAPS)), (f"pw{l}", (ci * MULT, N_F)), (f"b{l}", (N_F,)),
                (f"g{l}", (N_F,)), (f"be{l}", (N_F,))]
    out += [("g_e", (N_F,)), ("be_e", (N_F,)), ("fc_w", (N_F, n_out)), ("fc_b", (n_out,))]
    return out


def param_count(c_in: int, n_out: int) -> int:
    return int(sum(int(np.prod(s)) for _, s in param_shapes(c_in, n_out)))


def _truncated_normal(rng, shape, std):
    v = rng.standard_normal(shape)
    bad = np.abs(v) > 2.0
    while bad.any():
        v[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(v) > 2.0
    return v * std


def make_params(seed: int, c_in: int = 7, n_out: int = 2, std: float = 0.1, unit_gain: bool = False):
    """Variables drawn from the truncated normal of the paper's initialisation.

    unit_gain=True adds 1 to every layer-norm gain (the usual starting point of
    a layer norm), which drives the tanh units well into their non-linear range.
    """
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in param_shapes(c_in, n_out):
        v = _truncated_normal(rng, shape, std)
        if unit_gain and (name.startswith("g")):
            v = v + 1.0
        p[name] = v.astype(np.float32)
    return p


def flatten(params, c_in: int, n_out: int) -> np.ndarray:
    """The flat FP32 blob in the layout documented above."""
    parts = []
    for name, shape in param_shapes(c_in, n_out):
        a = np.asarray(params[name], dtype=np.float32)
        if a.shape != tuple(shape):
            raise ValueError(f"{name}: shape {a.shape}, expected {shape}")
        parts.append(a.ravel())
    return np.concatenate(parts).astype(np.float32)


def frames(seed: int, batch: int, c_in: int = 7, n_t: int = 1024, scale: float = 1.0) -> np.ndarray:
    """batch x c_in x n_t FP32 frames of N(0, scale^2) samples."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((batch, c_in, n_t)) * scale).astype(np.float32)
