"""Pins of the FP64 reverberation-time fit (oracle/rt_fit.py) against closed forms
and invariances that do not depend on the oracle's own code."""
import math

import numpy as np
import pytest

from oracle import rt_fit

FS = 8000.0
ROOM = dict(L=[4.0, 5.0, 3.0], src=[1.2, 1.5, 1.4], mic=[2.9, 3.6, 1.6])


@pytest.mark.parametrize("T", [0.2, 0.5, 1.3])
def test_t30_of_exact_exponential_decay(T):
    # h^2[n] = exp(-2 delta n / fs) with random signs: the Schroeder decay is a straight
    # line of -60 dB per T (the tail beyond the window is below 1e-14 of the total)
    delta = 3.0 * math.log(10.0) / T
    n = np.arange(int(3.0 * T * FS))
    rng = np.random.default_rng(1)
    h = np.exp(-delta * n / FS) * rng.choice([-1.0, 1.0], size=n.size)
    assert abs(rt_fit.t30(h, FS) - T) < 1e-9 * T


def test_t30_infinite_when_decay_too_short():
    h = np.exp(-np.arange(200) / 1000.0)      # only about 1.7 dB of decay in the window
    assert rt_fit.t30(h, FS) == math.inf


def test_t30_scales_with_room_and_speed_of_sound():
    # all lengths x2 at the same beta: every delay doubles, every image gain halves,
    # so the decay takes twice as long; c x2 halves every delay
    L, s, m = ROOM["L"], ROOM["src"], ROOM["mic"]
    n = int(0.6 * FS)
    a = rt_fit.t30(rt_fit.rir_uniform(L, 0.8, s, m, FS, 343.0, n, 8), FS)
    b = rt_fit.t30(rt_fit.rir_uniform([2 * v for v in L], 0.8, [2 * v for v in s], [2 * v for v in m],
                                      FS, 343.0, 2 * n, 8), FS)
    d = rt_fit.t30(rt_fit.rir_uniform(L, 0.8, s, m, FS, 686.0, n, 8), FS)
    assert abs(b / a - 2.0) < 0.02
    assert abs(d / a - 0.5) < 0.02


def test_t30_increases_with_beta_and_fit_hits_target():
    L, s, m = ROOM["L"], ROOM["src"], ROOM["mic"]
    n = int(0.8 * FS)
    rts = [rt_fit.t30(rt_fit.rir_uniform(L, b, s, m, FS, 343.0, n, 8), FS) for b in (0.5, 0.7, 0.85)]
    assert rts[0] < rts[1] < rts[2]
    beta, rt = rt_fit.fit_beta(L, s, m, FS, 343.0, 8, 0.25, int(2.5 * 0.25 * FS), iters=20)
    assert abs(rt - 0.25) < 1e-3 and 0.5 < beta < 0.95


# ---------------------------------------------------------------- room-level fit (mean T30)
SMALL = dict(L=[2.0, 2.5, 1.8], fs=4000.0, rt=0.1, n=1000, iters=16)
SRCS = [[0.6, 0.7, 0.9], [1.4, 1.9, 0.5]]
MICS = [[1.1, 1.2, 1.0], [1.15, 1.25, 1.0]]


def test_mean_fit_with_one_pair_is_the_single_pair_fit():
    L, fs, rt, n, it = SMALL["L"], SMALL["fs"], SMALL["rt"], SMALL["n"], SMALL["iters"]
    a = rt_fit.fit_beta(L, SRCS[0], MICS[0], fs, 343.0, 8, rt, n, iters=it)
    b = rt_fit.fit_beta_mean(L, [SRCS[0]], [MICS[0]], fs, 343.0, 8, rt, n, iters=it)
    assert a == b
    # the same position listed twice changes nothing (a mean of equal values)
    c = rt_fit.fit_beta_mean(L, [SRCS[0], SRCS[0]], [MICS[0], MICS[0]], fs, 343.0, 8, rt, n, iters=it)
    assert c[0] == a[0] and abs(c[1] - a[1]) <= 1e-12 * a[1]


def test_mean_fit_lies_between_the_pair_fits_and_hits_the_mean_target():
    # each pair's T30 increases with beta and reaches the target at its own beta_i; at
    # min beta_i every pair is at or below the target and at max beta_i at or above it, so
    # the mean crosses the target in between.  At the fitted beta the mean of independently
    # computed pair T30s is the target to the bisection's resolution.
    L, fs, rt, n, it = SMALL["L"], SMALL["fs"], SMALL["rt"], SMALL["n"], SMALL["iters"]
    pair = [rt_fit.fit_beta(L, s, m, fs, 343.0, 8, rt, n, iters=it)[0] for s in SRCS for m in MICS]
    beta, mt = rt_fit.fit_beta_mean(L, SRCS, MICS, fs, 343.0, 8, rt, n, iters=it)
    assert min(pair) - 2.0 ** -it <= beta <= max(pair) + 2.0 ** -it
    direct = np.mean([rt_fit.t30(rt_fit.rir_uniform(L, beta, s, m, fs, 343.0, n, 8), fs) for s in SRCS for m in MICS])
    assert abs(direct - mt) <= 1e-12 * mt
    assert abs(mt - rt) <= 0.01 * rt
