"""FP64 reference for the reverberation-time fit of the wall reflection
coefficients (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library.

Paper section III.A: the simulated rooms have homogeneous wall absorption,
chosen with the method of Lehmann and Johansson so that the simulated RIRs have
the target reverberation time (0.5 s).  That method's closed-form prediction is
only cited by the paper.  This oracle reaches the same goal directly, on the
simulated RIR itself (a reading, listed with the design notes):

* the reverberation time of an RIR is its T30 (ISO 3382): the Schroeder
  backward-integrated energy decay in dB, a least-squares line through the
  samples from the first one 5 dB down to the first one 35 dB down, and the
  time that line takes to fall 60 dB;
* the fitted coefficient is the uniform beta (all six walls) whose RIR, from
  the given source to the given microphone, has the target T30: bisection on
  beta in [0, 1), T30 being increasing in beta;
* the room-level fit takes the mean T30 over several (source, microphone)
  pairs, every RIR of the sources of the dataset's torus to every microphone of
  the array, in place of one pair; a mean of increasing functions is
  increasing, so the same bisection applies.
"""
from __future__ import annotations

import math

import numpy as np

import oracle


def schroeder_db(h):
    """10 log10 of the backward-integrated energy, normalised to 0 dB at n = 0."""
    e = np.cumsum(np.asarray(h, np.float64)[::-1] ** 2)[::-1]
    with np.errstate(divide="ignore"):
        return 10.0 * np.log10(e / e[0])


def t30(h, fs):
    """T30 in seconds; +inf when the decay does not reach -35 dB (or the fit range
    holds fewer than 3 samples)."""
    db = schroeder_db(h)
    i5 = np.nonzero(db <= -5.0)[0]
    i35 = np.nonzero(db <= -35.0)[0]
    if len(i5) == 0 or len(i35) == 0:
        return math.inf
    n5, n35 = int(i5[0]), int(i35[0])
    if n35 - n5 < 2:
        return math.inf
    n = np.arange(n5, n35 + 1, dtype=np.float64)
    x = n / fs
    y = db[n5:n35 + 1]
    slope = np.polyfit(x, y, 1)[0]
    return -60.0 / slope if slope < 0 else math.inf


def rir_uniform(L, beta, src, mic, fs, c, rir_len, fd_taps):
    out, _ = oracle.rir(L, [beta] * 6, src, mic, fs, c, -1, 0, rir_len, fd_taps)
    return out


def fit_beta(L, src, mic, fs, c, fd_taps, rt_target, rir_len, iters=30):
    """Bisection for the uniform beta whose RIR has T30 = rt_target.
    Returns (beta, T30 at beta)."""
    lo, hi = 0.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        rt = t30(rir_uniform(L, mid, src, mic, fs, c, rir_len, fd_taps), fs)
        if rt < rt_target:
            lo = mid
        else:
            hi = mid
    beta = 0.5 * (lo + hi)
    return beta, t30(rir_uniform(L, beta, src, mic, fs, c, rir_len, fd_taps), fs)


def _uniform_batch(L, beta, srcs, mics, fs, c, rir_len, fd_taps):
    """One room per source, all with the same walls and the same microphones."""
    srcs = np.atleast_2d(np.asarray(srcs, dtype=np.float64))
    mics = np.atleast_2d(np.asarray(mics, dtype=np.float64))
    R, M = len(srcs), len(mics)
    return {"L": np.tile(np.asarray(L, dtype=np.float64), (R, 1)), "beta": np.full((R, 6), float(beta)),
            "src": srcs, "mics": mics, "mic_offset": np.zeros(R, dtype=np.int32),
            "n_mics": np.full(R, M, dtype=np.int32), "max_order": np.full(R, -1, dtype=np.int32),
            "rir_len": np.full(R, int(rir_len), dtype=np.int32),
            "out_offset": np.arange(R, dtype=np.int64) * M * int(rir_len),
            "fs": float(fs), "c": float(c), "order_mode": 0, "fd_taps": int(fd_taps)}


def mean_t30(L, beta, srcs, mics, fs, c, rir_len, fd_taps):
    """Mean T30 over every (source, microphone) RIR of a room with uniform walls (+inf if any
    decay does not reach -35 dB)."""
    b = _uniform_batch(L, beta, srcs, mics, fs, c, rir_len, fd_taps)
    R, M = len(b["src"]), len(b["mics"])
    out, _ = oracle.rir_list(b, [(r, m) for r in range(R) for m in range(M)])
    rirs = out.reshape(R * M, int(rir_len))
    return float(np.mean([t30(h, fs) for h in rirs]))


def fit_beta_mean(L, srcs, mics, fs, c, fd_taps, rt_target, rir_len, iters=30):
    """Bisection for the uniform beta whose RIRs (every source to every microphone) have a mean
    T30 of rt_target.  Returns (beta, mean T30 at beta)."""
    lo, hi = 0.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mean_t30(L, mid, srcs, mics, fs, c, rir_len, fd_taps) < rt_target:
            lo = mid
        else:
            hi = mid
    beta = 0.5 * (lo + hi)
    return beta, mean_t30(L, beta, srcs, mics, fs, c, rir_len, fd_taps)
