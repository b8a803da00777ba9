"""Seeded synthetic scenes (inputs only).

This module draws room geometries, wall reflection coefficients, source and
microphone positions, RIR lengths, source signals and SNRs with numpy's PCG64
generator.  It holds none of the image-source arithmetic: both the GPU library
and the FP64 oracle receive the arrays it returns.

Scene shapes follow the workloads the paper trains on (section II.A: shoebox
rooms, compact microphone arrays, RIRs up to the reverberation time; section
III.A: RIRs convolved with source signals, Gaussian sensor noise at a drawn
SNR), at the sizes of the five benchmark configurations:

* ``c0``  one 5x4x3 m room, beta 0.7, index-L1 order 10, 4096 samples, 81 taps;
          ``c0_replicated``: 4096 copies of it, sources moved by up to 0.25 m;
* ``c1``  1024 rooms, dims U[3,10]xU[3,8]xU[2.5,4] m, RT60 U[0.2,0.8] s, Sabine
          beta, 8-mic circle r = 5 cm, len = round(0.8 RT60 fs), 81 taps;
* ``c2``  serving requests, RT60 U[0.1,1.0] s, len = round(RT60 fs),
          M uniform in {4,8,16,32};
* ``c3``  64 rooms 20x15x8 m, per-wall beta U[0.85,0.95], 48 kHz, 72000
          samples, 16 mics on a Fibonacci sphere r = 10 cm, 127 taps;
* ``c4``  256 rooms of the c1 distribution (8 mics), 1 s N(0,1) sources,
          SNR U[0,30] dB;
* ``paper_room1``  the paper's first training room: 7 x 10 x 3.7 m, RT 0.5 s,
          the 7-microphone array (centre + 6 on an 8 cm circle) at (4, 6, 1.5) m,
          sources uniform in the torus of central radius 2 m, +-0.5 m radially and
          +-7 degrees in elevation around it (48 000 positions per room);
* ``paper_room2``  the paper's second simulated room: 5 x 5 x 4 m, RT 0.5 s, the
          same array centred at (2.5, 2.5, 1.5) m and the same torus (positions
          within 0.1 m of a wall drawn again), 48 000 positions.

Seeds default to 2104 + config index.  The paper's recordings are not
available; white-noise sources stand in for them.
"""
from __future__ import annotations

import math

import numpy as np

C_SOUND = 343.0
ORDER_INDEX_L1 = 0
ORDER_REFLECTIONS = 1


def sabine_beta(L, rt60, c=C_SOUND):
    """Uniform pressure reflection coefficient from Sabine's RT60 formula
    (alpha = 24 ln10 V / (c S RT60), clamped to [0, 1]; beta = sqrt(1 - alpha))."""
    L = np.asarray(L, dtype=np.float64)
    V = L[..., 0] * L[..., 1] * L[..., 2]
    S = 2.0 * (L[..., 0] * L[..., 1] + L[..., 0] * L[..., 2] + L[..., 1] * L[..., 2])
    alpha = 24.0 * math.log(10.0) * V / (c * S * np.asarray(rt60))
    clamped = alpha >= 1.0
    alpha = np.clip(alpha, 0.0, 1.0)
    return np.sqrt(1.0 - alpha), clamped


def _uniform_inside(rng, L, margin, n=None):
    lo = margin
    return rng.uniform(lo, np.asarray(L) - margin, size=None if n is None else (n, 3))


def circle_array(center, M, radius, rot):
    ang = rot + 2.0 * math.pi * np.arange(M) / M
    return np.stack([center[0] + radius * np.cos(ang), center[1] + radius * np.sin(ang),
                     np.full(M, center[2])], axis=1)


def fibonacci_sphere(center, M, radius):
    i = np.arange(M) + 0.5
    z = 1.0 - 2.0 * i / M
    r = np.sqrt(1.0 - z * z)
    phi = np.arange(M) * math.pi * (3.0 - math.sqrt(5.0))
    return np.asarray(center) + radius * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def pack(rooms, fs, c, fd_taps, order_mode, name):
    """Pack a list of room dicts (L, beta, src, mics, max_order, rir_len) into batch arrays.
    Output of room i, mic m starts at out_offset[i] + m * rir_len[i] (float elements)."""
    R = len(rooms)
    n_mics = np.array([len(r["mics"]) for r in rooms], dtype=np.int32)
    mic_offset = np.zeros(R, dtype=np.int32)
    if R:
        mic_offset[1:] = np.cumsum(n_mics)[:-1]
    rir_len = np.array([r["rir_len"] for r in rooms], dtype=np.int32)
    sizes = n_mics.astype(np.int64) * rir_len.astype(np.int64)
    out_offset = np.zeros(R, dtype=np.int64)
    if R:
        out_offset[1:] = np.cumsum(sizes)[:-1]
    return {
        "name": name,
        "L": np.array([r["L"] for r in rooms], dtype=np.float64).reshape(R, 3),
        "beta": np.array([r["beta"] for r in rooms], dtype=np.float64).reshape(R, 6),
        "src": np.array([r["src"] for r in rooms], dtype=np.float64).reshape(R, 3),
        "mics": (np.concatenate([np.asarray(r["mics"], dtype=np.float64) for r in rooms])
                 if R else np.zeros((0, 3))),
        "mic_offset": mic_offset,
        "n_mics": n_mics,
        "max_order": np.array([r["max_order"] for r in rooms], dtype=np.int32),
        "rir_len": rir_len,
        "out_offset": out_offset,
        "out_size": int(sizes.sum()),
        "fs": float(fs), "c": float(c), "fd_taps": int(fd_taps), "order_mode": int(order_mode),
        "rt60": np.array([r.get("rt60", float("nan")) for r in rooms], dtype=np.float64),
    }


def subset(batch, idx):
    """Re-pack a subset of rooms of a packed batch."""
    rooms = []
    for i in idx:
        o, M = batch["mic_offset"][i], batch["n_mics"][i]
        rooms.append({"L": batch["L"][i], "beta": batch["beta"][i], "src": batch["src"][i],
                      "mics": batch["mics"][o:o + M], "max_order": int(batch["max_order"][i]),
                      "rir_len": int(batch["rir_len"][i]), "rt60": float(batch["rt60"][i])})
    return pack(rooms, batch["fs"], batch["c"], batch["fd_taps"], batch["order_mode"],
                batch["name"] + "-subset")


def uma8_array(center, rot=0.0):
    """The 7-microphone array of the paper: one at the centre, six evenly spread on a circle
    of 8 cm diameter, horizontal."""
    ring = circle_array(center, 6, 0.04, rot)
    return np.concatenate([np.asarray(center, dtype=np.float64)[None, :], ring])


def torus_sources(rng, center, n, R=2.0, dR=0.5, dphi_deg=7.0):
    """Positions uniform in volume in the torus around ``center``: distance R +- dR from it,
    any azimuth, elevation within +-dphi (spherical volume element r^2 cos(phi))."""
    r = np.cbrt(rng.uniform((R - dR) ** 3, (R + dR) ** 3, n))
    th = rng.uniform(0.0, 2.0 * math.pi, n)
    s = math.sin(math.radians(dphi_deg))
    ph = np.arcsin(rng.uniform(-s, s, n))
    return np.asarray(center) + np.stack([r * np.cos(ph) * np.cos(th), r * np.cos(ph) * np.sin(th),
                                          r * np.sin(ph)], axis=1)


def paper_room1(n_sources=48000, seed=2109, fs=16000.0, c=C_SOUND, fd_taps=8, beta=None):
    """The paper's first training room (section II.A and the dataset description): every source
    position is one entry of the batch, with the 7-microphone array; RIRs up to the
    reverberation time.  The paper names no sampling rate: 16 kHz here.  Reflection
    coefficients from Sabine's formula (the paper fits them with Lehmann's method)."""
    rng = np.random.default_rng(seed)
    L = np.array([7.0, 10.0, 3.7])
    rt = 0.5
    if beta is None:  # a caller may pass a fitted coefficient instead of Sabine's
        beta, _ = sabine_beta(L, rt, c)
    center = np.array([4.0, 6.0, 1.5])
    mics = uma8_array(center)
    src = torus_sources(rng, center, n_sources)
    rooms = [{"L": L, "beta": np.full(6, float(beta)), "src": src[i], "mics": mics, "max_order": -1,
              "rir_len": int(round(rt * fs)), "rt60": rt} for i in range(n_sources)]
    return pack(rooms, fs, c, fd_taps, ORDER_INDEX_L1, "paper_room1")


def paper_room2(n_sources=48000, seed=2110, fs=16000.0, c=C_SOUND, fd_taps=8, beta=None, wall_margin=0.1):
    """The paper's second simulated room (section III.A): almost cubic, 5 x 5 x 4 m, reverberation
    time 0.5 s, the same 7-microphone array and torus of sources.  The paper gives no array
    position for this room: centred in the floor plan at 1.5 m (as in room 1).  The torus then
    reaches the walls (2.5 m from the centre on the axes), so positions closer than wall_margin to
    a wall are drawn again.  Sabine's coefficient unless a fitted beta is passed."""
    rng = np.random.default_rng(seed)
    L = np.array([5.0, 5.0, 4.0])
    rt = 0.5
    if beta is None:
        beta, _ = sabine_beta(L, rt, c)
    center = np.array([2.5, 2.5, 1.5])
    mics = uma8_array(center)
    src = np.empty((0, 3))
    while len(src) < n_sources:
        cand = torus_sources(rng, center, n_sources)
        ok = np.all((cand > wall_margin) & (cand < L - wall_margin), axis=1)
        src = np.concatenate([src, cand[ok]])
    src = src[:n_sources]
    rooms = [{"L": L, "beta": np.full(6, float(beta)), "src": src[i], "mics": mics, "max_order": -1,
              "rir_len": int(round(rt * fs)), "rt60": rt} for i in range(n_sources)]
    return pack(rooms, fs, c, fd_taps, ORDER_INDEX_L1, "paper_room2")


def c0():
    room = {"L": (5.0, 4.0, 3.0), "beta": (0.7,) * 6, "src": (1.3, 2.1, 1.5),
            "mics": [(3.6, 1.7, 1.2)], "max_order": 10, "rir_len": 4096}
    return pack([room], 16000.0, C_SOUND, 81, ORDER_INDEX_L1, "c0")


def c0_replicated(n_rooms=4096, seed=2104, jitter=0.25):
    """The single-RIR room repeated: n_rooms copies of c0's room, microphone, order bound and
    length, each source moved by U[-jitter, jitter] m per axis (a batch of identical shape
    whose per-RIR work is that of c0)."""
    rng = np.random.default_rng(seed)
    base = c0()
    src0 = base["src"][0]
    rooms = [{"L": (5.0, 4.0, 3.0), "beta": (0.7,) * 6, "src": src0 + rng.uniform(-jitter, jitter, 3),
              "mics": [(3.6, 1.7, 1.2)], "max_order": 10, "rir_len": 4096} for _ in range(n_rooms)]
    return pack(rooms, 16000.0, C_SOUND, 81, ORDER_INDEX_L1, "c0x")


def _shoebox_room(rng, rt60_lo, rt60_hi, M, len_factor, fs, c):
    L = np.array([rng.uniform(3.0, 10.0), rng.uniform(3.0, 8.0), rng.uniform(2.5, 4.0)])
    rt60 = rng.uniform(rt60_lo, rt60_hi)
    beta, _ = sabine_beta(L, rt60, c)
    src = _uniform_inside(rng, L, 0.5)
    while True:
        center = _uniform_inside(rng, L, 0.5)
        if np.linalg.norm(center - src) > 0.3:
            break
    mics = circle_array(center, M, 0.05, rng.uniform(0.0, 2.0 * math.pi))
    return {"L": L, "beta": np.full(6, float(beta)), "src": src, "mics": mics, "max_order": -1,
            "rir_len": int(round(len_factor * rt60 * fs)), "rt60": rt60}


def c1(seed=2105, n_rooms=1024, fs=16000.0, c=C_SOUND):
    rng = np.random.default_rng(seed)
    rooms = [_shoebox_room(rng, 0.2, 0.8, 8, 0.8, fs, c) for _ in range(n_rooms)]
    return pack(rooms, fs, c, 81, ORDER_INDEX_L1, "c1")


def c2(seed=2106, n_requests=20000, fs=16000.0, c=C_SOUND):
    """Serving requests: a list of single-room batches plus unit-rate exponential gaps
    (scale by 1/lambda for Poisson arrivals at rate lambda)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_requests):
        M = int(rng.choice([4, 8, 16, 32]))
        reqs.append(_shoebox_room(rng, 0.1, 1.0, M, 1.0, fs, c))
    gaps = rng.exponential(1.0, size=n_requests)
    return reqs, gaps, {"fs": fs, "c": c, "fd_taps": 81, "order_mode": ORDER_INDEX_L1}


def c3(seed=2107, n_rooms=64, fs=48000.0, c=C_SOUND):
    rng = np.random.default_rng(seed)
    rooms = []
    L = np.array([20.0, 15.0, 8.0])
    for _ in range(n_rooms):
        beta = rng.uniform(0.85, 0.95, size=6)
        src = _uniform_inside(rng, L, 0.5)
        while True:
            center = _uniform_inside(rng, L, 0.6)
            if np.linalg.norm(center - src) > 0.3:
                break
        rooms.append({"L": L, "beta": beta, "src": src, "mics": fibonacci_sphere(center, 16, 0.10),
                      "max_order": -1, "rir_len": 72000, "rt60": 1.5})
    return pack(rooms, fs, c, 127, ORDER_INDEX_L1, "c3")


def c4(seed=2108, n_rooms=256, fs=16000.0, c=C_SOUND, src_len=16000, with_z=True):
    rng = np.random.default_rng(seed)
    rooms = [_shoebox_room(rng, 0.2, 0.8, 8, 0.8, fs, c) for _ in range(n_rooms)]
    batch = pack(rooms, fs, c, 81, ORDER_INDEX_L1, "c4")
    batch["x"] = rng.standard_normal((n_rooms, src_len)).astype(np.float32)
    batch["snr_db"] = rng.uniform(0.0, 30.0, size=n_rooms).astype(np.float32)
    # key of the sensor-noise generator when the deviates are drawn on the device
    batch["noise_seed"] = seed
    if with_z:
        # host-drawn standard normal deviates [room, mic, sample] for the caller-supplied
        # noise form; scaled to the drawn SNR by the convolution step
        batch["z"] = rng.standard_normal((n_rooms, 8, src_len)).astype(np.float32)
    return batch


def tiny(seed=7, n_rooms=4, fs=8000.0, c=C_SOUND, rir_len=64, M=2, taps=9):
    """Very small rooms (about 1 m) for brute-force checks."""
    rng = np.random.default_rng(seed)
    rooms = []
    for _ in range(n_rooms):
        L = np.array([rng.uniform(0.8, 1.3), rng.uniform(0.8, 1.3), rng.uniform(0.7, 1.0)])
        beta = rng.uniform(0.3, 0.9, size=6)
        src = _uniform_inside(rng, L, 0.1)
        mics = np.array([_uniform_inside(rng, L, 0.1) for _ in range(M)])
        rooms.append({"L": L, "beta": beta, "src": src, "mics": mics, "max_order": -1,
                      "rir_len": rir_len})
    return pack(rooms, fs, c, taps, ORDER_INDEX_L1, "tiny")


def synthetic_rirs(rir_len, M, seed=17, decay_s=0.15, fs=16000.0):
    """Decaying-noise RIR-like arrays (inputs for convolution tests): per room, M rows of
    N(0,1) * exp(-n / (decay_s fs)).  Returns (flat float32 array, per-room offsets)."""
    rng = np.random.default_rng(seed)
    rir_len = np.asarray(rir_len, dtype=np.int64)
    offs = np.zeros(len(rir_len), dtype=np.int64)
    if len(rir_len):
        offs[1:] = np.cumsum(rir_len * M)[:-1]
    out = np.empty(int((rir_len * M).sum()), dtype=np.float32)
    for r, L in enumerate(rir_len):
        env = np.exp(-np.arange(L) / (decay_s * fs))
        out[offs[r]:offs[r] + M * L] = (rng.standard_normal((M, L)) * env).astype(np.float32).ravel()
    return out, offs
