"""FP64 CPU oracle for the image-source RIR path (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The arithmetic lives in ``ism_oracle.c`` (plain C,
FP64, libm); this module only compiles it with gcc and marshals numpy arrays.

Each wrapper cites the passage of the paper it follows: section II.A
(synthetic dataset generation with the image-source method and fractional
delays) and section III.A (convolution of the RIRs with source signals, plus
Gaussian sensor noise at a drawn SNR).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ism_oracle.c")
_LIB = os.path.join(_HERE, "libism_oracle.so")

ORDER_INDEX_L1 = 0
ORDER_REFLECTIONS = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: plain IEEE FP64, no FMA contraction, no fast-math."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ism_oracle_fd_tap.restype = ctypes.c_double
        L.ism_oracle_fd_tap.argtypes = [ctypes.c_double, ctypes.c_int]
        L.ism_oracle_lagrange_tap.restype = ctypes.c_double
        L.ism_oracle_lagrange_tap.argtypes = [ctypes.c_int, ctypes.c_double]
        L.ism_oracle_images.restype = ctypes.c_long
        L.ism_oracle_images.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_long]
        L.ism_oracle_rir.restype = ctypes.c_int
        L.ism_oracle_rir.argtypes = [dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     dp, ctypes.POINTER(_Stats)]
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.ism_oracle_rir_list.restype = ctypes.c_long
        L.ism_oracle_rir_list.argtypes = [dp, dp, dp, dp, i32p, i32p, i32p, i32p, i64p,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, i64p, ctypes.c_long, ctypes.c_int, dp]
        L.ism_oracle_conv_room.restype = ctypes.c_int
        L.ism_oracle_conv_room.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp,
                                           ctypes.c_int, ctypes.c_double, dp, dp]
        _lib = L
    return _lib


class _Stats(ctypes.Structure):
    _fields_ = [("images", ctypes.c_long), ("contrib", ctypes.c_long), ("taps", ctypes.c_long),
                ("max_refl", ctypes.c_long)]


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fd_tap(t: float, taps: int) -> float:
    """Hann-windowed sinc kernel h(t) with half-length K = (taps-1)/2 (section II.A filter, as
    specified for these workloads: windowed sinc in place of the paper's Lagrange filter)."""
    return lib().ism_oracle_fd_tap(float(t), (int(taps) - 1) // 2)


def lagrange_tap(j: int, D: float) -> float:
    """Coefficient j (0..7) of the 7th-order Lagrange fractional-delay interpolator at delay D
    (section II.A: the paper's own filter; selected by fd_taps = 8)."""
    return lib().ism_oracle_lagrange_tap(int(j), float(D))


def images(L, src, max_order: int, mode: int):
    """Closed-form image positions and six wall exponents of an index-bounded set (II.A)."""
    L_, pL = _d(L)
    s_, ps = _d(src)
    n = lib().ism_oracle_images(pL, ps, int(max_order), int(mode), None, None, 0)
    pos = np.zeros((max(n, 1), 3))
    ex = np.zeros((max(n, 1), 6), dtype=np.int64)
    lib().ism_oracle_images(pL, ps, int(max_order), int(mode),
                            pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            ex.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n)
    return pos[:n], ex[:n]


def rir(L, beta, src, mic, fs, c, max_order, mode, rir_len, fd_taps):
    """One RIR (one source, one microphone) in FP64 (section II.A).  Returns (out, stats)."""
    L_, pL = _d(L)
    b_, pb = _d(beta)
    s_, ps = _d(src)
    m_, pm = _d(mic)
    out = np.zeros(int(rir_len))
    st = _Stats()
    rc = lib().ism_oracle_rir(pL, pb, ps, pm, float(fs), float(c), int(max_order), int(mode),
                              int(rir_len), int(fd_taps),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out, {"images": st.images, "contrib": st.contrib, "taps": st.taps,
                 "max_refl": st.max_refl}


def rir_list(batch, rirs, nthreads=None, out=None):
    """Selected (room, mic) RIRs of a room batch, threads over RIRs.  ``batch`` is a
    scene dict (see the scenes module); ``rirs`` a list of (room, mic).  Returns
    (out FP64 array laid out like the batch output, taps counted)."""
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    L, pL = _d(batch["L"])
    b, pb = _d(batch["beta"])
    s, ps = _d(batch["src"])
    m, pm = _d(batch["mics"])
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    mo, nm, mx, rl = i32(batch["mic_offset"]), i32(batch["n_mics"]), i32(batch["max_order"]), i32(batch["rir_len"])
    oo = i64(batch["out_offset"])
    lst = i64([(int(r) << 20) | int(k) for r, k in rirs])
    total = int(oo[-1] + nm[-1] * rl[-1]) if len(oo) else 0
    if out is None:
        out = np.zeros(total)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    taps = lib().ism_oracle_rir_list(pL, pb, ps, pm, P(mo, ctypes.c_int32), P(nm, ctypes.c_int32),
                                     P(mx, ctypes.c_int32), P(rl, ctypes.c_int32), P(oo, ctypes.c_int64),
                                     float(batch["fs"]), float(batch["c"]), int(batch["order_mode"]),
                                     int(batch["fd_taps"]), P(lst, ctypes.c_int64), len(lst), int(nthreads),
                                     P(out, ctypes.c_double))
    return out, int(taps)


def conv_sample(h, x, n):
    """One output sample of the clean source convolution (section III.A): y_m[n] = sum over
    j <= n, j < len(h_m), n - j < len(x) of h_m[j] x[n - j], for every microphone m, in FP64
    (a plain sum, for checking sampled outputs of launches too large for conv_room)."""
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    n = int(n)
    j = np.arange(h.shape[1])
    ok = (j <= n) & (n - j < x.shape[0])
    jj = j[ok]
    return (h[:, jj] * x[n - jj][None, :]).sum(axis=1)


def conv_room(h, x, out_len, snr_db=None, z=None):
    """Source convolution of one room's RIRs h [M, hlen] with x (direct FP64 sum), plus sensor
    noise sigma*z when z [M, out_len] is given, sigma^2 = mean(y^2) * 10^(-snr_db/10)
    (section III.A: RIRs convolved with source signals; Gaussian noise at a drawn SNR)."""
    h_, ph = _d(np.atleast_2d(h))
    x_, px = _d(x)
    M, hlen = h_.shape
    y = np.zeros((M, int(out_len)))
    if z is not None:
        z_, pz = _d(z)
        assert z_.shape == (M, int(out_len))
    else:
        pz = None
    rc = lib().ism_oracle_conv_room(int(M), int(hlen), ph, int(x_.shape[0]), px, int(out_len),
                                    float(snr_db or 0.0), pz,
                                    y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return y
