"""Seeded synthetic station voltages (shared by tests, the benchmark and the oracle harness).

This module holds no X-engine arithmetic.  It only turns (seed, stream, flat index) into
integer sample values, with the value distributions of the paper's workloads: complex
samples quantised to a few bits in two's complement (Sec. 2.1, digitiser precision of two
to twelve bits; Sec. 5, 8-bit input to the X-engine).

Random stream
    The n-th word of stream ``s`` under ``seed`` is the counter-based SplitMix64 output
    (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
    ``mix64(key + (n + 1) * GOLDEN)`` with ``key = mix64(seed ^ (s << 32))``; the top 32
    bits are used.  Any element can be generated on its own, so a test can regenerate a
    single channel of a huge workload.

Flat index of a component
    Input layout is the paper's corner-turned order (Sec. 4.1): station (and polarisation)
    fastest, then channel, then time.  Component ``c`` (0 = real, 1 = imaginary) of input
    ``i`` in channel ``f`` at time ``t`` has index ``((t * F + f) * N_in + i) * 2 + c``.

Distributions
    * ``uniform``: integers in ``[lo, hi]`` by multiply-shift of the 32-bit word.
    * ``gauss``: a zero-mean Gaussian of standard deviation ``sigma``, rounded to the
      nearest integer and clipped to ``[-clip, clip]``.  Sampled exactly by inverse CDF:
      the word is compared against 32-bit thresholds ``round(Phi((k + 1/2) / sigma) * 2^32)``
      so that numpy and torch produce identical integers.

Two backends with one definition: numpy (``backend="numpy"``) and torch on any device
(``backend="torch"``), the latter emulating unsigned 64-bit arithmetic with wrapping int64.
"""

from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_U64 = (1 << 64) - 1

# Stream numbers (kept distinct so independent draws never share words).
STREAM_VOLTAGE = 0
STREAM_GAIN = 2
STREAM_SOURCE = 3
STREAM_JOBS = 4
STREAM_JOB_BASE = 16

# Seed convention: 0x11074264 + index of the workload in the list of workloads.
SEED_BASE = 0x11074264


def _mix64_int(z: int) -> int:
    z &= _U64
    z = ((z ^ (z >> 30)) * _M1) & _U64
    z = ((z ^ (z >> 27)) * _M2) & _U64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    return _mix64_int((seed ^ (stream << 32)) & _U64)


# ----------------------------------------------------------------------------- numpy


def words_np(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """32-bit words (as uint64 values < 2^32) for an array of flat indices."""
    key = np.uint64(stream_key(seed, stream))
    z = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + (z + np.uint64(1)) * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z >> np.uint64(32)


@lru_cache(maxsize=None)
def gauss_thresholds(sigma: float, clip: int) -> tuple:
    """Cumulative thresholds th[k + clip] for k = -clip .. clip-1 (value k iff th[k-1] <= w < th[k])."""
    th = []
    for k in range(-clip, clip):
        x = (k + 0.5) / sigma
        cdf = 0.5 * math.erfc(-x / math.sqrt(2.0))
        th.append(min(max(int(round(cdf * 2.0**32)), 0), 1 << 32))
    return tuple(th)


def values_from_words_np(w: np.ndarray, dist: tuple) -> np.ndarray:
    kind = dist[0]
    if kind == "uniform":
        lo, hi = int(dist[1]), int(dist[2])
        span = np.uint64(hi - lo + 1)
        return ((w * span) >> np.uint64(32)).astype(np.int64) + lo
    if kind == "gauss":
        sigma, clip = float(dist[1]), int(dist[2])
        th = np.asarray(gauss_thresholds(sigma, clip), dtype=np.uint64)
        return np.searchsorted(th, w, side="right").astype(np.int64) - clip
    raise ValueError(f"unknown distribution {dist!r}")


def _flat_index_np(ntime, nchan, nin, t0=0, chans=None):
    t = np.arange(t0, t0 + ntime, dtype=np.uint64)[:, None, None, None]
    f = (np.arange(nchan, dtype=np.uint64) if chans is None
         else np.asarray(chans, dtype=np.uint64))[None, :, None, None]
    i = np.arange(nin, dtype=np.uint64)[None, None, :, None]
    c = np.arange(2, dtype=np.uint64)[None, None, None, :]
    return ((t * np.uint64(nchan) + f) * np.uint64(nin) + i) * np.uint64(2) + c


def voltages_np(seed, ntime, nchan, nin, dist, stream=STREAM_VOLTAGE, t0=0, chans=None):
    """int8 array [ntime][len(chans) or nchan][nin][2] (re, im); ``nchan`` is the workload's
    total channel count (it fixes the flat index), ``chans`` optionally selects channels."""
    idx = _flat_index_np(ntime, nchan, nin, t0, chans)
    return values_from_words_np(words_np(seed, stream, idx), dist).astype(np.int8)


# ----------------------------------------------------------------------------- torch


def _s64(v: int) -> int:
    v &= _U64
    return v - (1 << 64) if v >> 63 else v


def _lsr(z, s):
    import torch  # noqa: F401

    return (z >> s) & ((1 << (64 - s)) - 1)


def words_torch(seed, stream, index):
    """Same words as :func:`words_np` for an int64 torch tensor of flat indices."""
    z = index + 1
    z = z * _s64(GOLDEN) + _s64(stream_key(seed, stream))
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    z = z ^ _lsr(z, 31)
    return _lsr(z, 32)


def values_from_words_torch(w, dist):
    import torch

    kind = dist[0]
    if kind == "uniform":
        lo, hi = int(dist[1]), int(dist[2])
        return ((w * (hi - lo + 1)) >> 32) + lo
    if kind == "gauss":
        sigma, clip = float(dist[1]), int(dist[2])
        th = torch.tensor(gauss_thresholds(sigma, clip), dtype=torch.int64, device=w.device)
        return torch.searchsorted(th, w, right=True) - clip
    raise ValueError(f"unknown distribution {dist!r}")


def voltages_torch(seed, ntime, nchan, nin, dist, device, stream=STREAM_VOLTAGE, t0=0,
                   out=None, time_slice=None):
    """Torch int8 tensor [ntime][nchan][nin][2], generated slice by slice along time."""
    import torch

    if out is None:
        out = torch.empty((ntime, nchan, nin, 2), dtype=torch.int8, device=device)
    per_t = nchan * nin * 2
    step = time_slice or max(1, (1 << 26) // max(per_t, 1))
    base = torch.arange(per_t, dtype=torch.int64, device=device)
    for ts in range(0, ntime, step):
        te = min(ntime, ts + step)
        tt = torch.arange(t0 + ts, t0 + te, dtype=torch.int64, device=device)[:, None]
        idx = tt * per_t + base[None, :]
        vals = values_from_words_torch(words_torch(seed, stream, idx), dist)
        out[ts:te].copy_(vals.to(torch.int8).view(te - ts, nchan, nin, 2))
    return out


# ----------------------------------------------------------------------------- formats


def pack_ci4(v: np.ndarray) -> np.ndarray:
    """[..., 2] int8 with values in [-8, 7] -> [...] uint8, real part in the high nibble and
    imaginary part in the low nibble, both two's complement."""
    v = np.asarray(v)
    if v.min(initial=0) < -8 or v.max(initial=0) > 7:
        raise ValueError("ci4 samples must lie in [-8, 7]")
    re = v[..., 0].astype(np.int64) & 0xF
    im = v[..., 1].astype(np.int64) & 0xF
    return ((re << 4) | im).astype(np.uint8)


def unpack_ci4(b: np.ndarray) -> np.ndarray:
    b = np.asarray(b, dtype=np.uint8).astype(np.int64)
    re = (b >> 4) & 0xF
    im = b & 0xF
    re = np.where(re >= 8, re - 16, re)
    im = np.where(im >= 8, im - 16, im)
    return np.stack([re, im], axis=-1).astype(np.int8)


def pack_ci4_torch(v):
    """Torch version of :func:`pack_ci4` (no range check)."""
    import torch

    re = v[..., 0].to(torch.int32) & 0xF
    im = v[..., 1].to(torch.int32) & 0xF
    return ((re << 4) | im).to(torch.uint8)


# ----------------------------------------------------------------------------- workloads


def point_source_np(seed, ntime, nchan, nin, gain_max=3, source_max=21):
    """A single noiseless point source: x_i(t, f) = a_i * s(t, f).

    Returns (x int8 [T][F][nin][2], a int64 [nin][2], s int64 [T][F][2]).  Gains have real
    and imaginary parts uniform in [-gain_max, gain_max]; the source has parts uniform in
    [-source_max, source_max]; with the defaults every component of x lies in [-126, 126].
    """
    a = values_from_words_np(words_np(seed, STREAM_GAIN, np.arange(nin * 2, dtype=np.uint64)),
                             ("uniform", -gain_max, gain_max)).reshape(nin, 2)
    sidx = np.arange(ntime * nchan * 2, dtype=np.uint64)
    s = values_from_words_np(words_np(seed, STREAM_SOURCE, sidx),
                             ("uniform", -source_max, source_max)).reshape(ntime, nchan, 2)
    ar, ai = a[None, None, :, 0], a[None, None, :, 1]
    sr, si = s[:, :, None, 0], s[:, :, None, 1]
    x = np.stack([ar * sr - ai * si, ar * si + ai * sr], axis=-1)
    if np.abs(x).max(initial=0) > 127:
        raise ValueError("point source does not fit in 8 bits")
    return x.astype(np.int8), a, s


def draw_jobs(seed, njobs=64, nin_half=(24, 288), nchan=(32, 512), ntime=(128, 8192)):
    """Uneven sub-array jobs: N_in = 2*U{nin_half}, F = U{nchan}, T = U{ntime} (inclusive)."""
    w = words_np(seed, STREAM_JOBS, np.arange(3 * njobs, dtype=np.uint64)).reshape(njobs, 3)
    jobs = []
    for j in range(njobs):
        h = int(values_from_words_np(w[j, 0:1], ("uniform",) + tuple(nin_half))[0])
        f = int(values_from_words_np(w[j, 1:2], ("uniform",) + tuple(nchan))[0])
        t = int(values_from_words_np(w[j, 2:3], ("uniform",) + tuple(ntime))[0])
        jobs.append({"nstation": h, "npol": 2, "nchan": f, "ntime": t})
    return jobs
