"""CPU oracle for the F-engine and the corner turn (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this module.  The product path never does: it shares no code with the oracle.

What it computes (Sec. 2.1): the F-engine Fourier transforms the digitised signal of every
station, F complex samples at a time (one transform per input every F samples), and the
corner turn reorders the result from station-major to the frequency-major order the
X-engine reads (Sec. 4.1: station fastest, then channel, then time).  The spectra are then
requantised to 8-bit complex samples for the X-engine.

Readings where the paper is silent:
  * no window or polyphase filter: a plain F-point DFT of consecutive, non-overlapping
    blocks (the paper names only the Fourier transform);
  * channel k is DFT bin k, X[k] = sum_n x[n] exp(-2 pi i k n / F), in natural order;
  * a real gain scales the spectrum before requantisation; requantisation rounds each
    component half away from zero and clips it to [-127, 127] (the X-engine's int8 path
    needs no -128).

Input layout: int8 [nin][nsamp][2] (input = station * npol + pol, each input's samples
contiguous, (re, im) pairs); output [nframes][nchan][nin] (complex) and its requantised
int8 [nframes][nchan][nin][2].
"""

from __future__ import annotations

import numpy as np


def channelise(x: np.ndarray, nchan: int, gain: float) -> np.ndarray:
    """gain times the nchan-point DFT of every frame of every input, corner turned:
    complex128 [nframes][nchan][nin] with nframes = nsamp // nchan (a trailing partial
    frame is ignored).  The DFT is numpy's FFT in double precision."""
    x = np.asarray(x)
    if x.ndim != 3 or x.shape[2] != 2:
        raise ValueError("input must be [nin][nsamp][2]")
    nin, nsamp = x.shape[0], x.shape[1]
    nframes = nsamp // nchan
    z = x[:, : nframes * nchan, 0].astype(np.float64) + 1j * x[:, : nframes * nchan, 1].astype(np.float64)
    spec = np.fft.fft(z.reshape(nin, nframes, nchan), axis=-1) * float(gain)
    return np.ascontiguousarray(np.transpose(spec, (1, 2, 0)))


def round_half_away(v: np.ndarray) -> np.ndarray:
    """Nearest integer, halves rounded away from zero."""
    return np.sign(v) * np.floor(np.abs(v) + 0.5)


def requantise(spec: np.ndarray, lim: int = 127) -> np.ndarray:
    """Complex values -> int8 [..., 2]: each component rounded half away from zero and
    clipped to [-lim, lim]."""
    out = np.empty(spec.shape + (2,), dtype=np.int8)
    out[..., 0] = np.clip(round_half_away(spec.real), -lim, lim)
    out[..., 1] = np.clip(round_half_away(spec.imag), -lim, lim)
    return out


def fengine(x: np.ndarray, nchan: int, gain: float) -> np.ndarray:
    """Requantised, corner-turned spectra: int8 [nframes][nchan][nin][2], the X-engine's
    input layout."""
    return requantise(channelise(x, nchan, gain))
