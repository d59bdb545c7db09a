"""Pins of the F-engine oracle (DFT per input and frame, corner turn, requantisation)
against what the mathematics fixes (no GPU): the DFT sum written out on small sizes, the
transforms of an impulse and of a pure tone, Parseval's identity, linearity, the corner-turn
index map on explicit loops, and hand-worked rounding cases."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import fengine as FE


def _voltages(seed, nin, nsamp, lo=-60, hi=60):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(nin, nsamp, 2)).astype(np.int8)


@pytest.mark.parametrize("F", [1, 2, 4, 8, 16])
def test_matches_dft_sum(F):
    """X[t][k][i] = gain * sum_n x_i[tF + n] exp(-2 pi i k n / F), summed term by term."""
    nin, nframes, gain = 3, 4, 0.75
    x = _voltages(F, nin, nframes * F + (F // 2))  # a trailing partial frame is ignored
    got = FE.channelise(x, F, gain)
    assert got.shape == (nframes, F, nin)
    for i in range(nin):
        for t in range(nframes):
            for k in range(F):
                acc = 0j
                for n in range(F):
                    s = complex(int(x[i, t * F + n, 0]), int(x[i, t * F + n, 1]))
                    acc += s * complex(np.cos(-2 * np.pi * k * n / F), np.sin(-2 * np.pi * k * n / F))
                assert abs(got[t, k, i] - gain * acc) <= 1e-9 * max(1.0, abs(acc))


def test_impulse_is_flat():
    """A frame holding one sample at n = 0 transforms to that sample in every channel."""
    F, nin = 64, 2
    x = np.zeros((nin, 2 * F, 2), dtype=np.int8)
    x[0, 0] = (5, -3)
    x[1, F] = (-7, 2)
    got = FE.channelise(x, F, 1.0)
    assert np.allclose(got[0, :, 0], 5 - 3j, atol=1e-12)
    assert np.allclose(got[1, :, 1], -7 + 2j, atol=1e-12)
    assert np.allclose(got[1, :, 0], 0) and np.allclose(got[0, :, 1], 0)


def test_tone_lands_in_its_channel():
    """x[n] = A exp(2 pi i k0 n / F) puts F * A in channel k0 and nothing elsewhere."""
    F, k0, A = 128, 37, 40.0
    n = np.arange(F)
    z = A * np.exp(2j * np.pi * k0 * n / F)
    x = np.stack([z.real, z.imag], axis=-1)[None]  # float input: the oracle converts to float64
    got = FE.channelise(x, F, 1.0)[0, :, 0]
    assert abs(got[k0] - F * A) < 1e-9 * F * A
    others = np.delete(got, k0)
    assert np.max(np.abs(others)) < 1e-9 * F * A


def test_parseval():
    F, nin = 256, 5
    x = _voltages(9, nin, 3 * F)
    got = FE.channelise(x, F, 1.0)
    z = x[..., 0].astype(np.float64) + 1j * x[..., 1]
    for i in range(nin):
        for t in range(3):
            lhs = np.sum(np.abs(got[t, :, i]) ** 2)
            rhs = F * np.sum(np.abs(z[i, t * F:(t + 1) * F]) ** 2)
            assert abs(lhs - rhs) <= 1e-9 * rhs


def test_linearity_and_gain():
    F = 32
    a, b = _voltages(1, 2, 2 * F, -30, 30), _voltages(2, 2, 2 * F, -30, 30)
    s = (a.astype(np.int16) + b).astype(np.int8)
    assert np.allclose(FE.channelise(s, F, 1.0), FE.channelise(a, F, 1.0) + FE.channelise(b, F, 1.0), atol=1e-9)
    assert np.allclose(FE.channelise(a, F, 0.25), 0.25 * FE.channelise(a, F, 1.0), atol=1e-12)


def test_corner_turn_layout():
    """Output [t][k][i]: frame t of input i, channel k, with input = station * npol + pol."""
    F, ns, npol, nframes = 8, 3, 2, 5
    x = _voltages(3, ns * npol, nframes * F)
    got = FE.channelise(x, F, 1.0)
    for s in range(ns):
        for p in range(npol):
            i = s * npol + p
            z = x[i, :, 0].astype(np.float64) + 1j * x[i, :, 1]
            for t in range(nframes):
                spec = np.fft.fft(z[t * F:(t + 1) * F])
                assert np.allclose(got[t, :, i], spec, atol=1e-9)


def test_requantise_cases():
    v = np.array([2.5, -2.5, 2.49999, -0.5, 0.5, 0.49, 126.5, 127.4, 200.0, -200.0, -127.6, 0.0])
    want = np.array([3, -3, 2, -1, 1, 0, 127, 127, 127, -127, -127, 0])
    got = FE.requantise(v + 1j * v[::-1])
    assert np.array_equal(got[..., 0], want)
    assert np.array_equal(got[..., 1], want[::-1])
    assert got.dtype == np.int8
