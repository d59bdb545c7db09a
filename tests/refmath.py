"""Independent numpy-side helpers for the tests: brute-force visibilities by matrix product
and a baseline index built from ``np.tril_indices`` (not from a closed-form formula).

These pin the oracle (and, through it, the GPU path) to a library routine: for each channel
the visibility matrix is ``X @ X^H`` with ``X[i, t] = x_i(t)`` (Sec. 2.1, Eq. 4).
"""

from __future__ import annotations

import numpy as np


def to_complex(x: np.ndarray) -> np.ndarray:
    """int8/float [T][F][N][2] -> complex128 [T][F][N]."""
    x = np.asarray(x)
    return x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)


def station_pairs(nstation: int):
    """(s1, s2) with s1 >= s2 in packed order, from numpy's lower-triangle enumeration."""
    return np.tril_indices(nstation)


def brute(x: np.ndarray, nstation: int, npol: int) -> np.ndarray:
    """complex128 [F][nbl][npol*npol] from X @ X^H per channel."""
    xc = to_complex(x)  # [T][F][N]
    ntime, nchan, nin = xc.shape
    s1, s2 = station_pairs(nstation)
    out = np.zeros((nchan, s1.size, npol * npol), dtype=np.complex128)
    for f in range(nchan):
        X = xc[:, f, :].T  # [N][T]
        V = X @ X.conj().T
        for p in range(npol):
            for q in range(npol):
                out[f, :, p * npol + q] = V[s1 * npol + p, s2 * npol + q]
    return out


def as_complex_out(o: np.ndarray) -> np.ndarray:
    """[..., 2] real pairs -> complex128 [...]."""
    return o[..., 0].astype(np.float64) + 1j * o[..., 1].astype(np.float64)


def full_matrix(vis: np.ndarray, nstation: int, npol: int) -> np.ndarray:
    """Packed complex [nbl][npol*npol] of one channel -> full Hermitian [N][N]."""
    n = nstation * npol
    V = np.zeros((n, n), dtype=np.complex128)
    s1, s2 = station_pairs(nstation)
    for p in range(npol):
        for q in range(npol):
            V[s1 * npol + p, s2 * npol + q] = vis[:, p * npol + q]
            V[s2 * npol + q, s1 * npol + p] = np.conj(vis[:, p * npol + q])
    return V
