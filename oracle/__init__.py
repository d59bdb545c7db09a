"""CPU oracle for the X-engine (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product path never does: it shares no code with the oracle.

The library is plain C (``xcorr_oracle.c``), compiled with gcc -O2 and OpenMP over
channels; see that file for the definition it implements (Sec. 2.1, Eq. 4, lower triangle).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xcorr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CI8, CI4, CF32 = 0, 1, 2

_lib = None


def build(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile the oracle (always; cheap).  Returns the library path."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", *extra, src, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def load(path: str = LIB):
    lib = ctypes.CDLL(path)
    lib.oracle_xcorr_int.restype = ctypes.c_int
    lib.oracle_xcorr_int.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p]
    lib.oracle_xcorr_f64.restype = ctypes.c_int
    lib.oracle_xcorr_f64.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    lib.oracle_num_threads.restype = ctypes.c_int
    return lib


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = load()
    return _lib


def num_threads() -> int:
    return int(_get().oracle_num_threads())


def xcorr(x, nstation: int, npol: int, fmt: int = CI8, chans=None, lib=None) -> np.ndarray:
    """Visibilities of x for the selected channels.

    x: ci8 int8 [T][F][nstation*npol][2], ci4 uint8 [T][F][nstation*npol], or cf32 float32
    [T][F][nstation*npol][2].  Returns int64 (integer formats) or float64 (cf32) with shape
    [len(chans)][nstation*(nstation+1)/2][npol*npol][2].
    """
    lib = lib or _get()
    x = np.ascontiguousarray(x)
    ntime, nchan = int(x.shape[0]), int(x.shape[1])
    nin = nstation * npol
    if x.shape[2] != nin:
        raise ValueError(f"input has {x.shape[2]} inputs, expected {nin}")
    chans = np.arange(nchan, dtype=np.int32) if chans is None else np.asarray(chans, dtype=np.int32)
    if chans.size and (chans.min() < 0 or chans.max() >= nchan):
        raise ValueError("channel out of range")
    nbl = nstation * (nstation + 1) // 2
    shape = (chans.size, nbl, npol * npol, 2)
    if fmt == CF32:
        if x.dtype != np.float32 or x.shape[-1] != 2:
            raise ValueError("cf32 input must be float32 [..., 2]")
        out = np.zeros(shape, dtype=np.float64)
        rc = lib.oracle_xcorr_f64(x.ctypes.data, nstation, npol, nchan, ntime,
                                  chans.ctypes.data, chans.size, out.ctypes.data)
    else:
        if fmt == CI8 and (x.dtype != np.int8 or x.shape[-1] != 2):
            raise ValueError("ci8 input must be int8 [..., 2]")
        if fmt == CI4 and (x.dtype != np.uint8 or x.ndim != 3):
            raise ValueError("ci4 input must be uint8 [T][F][N_in]")
        out = np.zeros(shape, dtype=np.int64)
        rc = lib.oracle_xcorr_int(x.ctypes.data, fmt, nstation, npol, nchan, ntime,
                                  chans.ctypes.data, chans.size, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out
