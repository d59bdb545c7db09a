"""Thin ctypes binding of ``libxcorr.so`` (the C ABI declared in ``include/xcorr.h``).

Functions carry the C names; they only marshal arguments.  Every step of the X-engine
runs in the HIP kernels of the library.  The convenience class :class:`Correlator` takes
torch tensors for device memory and uses torch's current HIP stream.

There is no fallback: if the library is missing or fails to load, importing this module
raises.
"""

from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("XCORR_LIB", os.path.join(HERE, "libxcorr.so"))
HEADER = os.path.join(os.path.dirname(HERE), "include", "xcorr.h")

# enumerators of xcorr.h
IN_CI8, IN_CI4, IN_CF32 = 0, 1, 2
ACC_F32_CMAC, ACC_I8_MMA_I32, ACC_F16_MMA_F32, ACC_F8E4M3_MMA_F32, ACC_F32_MMA_F32, ACC_F6E3M2_MMA_F32 = range(6)
OUT_CI32, OUT_CI64, OUT_C64, OUT_C128 = 0, 1, 2, 3
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OOM, ERR_HIP, ERR_RANGE = 0, -1, -2, -3, -4, -5

IN_NAMES = {"ci8": IN_CI8, "ci4": IN_CI4, "cf32": IN_CF32}
ACC_NAMES = {"f32": ACC_F32_CMAC, "i8": ACC_I8_MMA_I32, "f16": ACC_F16_MMA_F32, "f8": ACC_F8E4M3_MMA_F32,
             "f32m": ACC_F32_MMA_F32, "f6": ACC_F6E3M2_MMA_F32}


class XcorrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"xcorr error {code}: {msg}")
        self.code = code


class Job(ctypes.Structure):
    _fields_ = [("nstation", ctypes.c_int), ("npol", ctypes.c_int), ("nchan", ctypes.c_int),
                ("ntime", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("nin", ctypes.c_int), ("tile", ctypes.c_int), ("ntile_side", ctypes.c_int),
        ("tiles_per_chan", ctypes.c_int), ("window", ctypes.c_int), ("nwindows", ctypes.c_int),
        ("max_abs", ctypes.c_int), ("out_dtype", ctypes.c_int), ("nitems", ctypes.c_int64),
        ("useful_cmacs", ctypes.c_int64), ("computed_cmacs", ctypes.c_int64),
        ("in_bytes", ctypes.c_size_t), ("out_bytes", ctypes.c_size_t),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run python -m paper_1107_4264_amd.build")
    # torch ships its own HIP runtime with the same soname.  Loading torch first makes the
    # library bind to that one runtime; the other order would put two runtimes in the
    # process, and the second one finds no device.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_i64, c_sz, c_vp = ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
    sig = {
        "xcorr_create": (c_vp, [c_int, c_int, c_int, c_int, c_int, c_int]),
        "xcorr_set_max_abs": (c_int, [c_vp, c_int]),
        "xcorr_set_tile": (c_int, [c_vp, c_int]),
        "xcorr_get_tile": (c_int, [c_vp]),
        "xcorr_set_window": (c_int, [c_vp, c_int]),
        "xcorr_stream_set_window": (c_int, [c_vp, c_int]),
        "xcorr_autotune": (c_int, [c_vp, c_vp, c_vp, c_vp, c_int]),
        "xcorr_autotune_lookup": (c_int, [ctypes.c_char_p, c_int, c_int, c_int, c_int, c_int, c_int, c_int,
                                          ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
        "xcorr_autotune_results": (c_int, [c_vp, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                           ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_double)]),
        "xcorr_set_staging": (c_int, [c_vp, c_int]),
        "xcorr_get_staging": (c_int, [c_vp]),
        "xcorr_set_variant": (c_int, [c_vp, c_int]),
        "xcorr_get_variant": (c_int, [c_vp]),
        "xcorr_autotune_save": (c_int, [ctypes.c_char_p]),
        "xcorr_autotune_load": (c_int, [ctypes.c_char_p]),
        "xcorr_autotune_clear": (None, []),
        "xcorr_run": (c_int, [c_vp, c_vp, c_vp, c_vp]),
        "xcorr_validate": (c_int, [c_vp, c_vp, c_vp, ctypes.POINTER(c_i64)]),
        "xcorr_set_validation": (c_int, [c_vp, c_int]),
        "xcorr_destroy": (None, [c_vp]),
        "xcorr_in_bytes": (c_sz, [c_vp]),
        "xcorr_out_bytes": (c_sz, [c_vp]),
        "xcorr_out_type": (c_int, [c_vp]),
        "xcorr_last_error": (ctypes.c_char_p, []),
        "xcorr_plan": (c_int, [c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int,
                               ctypes.POINTER(PlanInfo)]),
        "xcorr_window_limit": (c_i64, [c_int, c_int, c_int]),
        "xcorr_tile_coords": (c_int, [c_i64, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
        "xcorr_batch_create": (c_vp, [c_int, c_vp, c_int, c_int]),
        "xcorr_batch_set_max_abs": (c_int, [c_vp, c_int]),
        "xcorr_batch_run": (c_int, [c_vp, c_vp, c_vp, c_vp]),
        "xcorr_batch_in_bytes": (c_sz, [c_vp, c_int]),
        "xcorr_batch_out_bytes": (c_sz, [c_vp, c_int]),
        "xcorr_batch_out_type": (c_int, [c_vp, c_int]),
        "xcorr_batch_items": (c_i64, [c_vp]),
        "xcorr_batch_destroy": (None, [c_vp]),
        "xcorr_batch_run_noalloc": (c_int, [c_int, c_vp, c_int, c_int, c_int, c_vp, c_vp, c_vp]),
        "xcorr_stream_create": (c_vp, [c_int, c_int, c_int, c_int, c_int, c_int]),
        "xcorr_stream_set_max_abs": (c_int, [c_vp, c_int]),
        "xcorr_stream_begin": (c_int, [c_vp, c_vp, c_vp]),
        "xcorr_stream_push": (c_int, [c_vp, c_vp, c_vp]),
        "xcorr_stream_end": (c_i64, [c_vp, c_vp]),
        "xcorr_stream_chunk_bytes": (c_sz, [c_vp]),
        "xcorr_stream_out_bytes": (c_sz, [c_vp]),
        "xcorr_stream_out_type": (c_int, [c_vp]),
        "xcorr_stream_destroy": (None, [c_vp]),
        "xcorr_stream_capture": (c_int, [c_vp, c_int, c_vp, c_vp, ctypes.POINTER(c_vp)]),
        "xcorr_graph_launch": (c_int, [c_vp, c_vp]),
        "xcorr_graph_destroy": (None, [c_vp]),
        "xcorr_fengine_create": (c_vp, [c_int, c_int, c_int, c_int, ctypes.c_float]),
        "xcorr_fengine_in_bytes": (c_sz, [c_vp]),
        "xcorr_fengine_out_bytes": (c_sz, [c_vp, c_int]),
        "xcorr_fengine_run": (c_int, [c_vp, c_vp, c_vp, c_vp]),
        "xcorr_fengine_run_spectra": (c_int, [c_vp, c_vp, c_vp, c_vp]),
        "xcorr_fengine_destroy": (None, [c_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def header_functions(path: str = HEADER):
    """Names of the functions declared in the public header."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xcorr_[a-z0-9_]+)\s*\(", text)))


def last_error() -> str:
    return (_lib.xcorr_last_error() or b"").decode()


def _check(rc):
    if rc < 0:
        raise XcorrError(rc, last_error())
    return rc


# ------------------------------------------------------------------ C-named wrappers

def xcorr_create(nstation, npol, nchan, ntime, in_dtype, acc_dtype):
    h = _lib.xcorr_create(nstation, npol, nchan, ntime, in_dtype, acc_dtype)
    if not h:
        raise XcorrError(-1, last_error())
    return h


def xcorr_set_max_abs(h, max_abs):
    return _check(_lib.xcorr_set_max_abs(h, max_abs))


def xcorr_set_tile(h, tile):
    return _check(_lib.xcorr_set_tile(h, tile))


def xcorr_get_tile(h):
    return _check(_lib.xcorr_get_tile(h))


def xcorr_set_window(h, window):
    return _check(_lib.xcorr_set_window(h, window))


def xcorr_autotune(h, in_ptr, out_ptr, stream_ptr, reps=3):
    return _check(_lib.xcorr_autotune(h, in_ptr, out_ptr, stream_ptr, reps))


def xcorr_autotune_lookup(nstation, npol, nchan, ntime, in_dtype, acc_dtype, max_abs=0, arch=None, full=False):
    """Tile cached for the job's class (0: none); with full=True, (tile, staging, variant)."""
    st, var = ctypes.c_int(0), ctypes.c_int(0)
    t = _check(_lib.xcorr_autotune_lookup(arch.encode() if arch else None, nstation, npol, nchan, ntime, in_dtype,
                                          acc_dtype, max_abs, ctypes.byref(st), ctypes.byref(var)))
    return (t, st.value, var.value) if full else t


def xcorr_autotune_results(h):
    """Shapes timed by the handle's last autotune: list of dicts (tile, staging, variant, us)."""
    n = _check(_lib.xcorr_autotune_results(h, -1, None, None, None, None))
    res = []
    for k in range(n):
        t, st, var, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _lib.xcorr_autotune_results(h, k, ctypes.byref(t), ctypes.byref(st), ctypes.byref(var), ctypes.byref(us))
        res.append({"tile": t.value, "staging": st.value, "variant": var.value, "us": us.value})
    return res


def xcorr_set_staging(h, staging):
    return _check(_lib.xcorr_set_staging(h, staging))


def xcorr_get_staging(h):
    return _check(_lib.xcorr_get_staging(h))


def xcorr_set_variant(h, variant):
    return _check(_lib.xcorr_set_variant(h, variant))


def xcorr_get_variant(h):
    return _check(_lib.xcorr_get_variant(h))


def xcorr_autotune_save(path):
    return _check(_lib.xcorr_autotune_save(os.fsencode(path)))


def xcorr_autotune_load(path):
    return _check(_lib.xcorr_autotune_load(os.fsencode(path)))


def xcorr_autotune_clear():
    _lib.xcorr_autotune_clear()


def xcorr_run(h, in_ptr, out_ptr, stream_ptr):
    return _check(_lib.xcorr_run(h, in_ptr, out_ptr, stream_ptr))


def xcorr_validate(h, in_ptr, stream_ptr):
    n = ctypes.c_int64(0)
    _check(_lib.xcorr_validate(h, in_ptr, stream_ptr, ctypes.byref(n)))
    return int(n.value)


def xcorr_set_validation(h, on):
    return _check(_lib.xcorr_set_validation(h, int(on)))


def xcorr_destroy(h):
    _lib.xcorr_destroy(h)


def xcorr_in_bytes(h):
    return int(_lib.xcorr_in_bytes(h))


def xcorr_out_bytes(h):
    return int(_lib.xcorr_out_bytes(h))


def xcorr_out_type(h):
    return _check(_lib.xcorr_out_type(h))


def xcorr_plan(nstation, npol, nchan, ntime, in_dtype, acc_dtype, max_abs=0, tile=0, window=0):
    info = PlanInfo()
    _check(_lib.xcorr_plan(nstation, npol, nchan, ntime, in_dtype, acc_dtype, max_abs, tile, window,
                           ctypes.byref(info)))
    return info.as_dict()


def xcorr_window_limit(in_dtype, acc_dtype, max_abs):
    return _check(_lib.xcorr_window_limit(in_dtype, acc_dtype, max_abs))


def xcorr_tile_coords(g):
    bx, by = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.xcorr_tile_coords(g, ctypes.byref(bx), ctypes.byref(by)))
    return bx.value, by.value


def xcorr_batch_create(jobs, in_dtype, acc_dtype):
    """jobs: sequence of dicts or tuples (nstation, npol, nchan, ntime)."""
    arr = (Job * len(jobs))()
    for k, j in enumerate(jobs):
        if isinstance(j, dict):
            j = (j["nstation"], j["npol"], j["nchan"], j["ntime"])
        arr[k] = Job(*j)
    b = _lib.xcorr_batch_create(len(jobs), ctypes.cast(arr, ctypes.c_void_p), in_dtype, acc_dtype)
    if not b:
        raise XcorrError(-1, last_error())
    return b


def xcorr_batch_set_max_abs(b, max_abs):
    return _check(_lib.xcorr_batch_set_max_abs(b, max_abs))


def xcorr_batch_run(b, in_ptrs, out_ptrs, stream_ptr):
    n = len(in_ptrs)
    ins = (ctypes.c_void_p * n)(*in_ptrs)
    outs = (ctypes.c_void_p * n)(*out_ptrs)
    return _check(_lib.xcorr_batch_run(b, ctypes.cast(ins, ctypes.c_void_p), ctypes.cast(outs, ctypes.c_void_p),
                                       stream_ptr))


def xcorr_batch_in_bytes(b, job):
    return int(_lib.xcorr_batch_in_bytes(b, job))


def xcorr_batch_out_bytes(b, job):
    return int(_lib.xcorr_batch_out_bytes(b, job))


def xcorr_batch_out_type(b, job):
    return _check(_lib.xcorr_batch_out_type(b, job))


def xcorr_batch_items(b):
    return int(_lib.xcorr_batch_items(b))


def xcorr_batch_destroy(b):
    _lib.xcorr_batch_destroy(b)


def xcorr_batch_run_noalloc(jobs, in_dtype, acc_dtype, max_abs, in_ptrs, out_ptrs, stream_ptr):
    """jobs: sequence of dicts or tuples (nstation, npol, nchan, ntime)."""
    n = len(jobs)
    arr = (Job * n)()
    for k, j in enumerate(jobs):
        if isinstance(j, dict):
            j = (j["nstation"], j["npol"], j["nchan"], j["ntime"])
        arr[k] = Job(*j)
    ins = (ctypes.c_void_p * n)(*in_ptrs)
    outs = (ctypes.c_void_p * n)(*out_ptrs)
    return _check(_lib.xcorr_batch_run_noalloc(n, ctypes.cast(arr, ctypes.c_void_p), in_dtype, acc_dtype, max_abs,
                                               ctypes.cast(ins, ctypes.c_void_p), ctypes.cast(outs, ctypes.c_void_p),
                                               stream_ptr))


def xcorr_stream_create(nstation, npol, nchan, chunk_ntime, in_dtype, acc_dtype):
    s = _lib.xcorr_stream_create(nstation, npol, nchan, chunk_ntime, in_dtype, acc_dtype)
    if not s:
        raise XcorrError(-1, last_error())
    return s


def xcorr_stream_set_max_abs(s, max_abs):
    return _check(_lib.xcorr_stream_set_max_abs(s, max_abs))


def xcorr_stream_set_window(s, window):
    return _check(_lib.xcorr_stream_set_window(s, window))


def xcorr_stream_begin(s, out_ptr, stream_ptr):
    return _check(_lib.xcorr_stream_begin(s, out_ptr, stream_ptr))


def xcorr_stream_push(s, host_ptr, stream_ptr):
    return _check(_lib.xcorr_stream_push(s, host_ptr, stream_ptr))


def xcorr_stream_end(s, stream_ptr):
    return _check(_lib.xcorr_stream_end(s, stream_ptr))


def xcorr_stream_chunk_bytes(s):
    return int(_lib.xcorr_stream_chunk_bytes(s))


def xcorr_stream_out_bytes(s):
    return int(_lib.xcorr_stream_out_bytes(s))


def xcorr_stream_out_type(s):
    return _check(_lib.xcorr_stream_out_type(s))


def xcorr_stream_destroy(s):
    _lib.xcorr_stream_destroy(s)


def xcorr_stream_capture(s, host_ptrs, out_ptr):
    """Instantiated graph (as an integer handle) of a whole integration over host_ptrs."""
    n = len(host_ptrs)
    arr = (ctypes.c_void_p * n)(*host_ptrs)
    ex = ctypes.c_void_p()
    _check(_lib.xcorr_stream_capture(s, n, ctypes.cast(arr, ctypes.c_void_p), out_ptr, ctypes.byref(ex)))
    return ex.value


def xcorr_graph_launch(exec_handle, stream_ptr):
    return _check(_lib.xcorr_graph_launch(ctypes.c_void_p(exec_handle), stream_ptr))


def xcorr_graph_destroy(exec_handle):
    _lib.xcorr_graph_destroy(ctypes.c_void_p(exec_handle))


# ------------------------------------------------------------------ torch convenience

def xcorr_fengine_create(nstation, npol, nchan, nframes, gain):
    e = _lib.xcorr_fengine_create(nstation, npol, nchan, nframes, float(gain))
    if not e:
        raise XcorrError(-1, last_error())
    return e


def xcorr_fengine_in_bytes(e):
    return int(_lib.xcorr_fengine_in_bytes(e))


def xcorr_fengine_out_bytes(e, spectra=0):
    return int(_lib.xcorr_fengine_out_bytes(e, int(spectra)))


def xcorr_fengine_run(e, in_ptr, out_ptr, stream_ptr):
    return _check(_lib.xcorr_fengine_run(e, in_ptr, out_ptr, stream_ptr))


def xcorr_fengine_run_spectra(e, in_ptr, out_ptr, stream_ptr):
    return _check(_lib.xcorr_fengine_run_spectra(e, in_ptr, out_ptr, stream_ptr))


def xcorr_fengine_destroy(e):
    _lib.xcorr_fengine_destroy(e)


def out_torch_dtype(out_type):
    import torch

    return {OUT_CI32: torch.int32, OUT_CI64: torch.int64, OUT_C64: torch.float32,
            OUT_C128: torch.float64}[out_type]


def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Correlator:
    """One planned job.  ``in_dtype`` / ``acc`` take the enumerators or the short names
    ('ci8', 'ci4', 'cf32' / 'f32', 'i8', 'f16', 'f8')."""

    def __init__(self, nstation, npol, nchan, ntime, in_dtype="ci8", acc="f16", max_abs=None, tile=None,
                 window=None, staging=None, variant=None, validate=False):
        self.nstation, self.npol, self.nchan, self.ntime = nstation, npol, nchan, ntime
        self.in_dtype = IN_NAMES.get(in_dtype, in_dtype)
        self.acc = ACC_NAMES.get(acc, acc)
        self.h = xcorr_create(nstation, npol, nchan, ntime, self.in_dtype, self.acc)
        if max_abs is not None:
            xcorr_set_max_abs(self.h, int(max_abs))
        if window is not None:
            xcorr_set_window(self.h, int(window))
        if staging is not None:
            xcorr_set_staging(self.h, int(staging))
        if tile is not None:
            xcorr_set_tile(self.h, int(tile))
        if variant is not None:
            xcorr_set_variant(self.h, int(variant))
        if validate:
            xcorr_set_validation(self.h, 1)

    @property
    def tile(self):
        return xcorr_get_tile(self.h)

    @property
    def staging(self):
        return xcorr_get_staging(self.h)

    @property
    def variant(self):
        return xcorr_get_variant(self.h)

    def close(self):
        if self.h:
            xcorr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def out_type(self):
        return xcorr_out_type(self.h)

    @property
    def nbl(self):
        return self.nstation * (self.nstation + 1) // 2

    def out_shape(self):
        return (self.nchan, self.nbl, self.npol * self.npol, 2)

    def empty_out(self, device="cuda"):
        import torch

        return torch.empty(self.out_shape(), dtype=out_torch_dtype(self.out_type), device=device)

    def autotune(self, x, out=None, reps=3, stream=None):
        """Time every allowed kernel shape on x and keep the fastest; returns the tile."""
        if out is None:
            out = self.empty_out(x.device)
        return xcorr_autotune(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              _stream_ptr(stream), reps)

    def count_out_of_range(self, x, stream=None):
        """Number of sample components of x outside [-max_abs, max_abs] (waits for the
        stream)."""
        if not x.is_cuda or x.numel() * x.element_size() != xcorr_in_bytes(self.h):
            raise ValueError("input must be a device tensor of the plan's size")
        return xcorr_validate(self.h, ctypes.c_void_p(x.data_ptr()), _stream_ptr(stream))

    def run(self, x, out=None, stream=None):
        """x: device tensor holding xcorr_in_bytes bytes of samples; returns the output."""
        if not x.is_cuda:
            raise ValueError("input must be a device tensor")
        if x.numel() * x.element_size() != xcorr_in_bytes(self.h):
            raise ValueError("input size does not match the plan")
        if out is None:
            out = self.empty_out(x.device)
        if out.numel() * out.element_size() != xcorr_out_bytes(self.h) or out.dtype != out_torch_dtype(self.out_type):
            raise ValueError("output buffer does not match the plan")
        xcorr_run(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        return out


class Batch:
    """Many jobs in one persistent launch (torch tensors for memory)."""

    def __init__(self, jobs, in_dtype="ci8", acc="i8", max_abs=None):
        self.jobs = [j if isinstance(j, dict) else dict(zip(("nstation", "npol", "nchan", "ntime"), j))
                     for j in jobs]
        self.in_dtype = IN_NAMES.get(in_dtype, in_dtype)
        self.acc = ACC_NAMES.get(acc, acc)
        self.b = xcorr_batch_create(self.jobs, self.in_dtype, self.acc)
        if max_abs is not None:
            xcorr_batch_set_max_abs(self.b, int(max_abs))


    def close(self):
        if self.b:
            xcorr_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def out_shape(self, k):
        j = self.jobs[k]
        nbl = j["nstation"] * (j["nstation"] + 1) // 2
        return (j["nchan"], nbl, j["npol"] * j["npol"], 2)

    def empty_outs(self, device="cuda"):
        import torch

        return [torch.empty(self.out_shape(k), dtype=out_torch_dtype(xcorr_batch_out_type(self.b, k)), device=device)
                for k in range(len(self.jobs))]

    def run(self, xs, outs=None, stream=None):
        if len(xs) != len(self.jobs):
            raise ValueError("one input per job")
        for k, x in enumerate(xs):
            if x.numel() * x.element_size() != xcorr_batch_in_bytes(self.b, k):
                raise ValueError(f"input {k} size does not match the plan")
        if outs is None:
            outs = self.empty_outs(xs[0].device)
        for k, o in enumerate(outs):
            if o.numel() * o.element_size() != xcorr_batch_out_bytes(self.b, k):
                raise ValueError(f"output {k} size does not match the plan")
        xcorr_batch_run(self.b, [x.data_ptr() for x in xs], [o.data_ptr() for o in outs], _stream_ptr(stream))
        return outs


class Stream:
    """Chunked integration with copy/compute overlap (Algorithm 1).  Chunks are host tensors
    (pinned for asynchronous copies); totals are a device tensor of the wide type."""

    def __init__(self, nstation, npol, nchan, chunk_ntime, in_dtype="ci8", acc="i8", max_abs=None, window=None):
        self.nstation, self.npol, self.nchan, self.chunk_ntime = nstation, npol, nchan, chunk_ntime
        self.s = xcorr_stream_create(nstation, npol, nchan, chunk_ntime, IN_NAMES.get(in_dtype, in_dtype),
                                     ACC_NAMES.get(acc, acc))
        if max_abs is not None:
            xcorr_stream_set_max_abs(self.s, int(max_abs))
        if window is not None:
            xcorr_stream_set_window(self.s, int(window))
        self.out = None
        # host chunks whose copies may still be in flight (released as the library does:
        # push p releases chunk p - 2; end releases the rest once the stream is synchronised)
        self._inflight = []

    def close(self):
        if self.s:
            xcorr_stream_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_out(self, device="cuda"):
        import torch

        nbl = self.nstation * (self.nstation + 1) // 2
        return torch.empty((self.nchan, nbl, self.npol * self.npol, 2),
                           dtype=out_torch_dtype(xcorr_stream_out_type(self.s)), device=device)

    def begin(self, out=None, stream=None):
        self.out = self.empty_out() if out is None else out
        if self.out.numel() * self.out.element_size() != xcorr_stream_out_bytes(self.s):
            raise ValueError("totals buffer does not match the plan")
        xcorr_stream_begin(self.s, ctypes.c_void_p(self.out.data_ptr()), _stream_ptr(stream))
        return self.out

    def push(self, chunk, stream=None):
        if chunk.is_cuda:
            raise ValueError("chunks come from host memory")
        if chunk.numel() * chunk.element_size() != xcorr_stream_chunk_bytes(self.s):
            raise ValueError("chunk size does not match the plan")
        xcorr_stream_push(self.s, ctypes.c_void_p(chunk.data_ptr()), _stream_ptr(stream))
        self._inflight.append(chunk)
        del self._inflight[:-2]

    def end(self, stream=None):
        """Finish the integration; synchronises `stream` so that every pushed chunk is
        released (its copy has completed)."""
        import torch

        n = xcorr_stream_end(self.s, _stream_ptr(stream))
        (stream if stream is not None else torch.cuda.current_stream()).synchronize()
        self._inflight.clear()
        return n

    def capture(self, chunks, out=None):
        """A HIP graph of a whole integration over these host chunks into `out`: each
        launch zeroes `out` and integrates the chunks' current contents."""
        out = self.empty_out() if out is None else out
        if out.numel() * out.element_size() != xcorr_stream_out_bytes(self.s):
            raise ValueError("totals buffer does not match the plan")
        for ch in chunks:
            if ch.is_cuda or ch.numel() * ch.element_size() != xcorr_stream_chunk_bytes(self.s):
                raise ValueError("chunks must be host tensors of xcorr_stream_chunk_bytes")
        ex = xcorr_stream_capture(self.s, [ch.data_ptr() for ch in chunks], ctypes.c_void_p(out.data_ptr()))
        return Graph(ex, out, list(chunks))


class Graph:
    """An instantiated HIP graph of the library (keeps its buffers alive)."""

    def __init__(self, exec_handle, out, keep):
        self.exec = exec_handle
        self.out = out
        self._keep = keep

    def launch(self, stream=None):
        xcorr_graph_launch(self.exec, _stream_ptr(stream))
        return self.out

    def close(self):
        if self.exec:
            xcorr_graph_destroy(self.exec)
            self.exec = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FEngine:
    """F-engine and corner turn: int8 [nin][nframes * nchan][2] voltages -> int8
    [nframes][nchan][nin][2] requantised spectra (the X-engine's input), or complex float
    spectra with run(..., spectra=True)."""

    def __init__(self, nstation, npol, nchan, nframes, gain):
        self.nstation, self.npol, self.nchan, self.nframes = nstation, npol, nchan, nframes
        self.nin = nstation * npol
        self.e = xcorr_fengine_create(nstation, npol, nchan, nframes, gain)

    def close(self):
        if self.e:
            xcorr_fengine_destroy(self.e)
            self.e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_out(self, device="cuda", spectra=False):
        import torch

        if spectra:
            return torch.empty((self.nframes, self.nchan, self.nin, 2), dtype=torch.float32, device=device)
        return torch.empty((self.nframes, self.nchan, self.nin, 2), dtype=torch.int8, device=device)

    def run(self, x, out=None, spectra=False, stream=None):
        if not x.is_cuda:
            raise ValueError("input must be a device tensor")
        if x.numel() * x.element_size() != xcorr_fengine_in_bytes(self.e):
            raise ValueError("input size does not match the F-engine")
        if out is None:
            out = self.empty_out(x.device, spectra)
        if out.numel() * out.element_size() != xcorr_fengine_out_bytes(self.e, spectra):
            raise ValueError("output buffer does not match the F-engine")
        fn = xcorr_fengine_run_spectra if spectra else xcorr_fengine_run
        fn(self.e, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        return out
