"""MI355X-native X-engine: time-integrated lower-triangle visibilities of every station and
polarisation pair, per frequency channel (Clark, La Plante and Greenhill, Sec. 2.1, Eq. 4).

The compute path lives in the HIP library ``libxcorr.so`` (built from ``csrc/``) behind a
C ABI declared in ``include/xcorr.h``; :mod:`paper_1107_4264_amd.xcorr` is its thin ctypes
binding.  :mod:`paper_1107_4264_amd.synth` generates seeded synthetic voltages.
"""

__all__ = ["synth", "xcorr"]
