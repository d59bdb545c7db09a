"""Arithmetic-intensity and roofline model of the X-engine (Sec. 2.2, Sec. 4.1 / Table 1).

The paper's tile arithmetic (checked against Table 1 by the tests) and the MI355X peaks; the
benchmark takes its per-launch bytes and operation counts from the planner instead.  No part
of the compute path.
"""

from __future__ import annotations

import math

# MI355X published peaks (dense, no sparsity).
MI355X = {
    "hbm_gbps": 8000.0,
    "tflops": {"f32_vector": 157.3, "f32_vector_unpacked": 78.6, "f16": 2500.0, "fp8": 5000.0,
               "i8": 5000.0, "f64": 78.6},
    "cus": 256,
    "clock_ghz": 2.4,
}


def tile_ai(m: float, n: float, integration: float, word: float = 4.0) -> float:
    """Flops per byte of an m x n tile of baselines integrated over I samples with dual-pol
    float inputs (Sec. 2.2): 32 flops per baseline-sample, 4 words per station-sample loaded
    for the row and column, 16 words read+written per baseline accumulator.  With
    word = 4 bytes this is 32mnI / (16(m+n)I + 64mn)."""
    return 32.0 * m * n * integration / (4 * word * (m + n) * integration + 16 * word * m * n)


def tile_registers(m: int, n: int) -> int:
    """Registers of an m x n register tile: 8mn accumulators plus 4(m+n) operands (Sec. 2.2)."""
    return 8 * m * n + 4 * (m + n)


def staging_bytes(m: int, n: int, word: int = 4) -> int:
    """Storage of the input vectors of an m x n tile at an outer level: 4(m+n) words (Sec. 2.2)."""
    return 4 * (m + n) * word


def required_square_tile(ai_required: float) -> int:
    """For large I the AI of an m x m tile tends to m, so the tile must be at least the
    required intensity (Table 1)."""
    return max(1, math.ceil(ai_required - 1e-9))


def useful_cmacs(nin: int, nchan: int, ntime: int) -> int:
    """Complex MACs of Eq. 5 integrated: nin(nin+1)/2 pairs per channel and sample."""
    return nin * (nin + 1) // 2 * nchan * ntime


def algorithmic_bytes(nin: int, nchan: int, ntime: int, in_bytes_per_sample: int,
                      nstation: int, npol: int, out_bytes_per_value: int) -> int:
    """Input read once plus output written once."""
    nbl = nstation * (nstation + 1) // 2
    return nin * nchan * ntime * in_bytes_per_sample + nchan * nbl * npol * npol * out_bytes_per_value
