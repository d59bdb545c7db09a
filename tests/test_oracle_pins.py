"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test ties the oracle to something other than itself:
  * brute force: X @ X^H per channel (numpy) and the BLAS Hermitian rank-k update (zherk);
  * closed forms: one time sample is one outer product; a single noiseless point source
    gives V_ij = a_i conj(a_j) sum_t |s(t)|^2 (fixes the conjugated side and the
    polarisation order);
  * invariants: real non-negative autocorrelations, Hermitian cross-polarisation autos,
    Cauchy-Schwarz;
  * metamorphic relations that hold exactly in integers.
The last test plants mistakes in copies of the oracle source and checks that the pins fail.
"""

from __future__ import annotations


import numpy as np
import pytest
from scipy.linalg import blas

from paper_1107_4264_amd import synth
from tests import refmath

SHAPES = [(ns, npol, T) for ns in (1, 2, 3, 5, 17) for npol in (1, 2) for T in (1, 2, 7)]


def _rand(seed, T, F, nin, dist=("uniform", -8, 7)):
    return synth.voltages_np(seed, T, F, nin, dist)


@pytest.mark.parametrize("ns,npol,T", SHAPES)
def test_matches_matrix_product(oracle_mod, ns, npol, T):
    F = 3
    x = _rand(100 + ns * 7 + npol * 3 + T, T, F, ns * npol, ("gauss", 40.0, 127))
    got = refmath.as_complex_out(oracle_mod.xcorr(x, ns, npol))
    want = refmath.brute(x, ns, npol)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("ns,T", [(1, 1), (4, 3), (9, 16), (23, 5)])
def test_single_pol_is_blas_herk(oracle_mod, ns, T):
    """npol = 1 reduces to a plain Hermitian rank-k update: lower triangle of A A^H."""
    F = 2
    x = _rand(7 + ns, T, F, ns, ("gauss", 50.0, 127))
    got = refmath.as_complex_out(oracle_mod.xcorr(x, ns, 1))
    xc = refmath.to_complex(x)
    for f in range(F):
        A = np.asfortranarray(xc[:, f, :].T)  # [N][T]
        C = blas.zherk(1.0, A, lower=1)
        rows, cols = np.tril_indices(ns)
        assert np.array_equal(got[f, :, 0], C[rows, cols])


def test_ci4_matches_unpacked(oracle_mod):
    ns, npol, T, F = 6, 2, 9, 4
    v = _rand(31, T, F, ns * npol)
    packed = synth.pack_ci4(v)
    assert np.array_equal(synth.unpack_ci4(packed), v)
    got = oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4)
    want = oracle_mod.xcorr(v, ns, npol)
    assert np.array_equal(got, want)
    assert np.array_equal(refmath.as_complex_out(got), refmath.brute(v, ns, npol))


def test_ci4_nibble_convention(oracle_mod):
    """Real part in the high nibble, imaginary in the low nibble, two's complement."""
    # one station, one pol, one sample: 0x9E -> re = 0x9 - 16 = -7, im = 0xE - 16 = -2
    x = np.array([[[0x9E]]], dtype=np.uint8)
    o = oracle_mod.xcorr(x, 1, 1, fmt=oracle_mod.CI4)
    assert o[0, 0, 0].tolist() == [49 + 4, 0]
    # two stations: x0 = (1 + 2i) -> 0x12, x1 = (-8 + 7i) -> 0x87
    x = np.array([[[0x12, 0x87]]], dtype=np.uint8)
    o = oracle_mod.xcorr(x, 2, 1, fmt=oracle_mod.CI4)
    # V10 = x1 conj(x0) = (-8 + 7i)(1 - 2i) = -8 + 16i + 7i + 14 = 6 + 23i
    assert o[0, 1, 0].tolist() == [6, 23]


def test_cf32_matches_matrix_product(oracle_mod):
    ns, npol, T, F = 5, 2, 11, 2
    rng = np.random.default_rng(5)
    x = rng.standard_normal((T, F, ns * npol, 2)).astype(np.float32)
    got = refmath.as_complex_out(oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CF32))
    want = refmath.brute(x, ns, npol)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_one_sample_is_outer_product(oracle_mod):
    ns, npol = 4, 2
    x = _rand(9, 1, 1, ns * npol, ("gauss", 30.0, 127))
    o = oracle_mod.xcorr(x, ns, npol)
    v = x[0, 0].astype(np.int64)
    k = 0
    for s1 in range(ns):
        for s2 in range(s1 + 1):
            for p in range(npol):
                for q in range(npol):
                    ar, ai = v[s1 * npol + p]
                    br, bi = v[s2 * npol + q]
                    # (ar + i ai)(br - i bi)
                    assert o[0, k, p * npol + q].tolist() == [ar * br + ai * bi, ai * br - ar * bi]
            k += 1


def test_worked_example_by_hand(oracle_mod):
    """Two single-pol stations over two samples, worked by hand.

    x0 = (1+1i, 2+0i), x1 = (0+1i, 1-1i)
    V00 = |1+i|^2 + |2|^2 = 2 + 4 = 6
    V11 = |i|^2 + |1-i|^2 = 1 + 2 = 3
    V10 = x1 conj(x0) summed = i(1-i) + (1-i)(2) = (i + 1) + (2 - 2i) = 3 - 1i
    """
    x = np.array([[[[1, 1], [0, 1]]], [[[2, 0], [1, -1]]]], dtype=np.int8)
    o = oracle_mod.xcorr(x, 2, 1)
    assert o[0, :, 0].tolist() == [[6, 0], [3, -1], [3, 0]]


def test_point_source_closed_form(oracle_mod):
    ns, npol, T, F = 7, 2, 33, 3
    nin = ns * npol
    x, a, s = synth.point_source_np(0x5EED, T, F, nin)
    o = oracle_mod.xcorr(x, ns, npol)
    ac = a[:, 0] + 1j * a[:, 1]
    power = (s[..., 0].astype(np.int64) ** 2 + s[..., 1].astype(np.int64) ** 2).sum(axis=0)  # [F]
    k = 0
    for s1 in range(ns):
        for s2 in range(s1 + 1):
            for p in range(npol):
                for q in range(npol):
                    i, j = s1 * npol + p, s2 * npol + q
                    g = ac[i] * np.conj(ac[j])
                    for f in range(F):
                        want = g * power[f]
                        assert o[f, k, p * npol + q].tolist() == [int(want.real), int(want.imag)]
            k += 1


def test_invariants(oracle_mod):
    ns, npol, T, F = 9, 2, 40, 3
    x = _rand(77, T, F, ns * npol, ("gauss", 20.0, 127))
    o = refmath.as_complex_out(oracle_mod.xcorr(x, ns, npol))
    autos = [s * (s + 1) // 2 + s for s in range(ns)]
    for k in autos:
        for p in range(npol):
            assert np.all(o[:, k, p * npol + p].imag == 0)
            assert np.all(o[:, k, p * npol + p].real >= 0)
        assert np.array_equal(o[:, k, 1], np.conj(o[:, k, 2]))
    for f in range(F):
        V = refmath.full_matrix(o[f], ns, npol)
        d = np.real(np.diag(V))
        assert np.all(np.abs(V) ** 2 <= np.outer(d, d) * (1 + 1e-12) + 1e-9)
        assert np.array_equal(V, V.conj().T)


def test_metamorphic(oracle_mod):
    ns, npol, T, F = 6, 2, 24, 2
    x = _rand(123, T, F, ns * npol, ("gauss", 10.0, 60))
    base = oracle_mod.xcorr(x, ns, npol)
    # time split: V(T1 u T2) = V(T1) + V(T2)
    assert np.array_equal(base, oracle_mod.xcorr(x[:10], ns, npol) + oracle_mod.xcorr(x[10:], ns, npol))
    # time permutation
    perm = np.random.default_rng(1).permutation(T)
    assert np.array_equal(base, oracle_mod.xcorr(np.ascontiguousarray(x[perm]), ns, npol))
    # multiply every sample by i: (re, im) -> (-im, re)
    xi = np.stack([-x[..., 1], x[..., 0]], axis=-1).astype(np.int8)
    assert np.array_equal(base, oracle_mod.xcorr(xi, ns, npol))
    # conjugate every sample -> conjugate visibilities
    xc = np.stack([x[..., 0], -x[..., 1]], axis=-1).astype(np.int8)
    oc = oracle_mod.xcorr(xc, ns, npol)
    assert np.array_equal(oc[..., 0], base[..., 0]) and np.array_equal(oc[..., 1], -base[..., 1])
    # integer scaling by 2 -> 4 V
    assert np.array_equal(oracle_mod.xcorr((x * 2).astype(np.int8), ns, npol), 4 * base)
    # reversing station order: V'[s1', s2'] with s' = ns-1-s equals conj of the mirrored entry
    xr = np.ascontiguousarray(x.reshape(T, F, ns, npol, 2)[:, :, ::-1].reshape(T, F, ns * npol, 2))
    orv = refmath.as_complex_out(oracle_mod.xcorr(xr, ns, npol))
    bc = refmath.as_complex_out(base)
    for f in range(F):
        Vb = refmath.full_matrix(bc[f], ns, npol)
        Vr = refmath.full_matrix(orv[f], ns, npol)
        idx = np.arange(ns)[::-1]
        order = (idx[:, None] * npol + np.arange(npol)[None, :]).ravel()
        assert np.array_equal(Vr, Vb[np.ix_(order, order)])


def test_overflow_window_bound(oracle_mod):
    """The int32 window bound for 8-bit samples in [-127, 127]: the worst case grows by
    2 * 127^2 per sample (an autocorrelation of -127 - 127i), so floor((2^31 - 1) / 32258)
    samples fit in int32 and one more does not."""
    td = (2**31 - 1) // (2 * 127 * 127)
    x = np.full((td + 1, 1, 2, 2), -127, dtype=np.int8)
    o_fit = oracle_mod.xcorr(x[:td], 2, 1)
    o_over = oracle_mod.xcorr(x, 2, 1)
    assert np.abs(o_fit).max() <= 2**31 - 1
    assert np.abs(o_over).max() > 2**31 - 1
    assert td == 66572


MUTANTS = {
    "conj_on_wrong_side": ("acc_im += ai * br - ar * bi;", "acc_im += ar * bi - ai * br;"),
    "dropped_imag_term": ("acc_re += ar * br + ai * bi;", "acc_re += ar * br;"),
    "pol_transposed": ("tri(s1, s2)) * npp + p * npol + q) * 2;\n                        o[0] = acc_re;",
                       "tri(s1, s2)) * npp + q * npol + p) * 2;\n                        o[0] = acc_re;"),
    "last_sample_dropped": ("for (size_t t = 0; t < (size_t)ntime; ++t) {\n                            const size_t row = (t * (size_t)nchan + f) * nin;\n                            int64_t",
                            "for (size_t t = 1; t < (size_t)ntime; ++t) {\n                            const size_t row = (t * (size_t)nchan + f) * nin;\n                            int64_t"),
    "channel_stride_wrong": ("const size_t row = (t * (size_t)nchan + f) * nin;\n                            int64_t",
                             "const size_t row = (t + f * (size_t)ntime) * nin;\n                            int64_t"),
    "ci4_nibbles_swapped": ("int r = (p[n] >> 4) & 0xF;\n        int i = p[n] & 0xF;",
                            "int i = (p[n] >> 4) & 0xF;\n        int r = p[n] & 0xF;"),
}


def _pins_pass(mod, lib) -> bool:
    """Run a compact set of the pins above against an oracle library; True if all hold."""
    try:
        for ns, npol, T in [(3, 2, 7), (5, 1, 2), (2, 2, 1)]:
            x = _rand(55 + ns, T, 2, ns * npol, ("gauss", 40.0, 127))
            if not np.array_equal(refmath.as_complex_out(mod.xcorr(x, ns, npol, lib=lib)),
                                  refmath.brute(x, ns, npol)):
                return False
        v = _rand(31, 5, 2, 4)
        if not np.array_equal(refmath.as_complex_out(mod.xcorr(synth.pack_ci4(v), 2, 2, fmt=mod.CI4, lib=lib)),
                              refmath.brute(v, 2, 2)):
            return False
    except Exception:
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(oracle_mod, tmp_path, name):
    src = open(oracle_mod.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new)
    path = tmp_path / "mutant.c"
    path.write_text(mutated)
    out = str(tmp_path / "libmutant.so")
    oracle_mod.build(src=str(path), out=out)
    lib = oracle_mod.load(out)
    assert not _pins_pass(oracle_mod, lib), f"mutant {name} survived the pins"
    # and the unmutated oracle passes the same compact pins
    assert _pins_pass(oracle_mod, oracle_mod.load(oracle_mod.LIB))
