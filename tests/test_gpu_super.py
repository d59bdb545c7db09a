"""GPU parity of the super-tiled kernel (tile 512: 4-bit samples on the int8, fp8 or fp6
matrix cores, each channel cut into 256-input triangles and 256 x 128 rectangles, operands
widened in LDS to 8 x the samples as int8, or to fp8 e4m3; fp6 e3m2 units made by a
pre-pass) against the oracle, bit for bit."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, run_xeng, say

pytestmark = pytest.mark.gpu

SHAPES = [
    # (nstation, npol, nchan, ntime)
    (256, 2, 3, 100),    # 512 inputs: 2 triangles + 2 rectangles; last time block partial
    (384, 2, 2, 77),     # 768 inputs: 3 triangles + 6 rectangles
    (512, 2, 2, 70),     # 1024 inputs: 4 triangles + 12 rectangles
    (512, 1, 2, 33),     # single polarisation: the generic store path
    (256, 2, 2, 1),      # a single sample
    (256, 2, 1, 32),     # exactly one block
]


def _check(got, want, label):
    g = as_exact_int(got)
    if not np.array_equal(g, want):
        bad = np.argwhere(g != want)
        say(label, "MISMATCH count", len(bad), "first", bad[:5].tolist(),
            "got", g[tuple(bad[0])], "want", want[tuple(bad[0])])
    assert np.array_equal(g, want), label


ACCS = ["i8", "f8", "f6"]


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_super_matches_oracle(oracle_mod, acc, shape):
    ns, npol, F, T = shape
    v = synth.voltages_np(synth.SEED_BASE + 60 + ns + T, T, F, ns * npol, ("uniform", -8, 7))
    packed = synth.pack_ci4(v)
    say("super", acc, shape)
    got, _ = run_xeng(packed, ns, npol, "ci4", acc, tile=512)
    _check(got, oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4), f"super/{acc}/{shape}")


@pytest.mark.parametrize("acc", ACCS)
def test_super_extreme_values(oracle_mod, acc):
    """Full-scale 4-bit samples, some inputs pinned at -8 (the widened operand -64, whose
    rotation +64 still fits int8)."""
    ns, npol, F, T = 256, 2, 2, 150
    v = synth.voltages_np(synth.SEED_BASE + 61, T, F, ns * npol, ("uniform", -8, 7))
    v[:, :, :6] = -8
    v[:, :, 300:302] = 7
    packed = synth.pack_ci4(v)
    say("super extreme", acc)
    got, _ = run_xeng(packed, ns, npol, "ci4", acc, tile=512)
    _check(got, oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4), f"super-extreme/{acc}")


# channels sampled from a walk over 150 channels of 512 inputs (4 pieces each, 600 items):
# first, second and third items of workgroups, and the last channel
WALK_CHANS = [0, 1, 31, 32, 63, 64, 65, 127, 128, 149]


@pytest.mark.parametrize("acc", ACCS)
def test_super_many_items_per_workgroup(oracle_mod, acc):
    ns, npol, F, T = 256, 2, 150, 40
    v = synth.voltages_np(synth.SEED_BASE + 62, T, F, ns * npol, ("uniform", -8, 7))
    packed = synth.pack_ci4(v)
    say("super walk", acc, F)
    got, _ = run_xeng(packed, ns, npol, "ci4", acc, tile=512)
    want = oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4, chans=WALK_CHANS)
    _check(got[WALK_CHANS], want, f"super-walk/{acc}")


@pytest.mark.parametrize("acc", ACCS)
def test_super_equals_tiles(acc):
    """Super-tiles and 128-tiles give the same bits."""
    ns, npol, F, T = 512, 2, 3, 200
    v = synth.voltages_np(synth.SEED_BASE + 63, T, F, ns * npol, ("uniform", -8, 7))
    packed = synth.pack_ci4(v)
    a, _ = run_xeng(packed, ns, npol, "ci4", acc, tile=512)
    b, _ = run_xeng(packed, ns, npol, "ci4", acc, tile=128)
    assert np.array_equal(a, b)


def test_super_f8_windows(oracle_mod):
    """fp8 super-tiles with two fp32 windows (131072 samples each at the default bound)
    summed into fp64 totals, against the oracle (272 inputs: a full and a partial
    super-row)."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F, T = 136, 2, 1, 131072 + 300
    p = X.xcorr_plan(ns, npol, F, T, X.IN_CI4, X.ACC_F8E4M3_MMA_F32, 0, 512)
    assert p["nwindows"] == 2 and p["out_dtype"] == X.OUT_C128
    packed = synth.pack_ci4(synth.voltages_np(synth.SEED_BASE + 66, T, F, ns * npol, ("uniform", -8, 7)))
    say("super f8 windows", T)
    full, ot = run_xeng(packed, ns, npol, "ci4", "f8", tile=512)
    assert ot == X.OUT_C128
    _check(full, oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4), "super-f8-windows")


def test_super_f6_windows(oracle_mod):
    """fp6 super-tiles with two fp32 windows summed into fp64 totals (the windows start on
    whole 32-sample blocks of the pre-pass's units), against the oracle."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F, T = 136, 2, 1, 131072 + 300
    p = X.xcorr_plan(ns, npol, F, T, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0, 512)
    assert p["nwindows"] == 2 and p["out_dtype"] == X.OUT_C128 and p["window"] % 32 == 0
    packed = synth.pack_ci4(synth.voltages_np(synth.SEED_BASE + 67, T, F, ns * npol, ("uniform", -8, 7)))
    say("super f6 windows", T)
    full, ot = run_xeng(packed, ns, npol, "ci4", "f6", tile=512)
    assert ot == X.OUT_C128
    _check(full, oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4), "super-f6-windows")


def test_super_f6_forced_windows(oracle_mod):
    """Forced windows of whole blocks (96 samples) run on fp6 super-tiles; a window that
    does not start on a block (100 samples) is refused for tile 512."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F, T = 136, 2, 2, 300
    p = X.xcorr_plan(ns, npol, F, T, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0, 512, window=96)
    assert p["tile"] == 512 and p["nwindows"] == 4
    with pytest.raises(Exception):
        X.xcorr_plan(ns, npol, F, T, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0, 512, window=100)
    packed = synth.pack_ci4(synth.voltages_np(synth.SEED_BASE + 68, T, F, ns * npol, ("uniform", -8, 7)))
    c = X.Correlator(ns, npol, F, T, "ci4", "f6", tile=512, window=96)
    import torch

    from tests.gpu_util import device

    out = c.run(torch.from_numpy(packed).to(device()))
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4), "super-f6-forced")
    c.close()


def test_super_stream_accumulates(oracle_mod):
    """A streaming integration planned on super-tiles adds every chunk into the int64
    totals (the accumulating stores of the super-tiled kernel)."""
    import torch

    from paper_1107_4264_amd import xcorr as X
    from tests.gpu_util import device

    device()
    ns, npol, F, chunk, nchunk = 256, 2, 2, 50, 3
    assert X.xcorr_plan(ns, npol, F, chunk, X.IN_CI4, X.ACC_I8_MMA_I32, 0)["tile"] == 512
    v = synth.voltages_np(synth.SEED_BASE + 64, chunk * nchunk, F, ns * npol, ("uniform", -8, 7))
    packed = synth.pack_ci4(v)
    want = oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4)
    st = X.Stream(ns, npol, F, chunk, "ci4", "i8")
    out = st.begin()
    for c in range(nchunk):
        st.push(torch.from_numpy(np.ascontiguousarray(packed[c * chunk:(c + 1) * chunk])).pin_memory())
    assert st.end() == chunk * nchunk
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), want, "super-stream")
    st.close()


def test_super_f6_without_workspace_falls_back(oracle_mod):
    """The stream and batch entry points hold no fp6 workspace: a 4-bit fp6 job that plans
    super-tiles (512 inputs) runs 128-tiles there and still gives the oracle's bits."""
    import torch

    from paper_1107_4264_amd import xcorr as X
    from tests.gpu_util import device

    dev = device()
    ns, npol, F, chunk, nchunk = 256, 2, 2, 40, 2
    assert X.xcorr_plan(ns, npol, F, chunk, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0)["tile"] == 512
    v = synth.voltages_np(synth.SEED_BASE + 69, chunk * nchunk, F, ns * npol, ("uniform", -8, 7))
    packed = synth.pack_ci4(v)
    want = oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4)
    say("super f6 stream fallback")
    st = X.Stream(ns, npol, F, chunk, "ci4", "f6")
    chunks = [torch.from_numpy(np.ascontiguousarray(packed[c * chunk:(c + 1) * chunk])).pin_memory()
              for c in range(nchunk)]
    out = st.begin()
    for c in range(nchunk):
        st.push(chunks[c])
    assert st.end() == chunk * nchunk
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), want, "super-f6-stream")
    st.close()
    say("super f6 batch fallback")
    first = np.ascontiguousarray(packed[:chunk])
    b = X.Batch([(ns, npol, F, chunk), (20, 2, 1, 33)], "ci4", "f6")
    small = synth.pack_ci4(synth.voltages_np(synth.SEED_BASE + 70, 33, 1, 40, ("uniform", -8, 7)))
    outs = b.run([torch.from_numpy(first).to(dev), torch.from_numpy(small).to(dev)])
    torch.cuda.synchronize()
    _check(outs[0].cpu().numpy(), oracle_mod.xcorr(first, ns, npol, fmt=oracle_mod.CI4), "super-f6-batch/0")
    _check(outs[1].cpu().numpy(), oracle_mod.xcorr(small, 20, 2, fmt=oracle_mod.CI4), "super-f6-batch/1")
    b.close()


def test_super_misaligned_input_falls_back(oracle_mod):
    """An input pointer off the 16-byte grid runs 128-tiles (the row copies need aligned
    rows) and still gives the oracle's bits."""
    import torch

    from paper_1107_4264_amd import xcorr as X
    from tests.gpu_util import device

    dev = device()
    ns, npol, F, T = 256, 2, 2, 40
    v = synth.voltages_np(synth.SEED_BASE + 65, T, F, ns * npol, ("uniform", -8, 7))
    packed = synth.pack_ci4(v)
    flat = torch.zeros(packed.size + 16, dtype=torch.uint8, device=dev)
    flat[3:3 + packed.size] = torch.from_numpy(packed.reshape(-1)).to(dev)
    xin = flat[3:3 + packed.size].view(packed.shape)
    assert xin.data_ptr() % 16 == 3
    c = X.Correlator(ns, npol, F, T, "ci4", "i8", tile=512)
    out = c.run(xin)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4), "super-misaligned")
    c.close()


CI8_SHAPES = [(256, 2, 3, 100), (384, 2, 2, 77), (512, 1, 2, 33), (256, 2, 1, 1)]


@pytest.mark.parametrize("shape", CI8_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_super_ci8_matches_oracle(oracle_mod, shape):
    """8-bit samples on super-tiles (int8 path): rows moved into the operand layout."""
    ns, npol, F, T = shape
    x = synth.voltages_np(synth.SEED_BASE + 70 + ns + T, T, F, ns * npol, ("gauss", 40.0, 127))
    say("super ci8", shape)
    got, _ = run_xeng(x, ns, npol, "ci8", "i8", tile=512)
    _check(got, oracle_mod.xcorr(x, ns, npol), f"super-ci8/{shape}")


def test_super_ci8_extreme_and_tiles(oracle_mod):
    """Full-scale 8-bit samples (+-127) on super-tiles equal the oracle and the 128-tiles."""
    ns, npol, F, T = 256, 2, 2, 90
    x = synth.voltages_np(synth.SEED_BASE + 71, T, F, ns * npol, ("uniform", -127, 127))
    x[:, :, :4] = -127
    x[:, :, 500:502] = 127
    a, _ = run_xeng(x, ns, npol, "ci8", "i8", tile=512)
    _check(a, oracle_mod.xcorr(x, ns, npol), "super-ci8-extreme")
    b, _ = run_xeng(x, ns, npol, "ci8", "i8", tile=128)
    assert np.array_equal(a, b)


def test_super_ci8_windows(oracle_mod):
    """Two int32 windows (66572 samples each at the default bound) of 8-bit super-tiles
    summed into the int64 totals, against the oracle (272 inputs)."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F, T = 136, 2, 1, 66572 + 200
    p = X.xcorr_plan(ns, npol, F, T, X.IN_CI8, X.ACC_I8_MMA_I32, 0, 512)
    assert p["nwindows"] == 2 and p["out_dtype"] == X.OUT_CI64
    x = synth.voltages_np(synth.SEED_BASE + 72, T, F, ns * npol, ("uniform", -127, 127))
    say("super ci8 windows", T)
    full, ot = run_xeng(x, ns, npol, "ci8", "i8", tile=512)
    assert ot == X.OUT_CI64
    _check(full, oracle_mod.xcorr(x, ns, npol), "super-ci8-windows")



@pytest.mark.parametrize("fmt_acc", [("ci4", "i8"), ("ci4", "f8"), ("ci4", "f6"), ("ci8", "i8")],
                         ids=lambda t: "-".join(t))
@pytest.mark.parametrize("shape", [(136, 2, 2, 45), (200, 2, 2, 37), (392, 2, 1, 33), (304, 1, 2, 40)],
                         ids=lambda s: "x".join(map(str, s)))
def test_super_ragged(oracle_mod, fmt_acc, shape):
    """Arrays that are not a multiple of 256 inputs (272, 400, 784 and 304 single
    polarisation): the last super-row is partial; its missing inputs read as zeros."""
    fmt, acc = fmt_acc
    ns, npol, F, T = shape
    if fmt == "ci4":
        x = synth.pack_ci4(synth.voltages_np(synth.SEED_BASE + 80 + ns, T, F, ns * npol, ("uniform", -8, 7)))
        want = oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4)
    else:
        x = synth.voltages_np(synth.SEED_BASE + 81 + ns, T, F, ns * npol, ("gauss", 40.0, 127))
        want = oracle_mod.xcorr(x, ns, npol)
    say("super ragged", fmt, acc, shape)
    got, _ = run_xeng(x, ns, npol, fmt, acc, tile=512)
    _check(got, want, f"super-ragged/{fmt}/{acc}/{shape}")
