"""Host-side tuning cache: file round trip, lookup by (architecture, job class) with the
default bound resolved as planning resolves it and channel / sample counts bucketed by
powers of two, rejection of malformed files."""

from __future__ import annotations

import pytest

from paper_1107_4264_amd import xcorr as X


@pytest.fixture(autouse=True)
def clean_cache():
    X.xcorr_autotune_clear()
    yield
    X.xcorr_autotune_clear()


LINE = ('{{"arch": "{arch}", "nstation": {ns}, "npol": 2, "nchan_log2": {fc}, "ntime_log2": {tc}, "in": {fmt}, '
        '"acc": {acc}, "max_abs": {ma}, "window": 0, "tile": {tile}, "staging": {st}, "variant": {var}, '
        '"us": {us}}}\n')


def test_load_lookup_save_roundtrip(tmp_path):
    src = tmp_path / "tuned.jsonl"
    src.write_text(
        LINE.format(arch="gfx950", ns=128, fc=10, tc=10, fmt=0, acc=2, ma=18, tile=256, st=0, var=2, us=250.5)
        + "\n"
        + LINE.format(arch="gfx950", ns=512, fc=8, tc=12, fmt=1, acc=1, ma=8, tile=128, st=1, var=0, us=3000.0)
        + LINE.format(arch="gfx942", ns=128, fc=10, tc=10, fmt=0, acc=2, ma=18, tile=128, st=0, var=0, us=400.0))
    assert X.xcorr_autotune_load(str(src)) == 3
    look = X.xcorr_autotune_lookup
    assert look(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18, arch="gfx950", full=True) == (256, 0, 2)
    # the class buckets channels and samples by powers of two: 513..1024 channels, 513..1024 samples
    assert look(128, 2, 600, 513, X.IN_CI8, X.ACC_F16_MMA_F32, 18, arch="gfx950") == 256
    assert look(128, 2, 1025, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18, arch="gfx950") == 0
    # the entry of another architecture is kept apart
    assert look(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18, arch="gfx942") == 128
    assert look(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18, arch="gfx90a") == 0
    # the 4-bit default bound is 8: a lookup with max_abs 0 resolves to it
    assert look(512, 2, 256, 4096, X.IN_CI4, X.ACC_I8_MMA_I32, 0, arch="gfx950", full=True) == (128, 1, 0)
    # other bounds or paths are not cached
    assert look(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 17, arch="gfx950") == 0
    assert look(128, 2, 1024, 1000, X.IN_CI8, X.ACC_I8_MMA_I32, 18, arch="gfx950") == 0
    out = tmp_path / "saved.jsonl"
    assert X.xcorr_autotune_save(str(out)) == 3
    assert '"arch": "gfx942"' in out.read_text()
    X.xcorr_autotune_clear()
    assert look(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18, arch="gfx950") == 0
    assert X.xcorr_autotune_load(str(out)) == 3
    assert look(512, 2, 256, 4096, X.IN_CI4, X.ACC_I8_MMA_I32, 8, arch="gfx950", full=True) == (128, 1, 0)


@pytest.mark.parametrize("text", [
    '{"nstation": 1, "npol": 2}\n',
    # tile 96 does not exist
    LINE.format(arch="gfx950", ns=128, fc=2, tc=4, fmt=0, acc=2, ma=18, tile=96, st=0, var=0, us=1.0),
    # staging through the caches only on 64 / 128 tiles
    LINE.format(arch="gfx950", ns=128, fc=2, tc=4, fmt=0, acc=2, ma=18, tile=256, st=1, var=0, us=1.0),
    # super-tiles have four variants
    LINE.format(arch="gfx950", ns=512, fc=2, tc=4, fmt=1, acc=1, ma=8, tile=512, st=0, var=4, us=1.0),
    # the old format without an architecture
    '{"nstation": 128, "npol": 2, "nchan": 4, "ntime": 10, "in": 0, "acc": 2, "max_abs": 18, "tile": 128, "us": 1.0}\n',
    "not json\n",
])
def test_load_rejects_malformed(tmp_path, text):
    bad = tmp_path / "bad.jsonl"
    bad.write_text(text)
    with pytest.raises(X.XcorrError) as ei:
        X.xcorr_autotune_load(str(bad))
    assert ei.value.code == X.ERR_INVALID_ARG
    assert "bad entry" in X.last_error()


def test_missing_file():
    with pytest.raises(X.XcorrError):
        X.xcorr_autotune_load("/nonexistent/dir/tuned.jsonl")
