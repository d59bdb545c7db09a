"""Host-side tuning cache: file round trip, lookup by job shape (with the default bound
resolved as planning resolves it), rejection of malformed files."""

from __future__ import annotations

import pytest

from paper_1107_4264_amd import xcorr as X


@pytest.fixture(autouse=True)
def clean_cache():
    X.xcorr_autotune_clear()
    yield
    X.xcorr_autotune_clear()


def test_load_lookup_save_roundtrip(tmp_path):
    src = tmp_path / "tuned.jsonl"
    src.write_text(
        '{"nstation": 128, "npol": 2, "nchan": 1024, "ntime": 1000, "in": 0, "acc": 2, "max_abs": 18, "tile": 128, "us": 301.5}\n'
        "\n"
        '{"nstation": 512, "npol": 2, "nchan": 256, "ntime": 4096, "in": 1, "acc": 1, "max_abs": 8, "tile": 64, "us": 3000.0}\n')
    assert X.xcorr_autotune_load(str(src)) == 2
    assert X.xcorr_autotune_lookup(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18) == 128
    # the 4-bit default bound is 8: a lookup with max_abs 0 resolves to it
    assert X.xcorr_autotune_lookup(512, 2, 256, 4096, X.IN_CI4, X.ACC_I8_MMA_I32, 0) == 64
    # other shapes, bounds or paths are not cached
    assert X.xcorr_autotune_lookup(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 17) == 0
    assert X.xcorr_autotune_lookup(128, 2, 1024, 1000, X.IN_CI8, X.ACC_I8_MMA_I32, 18) == 0
    out = tmp_path / "saved.jsonl"
    assert X.xcorr_autotune_save(str(out)) == 2
    X.xcorr_autotune_clear()
    assert X.xcorr_autotune_lookup(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18) == 0
    assert X.xcorr_autotune_load(str(out)) == 2
    assert X.xcorr_autotune_lookup(512, 2, 256, 4096, X.IN_CI4, X.ACC_I8_MMA_I32, 8) == 64


@pytest.mark.parametrize("text", [
    '{"nstation": 1, "npol": 2}\n',
    '{"nstation": 128, "npol": 2, "nchan": 4, "ntime": 10, "in": 0, "acc": 2, "max_abs": 18, "tile": 96, "us": 1.0}\n',
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
