"""The GEMM tile table of the autotuner on the host (no GPU): text save and
load, merging, rejection of malformed files."""
import os

import pytest

from paper_1912_13403_amd import hsdm


@pytest.fixture
def lib():
    lib = hsdm.load_library()
    lib.hsdm_tune_clear()
    yield lib
    lib.hsdm_tune_clear()


def test_load_save_roundtrip(lib, tmp_path):
    src = tmp_path / "tiles.txt"
    src.write_text("hsdm-gemm-tiles 1\n80e30b1ad 0\n80e30b1ae 2\n")
    assert lib.hsdm_tune_load(str(src).encode()) == 2
    assert lib.hsdm_tune_entries() == 2
    out = tmp_path / "out.txt"
    assert lib.hsdm_tune_save(str(out).encode()) == hsdm.HSDM_OK
    lines = out.read_text().split("\n")
    assert lines[0] == "hsdm-gemm-tiles 1"
    assert sorted(l for l in lines[1:] if l) == ["80e30b1ad 0", "80e30b1ae 2"]
    # merging: a later file overrides a class and adds others
    more = tmp_path / "more.txt"
    more.write_text("hsdm-gemm-tiles 1\n80e30b1ae 1\n10 2\n")
    assert lib.hsdm_tune_load(str(more).encode()) == 2
    assert lib.hsdm_tune_entries() == 3
    assert lib.hsdm_tune_save(str(out).encode()) == hsdm.HSDM_OK
    assert "80e30b1ae 1" in out.read_text()


@pytest.mark.parametrize("text", ["", "something else 1\n", "hsdm-gemm-tiles 2\n",
                                  "hsdm-gemm-tiles 1\n10 7\n", "hsdm-gemm-tiles 1\n10 x\n"])
def test_malformed_files_merge_nothing(lib, tmp_path, text):
    f = tmp_path / "bad.txt"
    f.write_text(text)
    assert lib.hsdm_tune_load(str(f).encode()) == -3
    assert lib.hsdm_tune_entries() == 0


def test_missing_file_and_path(lib, tmp_path):
    assert lib.hsdm_tune_load(str(tmp_path / "none.txt").encode()) == -2
    assert lib.hsdm_tune_load(None) == -1
    assert lib.hsdm_tune_save(None) == -1
    assert lib.hsdm_tune_save(os.path.join(str(tmp_path), "no", "dir.txt").encode()) == \
        hsdm.HSDM_DEVICE_ERROR
