"""The tuning cache's file format, read without a GPU: tagged lines with the
eleven key fields and a variant in range are entries; anything else is
skipped; a later line for the same key replaces the earlier one."""
import pytest

from paper_2607_20766_amd.engine import (ShapeError, tune_cache_clear, tune_cache_file,
                                         tune_cache_size)

KEY = "gfx950:sramecc+:xnack- 256 1 0 0 512 65536 0 16 4 4"


def test_file_entries_and_junk(tmp_path):
    path = tmp_path / "tune.txt"
    path.write_text("\n".join([
        f"shape-tune-v1 {KEY} 3",
        f"shape-tune-v1 {KEY} 5",                       # same key: replaces
        "shape-tune-v1 gfx950 256 0 0 4096 0 0 0 16 4 4 0",
        "shape-tune-v0 gfx950 256 0 0 4096 0 0 0 16 4 4 1",   # other tag
        "shape-tune-v1 gfx950 256 0 0 4096 0 0 0 16 4 4 8",   # variant out of range
        "shape-tune-v1 gfx950 256 0 0 4096 0 0 0 16",         # too short
        "# a comment",
        "",
    ]) + "\n")
    tune_cache_clear()
    try:
        tune_cache_file(str(path))
        assert tune_cache_size() == 2
        tune_cache_clear()
        assert tune_cache_size() == 0
    finally:
        tune_cache_file(None)


def test_new_file_is_created_and_bad_path_refused(tmp_path):
    path = tmp_path / "new.txt"
    try:
        tune_cache_file(str(path))
        assert path.exists() and path.read_text() == ""
        with pytest.raises(ShapeError):
            tune_cache_file(str(tmp_path / "missing_dir" / "x.txt"))
        with pytest.raises(ShapeError):
            tune_cache_file("")
    finally:
        tune_cache_file(None)
