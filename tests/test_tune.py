"""The autotuner's cache file round-trips through the library (host only)."""
import os

import pytest


def test_tune_cache_round_trip(tmp_path):
    from paper_1608_04329_amd import hsp
    path = str(tmp_path / "tune.txt")
    assert hsp.hsp_tune_cache_get(path, "a") is None  # no file yet
    hsp.hsp_tune_cache_put(path, "sweep-v1 gfx950 cus=256 xt=0 N=1000 p=10", "gp=1 pct=40 unit=8")
    hsp.hsp_tune_cache_put(path, "batch-v1 gfx950 cus=256 h=00ff", "mc_gz=256 bw=100")
    assert hsp.hsp_tune_cache_get(path, "sweep-v1 gfx950 cus=256 xt=0 N=1000 p=10") == "gp=1 pct=40 unit=8"
    assert hsp.hsp_tune_cache_get(path, "batch-v1 gfx950 cus=256 h=00ff") == "mc_gz=256 bw=100"
    # a new value replaces the old one; other entries stay
    hsp.hsp_tune_cache_put(path, "sweep-v1 gfx950 cus=256 xt=0 N=1000 p=10", "gp=1 pct=0 unit=16 ms=0.1")
    assert hsp.hsp_tune_cache_get(path, "sweep-v1 gfx950 cus=256 xt=0 N=1000 p=10") == "gp=1 pct=0 unit=16 ms=0.1"
    assert hsp.hsp_tune_cache_get(path, "batch-v1 gfx950 cus=256 h=00ff") == "mc_gz=256 bw=100"
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and all("\t" in l for l in lines)
    # a prefix of a key is another key
    assert hsp.hsp_tune_cache_get(path, "sweep-v1 gfx950") is None
    assert not [f for f in os.listdir(tmp_path) if ".tmp" in f]  # no temporary files left


def test_tune_cache_keeps_foreign_lines_and_rejects_bad_entries(tmp_path):
    from paper_1608_04329_amd import hsp
    path = str(tmp_path / "tune.txt")
    with open(path, "w") as f:
        f.write("# written by hand\nnot an entry\nk1\tv1\n")
    hsp.hsp_tune_cache_put(path, "k2", "v2")
    text = open(path).read()
    assert "# written by hand" in text and "not an entry" in text
    assert hsp.hsp_tune_cache_get(path, "k1") == "v1" and hsp.hsp_tune_cache_get(path, "k2") == "v2"
    for key, value in [("a\tb", "v"), ("a\nb", "v"), ("", "v"), ("k", "v\nw")]:
        with pytest.raises(hsp.HspError) as e:
            hsp.hsp_tune_cache_put(path, key, value)
        assert e.value.code == hsp.HSP_EINVAL
    assert hsp.hsp_tune_cache_get(path, "k1") == "v1"


def test_tune_cache_unwritable_path(tmp_path):
    from paper_1608_04329_amd import hsp
    with pytest.raises(hsp.HspError):
        hsp.hsp_tune_cache_put(str(tmp_path / "no_such_dir" / "tune.txt"), "k", "v")
