"""CPU-side checks of the autotuning table (no device needed): its shape
key, its text file, the merge and clear calls, and the file named by
TL_TUNE_CACHE read at the table's first use."""
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = "# tl tuning table v1: bx by mixed set_edge overlap inner_iters nx ny ms\n"


def _tl():
    from paper_1208_4093_amd import tl
    if not Path(tl.LIB_PATH).exists():
        pytest.skip("libtl.so not built")
    tl.load()
    return tl


def _bucket(s):
    import math
    return round(2 * math.log2(s))


def _line(nx, ny, mixed, E, ov, inner, ms=12.5):
    return f"{_bucket(nx)} {_bucket(ny)} {mixed} {E} {ov} {inner} {nx} {ny} {ms}\n"


@pytest.fixture
def tl(tmp_path):
    t = _tl()
    t.tl_tune_clear()
    yield t
    t.tl_tune_clear()


def test_load_lookup_save_round_trip(tl, tmp_path):
    f = tmp_path / "table.txt"
    f.write_text(HEADER + _line(300, 200, 1, 32, 4, 12) + _line(300, 200, 0, 64, 1, 28, 40.0))
    tl.tl_tune_load(str(f))
    e = tl.tl_tune_lookup(300, 200, tl.TL_MIXED)
    assert (e["set_edge"], e["overlap"], e["inner_iters"], e["nx"], e["ny"]) == (32, 4, 12, 300, 200)
    e = tl.tl_tune_lookup(300, 200, tl.TL_FP64)
    assert (e["set_edge"], e["overlap"], e["inner_iters"]) == (64, 1, 28)
    g = tmp_path / "saved.txt"
    tl.tl_tune_save(str(g))
    tl.tl_tune_clear()
    assert tl.tl_tune_lookup(300, 200, tl.TL_MIXED) is None
    tl.tl_tune_load(str(g))
    assert tl.tl_tune_lookup(300, 200, tl.TL_MIXED)["inner_iters"] == 12
    assert g.read_text().startswith("# tl tuning table v1")


def test_shapes_in_the_same_half_octaves_share_an_entry(tl, tmp_path):
    f = tmp_path / "t.txt"
    f.write_text(HEADER + _line(256, 256, 1, 32, 2, 16))
    tl.tl_tune_load(str(f))
    # 2 log2 s rounds to 16 for s in [2^7.75, 2^8.25) = [215.3, 304.4)
    for nx, ny in ((216, 300), (304, 216), (256, 256)):
        assert tl.tl_tune_lookup(nx, ny, tl.TL_MIXED)["set_edge"] == 32
    for nx, ny in ((215, 256), (256, 305), (128, 256)):
        assert tl.tl_tune_lookup(nx, ny, tl.TL_MIXED) is None
    assert tl.tl_tune_lookup(256, 256, tl.TL_FP64) is None   # precision is part of the key


@pytest.mark.parametrize("bad", [
    "16 16 1 32 2 16 256 256\n",             # a field missing
    "16 16 1 24 2 16 256 256 1.0\n",         # unsupported set edge
    "16 16 1 32 3 16 256 256 1.0\n",         # unsupported overlap
    "16 16 1 32 2 0 256 256 1.0\n",          # no sweeps
    "16 16 2 32 2 16 256 256 1.0\n",         # precision flag not 0/1
    "17 16 1 32 2 16 256 256 1.0\n",         # key does not match the lattice it names
    "16 16 1 32 2 16 256 256 1.0 extra\n",   # trailing field
])
def test_malformed_files_are_rejected_whole(tl, tmp_path, bad):
    good = tmp_path / "good.txt"
    good.write_text(HEADER + _line(100, 100, 0, 16, 2, 20))
    tl.tl_tune_load(str(good))
    f = tmp_path / "bad.txt"
    f.write_text(HEADER + _line(512, 512, 1, 32, 2, 16) + bad)
    with pytest.raises(tl.TLError) as ei:
        tl.tl_tune_load(str(f))
    assert ei.value.status == tl.TL_E_INVAL
    assert tl.tl_tune_lookup(512, 512, tl.TL_MIXED) is None      # nothing of it merged
    assert tl.tl_tune_lookup(100, 100, tl.TL_FP64)["inner_iters"] == 20
    with pytest.raises(tl.TLError):
        tl.tl_tune_load(str(tmp_path / "missing.txt"))


def test_cache_file_is_read_at_first_use(tmp_path):
    _tl()
    f = tmp_path / "cache.txt"
    f.write_text(HEADER + _line(640, 480, 1, 64, 4, 20))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1208_4093_amd import tl\n"
            "e = tl.tl_tune_lookup(640, 480, tl.TL_MIXED)\n"
            "print(e['set_edge'], e['overlap'], e['inner_iters'])\n") % str(ROOT)
    env = dict(os.environ, TL_TUNE_CACHE=str(f))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["64", "4", "20"]
