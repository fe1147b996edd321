"""Host-side pieces of the FFT autotuner: cache keys and the JSON cache file.
No device is needed: these entry points only read and write files."""

import json

import numpy as np
import pytest

from paper_1210_2687_amd import admm as A
from paper_1210_2687_amd import workloads as WL


def _tv(H, W, k=5):
    return A.make_problem(WL.kernel_uniform(k), np.ones((H, W), np.uint8), 1e-3)


def _fa(H, W, J):
    return A.make_problem(WL.kernel_uniform(3), np.ones((H, W), np.uint8), 1e-3, reg=A.ADMM_REG_FRAME, levels=J)


def test_key_of_uniform_batch():
    assert A.admm_tune_key([_tv(512, 512)] * 8, "gfx950") == "gfx950|tv512x512*8"


def test_key_is_order_independent_and_counts_shapes():
    a = [_tv(64, 96), _fa(128, 128, 3), _tv(64, 96), _tv(32, 32)]
    b = [a[3], a[1], a[0], a[2]]
    k = A.admm_tune_key(a, "gfx950")
    assert k == A.admm_tune_key(b, "gfx950")
    assert k == "gfx950|fa128x128j3*1,tv32x32*1,tv64x96*2"


def test_key_of_long_ragged_batch_is_a_hash():
    probs = [_tv(8 * (i % 40 + 1), 8 * (i % 37 + 1)) for i in range(120)]
    k = A.admm_tune_key(probs, "gfx950")
    assert k.startswith("gfx950|h") and k.endswith("*120") and len(k) < 64
    assert k == A.admm_tune_key(list(reversed(probs)), "gfx950")
    assert k != A.admm_tune_key(probs[:-1], "gfx950")


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert A.admm_tune_cache_lookup(path, "gfx950|tv8x8*1") is None   # no file yet
    A.admm_tune_cache_store(path, "gfx950|tv512x512*8", 4, 8, 16.1, 30.6)
    A.admm_tune_cache_store(path, "gfx950|tv64x64*2", 2, 3)
    assert A.admm_tune_cache_lookup(path, "gfx950|tv512x512*8") == (4, 8)
    assert A.admm_tune_cache_lookup(path, "gfx950|tv64x64*2") == (2, 3)
    assert A.admm_tune_cache_lookup(path, "gfx950|tv1x1*1") is None
    A.admm_tune_cache_store(path, "gfx950|tv512x512*8", 3, 6)          # replace
    assert A.admm_tune_cache_lookup(path, "gfx950|tv512x512*8") == (3, 6)
    data = json.load(open(path))                                       # plain JSON
    assert data["gfx950|tv64x64*2"] == {"tc": 2, "rows": 3, "col_us": 0.0, "row_us": 0.0}
    assert set(data) == {"gfx950|tv512x512*8", "gfx950|tv64x64*2"}


def test_cache_written_by_hand_is_read(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"gfx950|tv96x96*1": {"rows": 5, "tc": 1}}, indent=3))
    assert A.admm_tune_cache_lookup(str(path), "gfx950|tv96x96*1") == (1, 5)
    path.write_text("{}")
    assert A.admm_tune_cache_lookup(str(path), "gfx950|tv96x96*1") is None


@pytest.mark.parametrize("text", ["", "[]", "{\"k\": 3}", "{\"k\": {\"tc\": }}", "{\"k\": {\"tc\": 1}"])
def test_malformed_cache_is_an_error(tmp_path, text):
    path = tmp_path / "tune.json"
    path.write_text(text)
    with pytest.raises(A.AdmmError):
        A.admm_tune_cache_lookup(str(path), "k")
    with pytest.raises(A.AdmmError):
        A.admm_tune_cache_store(str(path), "k", 1, 1)
    assert path.read_text() == text                                     # left untouched


@pytest.mark.parametrize("key,tc,rows", [("a\"b", 1, 1), ("ok", 0, 1), ("ok", 1, 0)])
def test_store_rejects_bad_entries(tmp_path, key, tc, rows):
    with pytest.raises(A.AdmmError):
        A.admm_tune_cache_store(str(tmp_path / "t.json"), key, tc, rows)


def test_per_class_row_counts_survive_other_writes(tmp_path):
    # the autotuner may record row counts per size class of the row length
    # ("rows_512", "rows_1024", ..., "rows_8192"); lookup reports the common
    # (tc, rows), and rewriting the file for another key keeps those fields
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"gfx950|h0123456789abcdef*256": {"tc": 4, "rows": 5, "rows_512": 8,
                                                                 "col_us": 896.0, "row_us": 1597.0}}))
    assert A.admm_tune_cache_lookup(str(path), "gfx950|h0123456789abcdef*256") == (4, 5)
    A.admm_tune_cache_store(str(path), "gfx950|tv64x64*1", 1, 2)
    data = json.load(open(path))
    assert data["gfx950|h0123456789abcdef*256"]["rows_512"] == 8
    assert "rows_1024" not in data["gfx950|h0123456789abcdef*256"]
    assert data["gfx950|tv64x64*1"] == {"tc": 1, "rows": 2, "col_us": 0.0, "row_us": 0.0}
