"""The autotuner's persistent cost cache (host only): entries keyed by GPU
architecture, encoding of p (FP4 codes for p <= 8, centred int8 otherwise) and
shape bucket round-trip through the JSON file, lookups fall back to the nearest
bucket of the same architecture and encoding, and malformed files or costs are
refused.  The calibration that fills the cache runs on the GPU
(test_gpu_batched.py)."""
import json

import pytest

from paper_0803_1975_amd import qmm

COSTS_A = [2.5, 1.0, 2.25, 1.125, 2.0, 1.0625, 3.5, 2.75]
COSTS_B = [1.0, 1.0, 4.0, 1.5, 4.0, 1.5, 9.0, 3.0]
COSTS_C = [0.0, 0.5, 0.1, 0.6, 0.1, 0.7, 0.2, 2.0]


@pytest.fixture(autouse=True)
def empty_cache():
    qmm.tune_cache_clear()
    yield
    qmm.tune_cache_clear()


def test_put_get_by_architecture_encoding_and_bucket():
    qmm.tune_cache_put("gfx950", 7, 256, 256, COSTS_A)     # fp4, le512
    qmm.tune_cache_put("gfx950", 101, 256, 256, COSTS_B)   # int8, le512
    qmm.tune_cache_put("gfx950", 101, 64, 100, COSTS_C)    # int8, le128
    assert qmm.tune_cache_get("gfx950", 3, 300, 500) == COSTS_A       # any p <= 8, same bucket
    assert qmm.tune_cache_get("gfx950", 13, 400, 129) == COSTS_B
    assert qmm.tune_cache_get("gfx950", 251, 128, 1) == COSTS_C
    assert qmm.tune_cache_get("gfx950", 101, 4096, 16) == COSTS_B     # gt512: nearest is le512
    assert qmm.tune_cache_get("gfx950", 2, 16, 16) == COSTS_A         # only fp4 entry
    assert qmm.tune_cache_get("gfx942", 7, 256, 256) is None          # other architecture
    qmm.tune_cache_put("gfx950", 5, 500, 500, COSTS_C)                # replaces (fp4, le512)
    assert qmm.tune_cache_get("gfx950", 7, 256, 256) == COSTS_C


def test_file_round_trip_and_merge(tmp_path):
    path = str(tmp_path / "tune.json")
    qmm.tune_cache_put("gfx950", 7, 256, 256, COSTS_A)
    qmm.tune_cache_put("gfx950", 31, 1024, 8, COSTS_B)
    qmm.tune_cache_save(path)
    doc = json.load(open(path))
    assert doc["version"] == 1 and len(doc["entries"]) == 2
    keys = {(e["arch"], e["enc"], e["bucket"]) for e in doc["entries"]}
    assert keys == {("gfx950", "fp4", "le512"), ("gfx950", "int8", "gt512")}
    for e in doc["entries"]:
        assert e["costs"] == (COSTS_A if e["enc"] == "fp4" else COSTS_B)   # exact: %.17g
    qmm.tune_cache_clear()
    assert qmm.tune_cache_get("gfx950", 7, 256, 256) is None
    qmm.tune_cache_put("gfx950", 101, 64, 64, COSTS_C)                # kept by the merge
    qmm.tune_cache_load(path)
    assert qmm.tune_cache_get("gfx950", 7, 256, 256) == COSTS_A
    assert qmm.tune_cache_get("gfx950", 31, 2048, 2048) == COSTS_B
    assert qmm.tune_cache_get("gfx950", 31, 64, 64) == COSTS_C


@pytest.mark.parametrize("text", [
    "", "[]", "{", '{"version": 2, "entries": []}', '{"version": 1}',
    '{"version": 1, "entries": [{"arch": "gfx950", "enc": "fp8", "bucket": "le128", "costs": [1,1,1,1,1,1,1,1]}]}',
    '{"version": 1, "entries": [{"arch": "gfx950", "enc": "fp4", "bucket": "le64", "costs": [1,1,1,1,1,1,1,1]}]}',
    '{"version": 1, "entries": [{"arch": "gfx950", "enc": "fp4", "bucket": "le128", "costs": [1,1,1]}]}',
    '{"version": 1, "entries": [{"arch": "gfx950", "enc": "fp4", "bucket": "le128", "costs": [1,0,1,1,1,1,1,1]}]}',
    '{"version": 1, "entries": [{"arch": "gfx950", "enc": "fp4", "bucket": "le128", "costs": [1,1,1,1,1,1,1,"x"]}]}',
])
def test_malformed_files_are_refused_and_change_nothing(tmp_path, text):
    path = tmp_path / "bad.json"
    path.write_text(text)
    qmm.tune_cache_put("gfx950", 7, 256, 256, COSTS_A)
    with pytest.raises(qmm.QmmError) as e:
        qmm.tune_cache_load(str(path))
    assert e.value.status == qmm.EINVAL
    assert qmm.tune_cache_get("gfx950", 7, 256, 256) == COSTS_A


def test_missing_file_and_bad_keys_are_refused(tmp_path):
    with pytest.raises(qmm.QmmError):
        qmm.tune_cache_load(str(tmp_path / "absent.json"))
    with pytest.raises(qmm.QmmError):
        qmm.tune_cache_put("", 7, 256, 256, COSTS_A)
    with pytest.raises(qmm.QmmError):
        qmm.tune_cache_put("gfx950", 1, 256, 256, COSTS_A)
    with pytest.raises(qmm.QmmError):
        qmm.tune_cache_put("gfx950", 7, 256, 256, [1.0, -1.0] * 4)
    with pytest.raises(qmm.QmmError):
        qmm.tune_cache_put("gfx950", 7, 256, 256, [1.0, float("nan")] * 4)


def test_tune_checks_arguments_before_device_work():
    assert qmm.batched_tune_workspace_size(256, 256) >= 256 * 1024 * 2 + 256 * 256 * 16
    with pytest.raises(qmm.QmmError):
        qmm.batched_tune_workspace_size(0, 256)
    L = qmm.lib()
    import ctypes
    out = (ctypes.c_double * qmm.N_BATCH_COSTS)()
    assert L.qmm_batched_tune(1, 256, 256, None, 0, None, out) == qmm.EINVAL
    assert L.qmm_batched_tune(7, 256, 5000, None, 0, None, out) == qmm.EINVAL
    assert L.qmm_batched_tune(7, 256, 256, None, 0, None, out) == qmm.ENOSPACE
