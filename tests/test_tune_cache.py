"""The autotuner's table leaves and re-enters a process as plain records
(gc_autotune_export / gc_autotune_import, and the JSON file the Python
layer keeps them in).  Neither call touches the GPU."""
import ctypes
import json
import math

import pytest

import paper_1911_13074_amd as gc
from paper_1911_13074_amd import abi

F = abi.GC_TUNE_FAMILIES


def record(dtype=0, op=0, geodesic=1, lw=10, lh=10, best=2, k=None, rate=None):
    return {"dtype": dtype, "op": op, "geodesic": geodesic, "log2_width": lw, "log2_height": lh,
            "best_tile": best, "k": k if k is not None else [20, 16, 20, 16, 16],
            "rate": rate if rate is not None else [2.0e12, 1.0e12, 2.5e12, 1.5e12, 1.2e12]}


def write(path, records, **over):
    doc = {"format": "geochain-autotune", "version": 1, "families": F, "records": records}
    doc.update(over)
    path.write_text(json.dumps(doc))
    return path


@pytest.fixture(autouse=True)
def empty_table():
    gc.autotune_clear()
    yield
    gc.autotune_clear()


def test_round_trip_through_a_file(tmp_path):
    recs = [record(), record(dtype=1, op=1, geodesic=0, lw=7, lh=11, best=0)]
    gc.autotune_load(write(tmp_path / "a.json", recs))
    got = gc.autotune_records()
    key = lambda r: (r["dtype"], r["op"], r["geodesic"], r["log2_width"], r["log2_height"])
    assert sorted(got, key=key) == sorted(recs, key=key)
    gc.autotune_save(tmp_path / "b.json")
    gc.autotune_clear()
    assert gc.autotune_records() == []
    gc.autotune_load(tmp_path / "b.json")
    assert sorted(gc.autotune_records(), key=key) == sorted(recs, key=key)


def test_a_record_replaces_its_size_class(tmp_path):
    gc.autotune_load(write(tmp_path / "a.json", [record()]))
    gc.autotune_load(write(tmp_path / "b.json", [record(best=0, k=[24, 16, 20, 16, 16])]))
    got = gc.autotune_records()
    assert len(got) == 1 and got[0]["best_tile"] == 0 and got[0]["k"][0] == 24


@pytest.mark.parametrize("bad", [
    {"dtype": 3}, {"op": 2}, {"geodesic": 2}, {"log2_width": 15}, {"log2_height": -1}, {"best_tile": F},
    {"k": [64, 16, 20, 16, 16]}, {"k": [20, 16, 0, 16, 16]},            # chosen family without steps
    {"rate": [math.nan, 1.0, 1.0, 1.0, 1.0]}, {"rate": [-1.0, 1.0, 1.0, 1.0, 1.0]},
    {"rate": [math.inf, 1.0, 1.0, 1.0, 1.0]},
])
def test_a_bad_record_leaves_the_table_unchanged(tmp_path, bad):
    gc.autotune_load(write(tmp_path / "a.json", [record(lw=5)]))
    before = gc.autotune_records()
    rec = record()
    rec.update(bad)
    with pytest.raises(abi.GeochainError) as e:
        gc.autotune_load(write(tmp_path / "b.json", [record(lw=6), rec]))
    assert e.value.status == abi.GC_ERR_INVALID_ARG
    assert "record 1" in str(e.value)
    assert gc.autotune_records() == before


@pytest.mark.parametrize("over,match", [({"format": "other"}, "not an autotune file"),
                                        ({"version": 2}, "not an autotune file"),
                                        ({"families": F + 1}, "tile families")])
def test_files_of_another_shape_are_refused(tmp_path, over, match):
    with pytest.raises(ValueError, match=match):
        gc.autotune_load(write(tmp_path / "a.json", [record()], **over))
    broken = record()
    del broken["k"]
    with pytest.raises(ValueError, match="record 0"):
        gc.autotune_load(write(tmp_path / "b.json", [broken]))
    short = record(rate=[1.0, 2.0])
    with pytest.raises(ValueError, match="record 0"):
        gc.autotune_load(write(tmp_path / "c.json", [short]))
    assert gc.autotune_records() == []


def test_abi_argument_checks():
    count = ctypes.c_int32(-1)
    assert abi.gc_autotune_export(None, 0, ctypes.byref(count)) == abi.GC_OK and count.value == 0
    assert abi.gc_autotune_export(None, 0, None) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_autotune_export(None, -1, ctypes.byref(count)) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_autotune_export(None, 1, ctypes.byref(count)) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_autotune_import(None, -1) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_autotune_import(None, 1) == abi.GC_ERR_INVALID_ARG
    assert abi.gc_autotune_import(None, 0) == abi.GC_OK
    # a short buffer gets the first records and the full count
    entries = (abi.gc_tune_entry * 3)()
    for i in range(3):
        entries[i].dtype, entries[i].op, entries[i].geodesic = 0, 0, 1
        entries[i].log2_width, entries[i].log2_height, entries[i].best_tile = 4 + i, 4, 2
        entries[i].k[2] = 20
        entries[i].rate[2] = 1.0e12
    assert abi.gc_autotune_import(entries, 3) == abi.GC_OK
    out = (abi.gc_tune_entry * 2)()
    assert abi.gc_autotune_export(out, 2, ctypes.byref(count)) == abi.GC_OK
    assert count.value == 3 and [out[i].log2_width for i in range(2)] == [4, 5]
