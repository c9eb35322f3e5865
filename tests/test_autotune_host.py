"""Host-side checks of the tuned-shape table (no GPU needed)."""
import json

import pytest

from paper_2311_18715_amd import autotune as T


def test_buckets():
    assert T.n_bucket(160000) == 17          # log2 = 17.29
    assert T.n_bucket(1 << 20) == 20
    assert T.n_bucket(10000) == 13           # log2 = 13.29
    assert T.n_bucket(12000) == 14           # log2 = 13.55
    assert T.r_bucket(1) == 16 and T.r_bucket(16) == 16 and T.r_bucket(17) == 32
    assert T.r_bucket(40) == 48 and T.r_bucket(64) == 64
    with pytest.raises(ValueError):
        T.r_bucket(65)
    with pytest.raises(ValueError):
        T.n_bucket(0)
    with pytest.raises(ValueError):
        T.key("gfx950", "f32", "f32", 16, 100, "fastest")


def test_lookup_and_round_trip(tmp_path):
    path = str(tmp_path / "shapes.json")
    k = T.key("gfx950", "f32", "f32", 40, 160000, "throughput")
    assert k == "gfx950/f32/f32/r48/n2^17/throughput"
    shapes = {
        k: {"shape": [256, 1024, 512], "us_best": 1.0, "us_default": 1.2, "streams": 16},
        T.key("gfx950", "f64", "f64", 8, 4096, "latency"): {"shape": [384, 256, 256]},   # invalid
        T.key("gfx950", "f64", "f64", 8, 8192, "latency"): {"shape": [512, 24, 256]},    # invalid
    }
    T.save_table(shapes, path, meta={"note": "test"})
    table = T.load_table(path)
    assert json.load(open(path))["meta"] == {"note": "test"}
    # any n and r_max of the bucket find the entry; a BF16 basis defaults to FP32 snapshots
    assert T.lookup(150000, 33, "f32", objective="throughput", table=table, arch="gfx950") == \
        (256, 1024, 512)
    assert T.lookup(150000, 33, "f32", objective="latency", table=table, arch="gfx950") is None
    assert T.lookup(150000, 33, "bf16", objective="throughput", table=table, arch="gfx950") is None
    assert T.lookup(150000, 33, "f32", objective="throughput", table=table, arch="gfx942") is None
    assert T.lookup(4096, 8, "f64", table=table, arch="gfx950") is None
    assert T.lookup(8192, 8, "f64", table=table, arch="gfx950") is None
    assert T.load_table(str(tmp_path / "missing.json")) == {}


def test_shipped_table_is_valid():
    table = T.load_table(T.TABLE_PATH)
    for k, entry in table.items():
        arch, basis, io, r, n, objective = k.split("/")
        assert basis in ("f64", "f32", "bf16") and io in ("f64", "f32")
        assert r.startswith("r") and n.startswith("n2^") and objective in T.OBJECTIVES
        assert T._valid(entry), k
        assert entry["us_best"] <= entry["us_default"], k


def test_bucket_ranges_parse():
    assert T._parse_range("13-16") == [13, 14, 15, 16]
    assert T._parse_range("16,32,48,64") == [16, 32, 48, 64]
    assert T._parse_range("13-14,21") == [13, 14, 21]


def test_invalid_entries_are_ignored(tmp_path):
    path = str(tmp_path / "shapes.json")
    k = T.key("gfx950", "f64", "f64", 40, 160000, "latency")
    T.save_table({k: {"shape": [512, 256]}}, path)            # too short
    assert T.lookup(160000, 40, "f64", table=T.load_table(path), arch="gfx950") is None
    T.save_table({k: {"us_best": 1.0}}, path)                 # no shape
    assert T.lookup(160000, 40, "f64", table=T.load_table(path), arch="gfx950") is None
    T.save_table({k: {"shape": [512, 256, 256]}}, path)
    assert T.lookup(160000, 40, "f64", table=T.load_table(path), arch="gfx950") == (512, 256, 256)
