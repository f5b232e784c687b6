"""The package's tuned launch parameters per workload class (no GPU): class
keys, lookups with their fallbacks, the stored table, and that the library
accepts every stored setting."""

import json

import pytest

from workloads import workload


def test_class_keys():
    from paper_1202_2355_amd import tuning
    assert tuning.class_key("single", "f32", workload(2).layout, 1_000_000) == "single:f32:gh:6"
    assert tuning.class_key("single", "f32", workload(3).layout, 8_000_000) == "single:f32:losvd:7"
    assert tuning.class_key("batch", "f32", workload(2).layout) == "batch:f32:gh"
    alm = dict(workload(2).layout, dens="alm")
    assert tuning.class_key("single", "f32", alm, 10 ** 6) == "single:f32:gh+alm:6"


def test_lookup_falls_back_to_nearest_size_then_defaults():
    from paper_1202_2355_amd import tuning
    table = {"single:f32:gh:6": {"params": {"block": 512, "tiles_per_cu": 2}}}
    lay = workload(2).layout
    assert tuning.lookup("single", "f32", lay, 10 ** 6, table)["block"] == 512
    assert tuning.lookup("single", "f32", lay, 10 ** 4, table)["tiles_per_cu"] == 2
    assert tuning.lookup("single", "f32", workload(3).layout, 10 ** 6, table) == tuning.DEFAULT
    assert tuning.lookup("single", "f64", lay, 10 ** 6, {})["block"] == 256


def test_record_round_trip(tmp_path):
    from paper_1202_2355_amd import tuning
    path = str(tmp_path / "t.json")
    p = dict(tuning.DEFAULT, block=256, tiles_per_cu=8)
    tuning.record("batch:f32:gh", p, 450.0, "test", path=path)
    assert tuning.load(path)["batch:f32:gh"]["params"] == p
    assert json.load(open(path))["classes"]["batch:f32:gh"]["us_per_step"] == 450.0


def test_stored_table_is_accepted_by_the_library():
    from paper_1202_2355_amd import tuning
    table = tuning.load()
    assert "batch:f32:gh" in table and "single:f32:gh:6" in table
    before = tuning.current()
    try:
        for key, e in table.items():
            tuning.apply(dict(tuning.DEFAULT, **e["params"]))
            assert tuning.current() == dict(tuning.DEFAULT, **e["params"]), key
    finally:
        tuning.apply(before)
    assert tuning.current() == before


def test_library_refuses_bad_settings():
    from paper_1202_2355_amd import _abi
    for bad in (3, 16, -1):
        with pytest.raises(_abi.M2MError):
            _abi.m2m_set_private_copies(bad)
    for bad in (0, 3):
        with pytest.raises(_abi.M2MError):
            _abi.m2m_set_batch_groups(bad)
    for bad in (-2, 2):
        with pytest.raises(_abi.M2MError):
            _abi.m2m_set_interleave(bad)
    assert _abi.m2m_get_interleave() == -1   # the default: by state size
    for mode in (0, 1, -1):
        _abi.m2m_set_interleave(mode)
        assert _abi.m2m_get_interleave() == mode
