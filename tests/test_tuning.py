"""Launch-shape cache of the autotuner: keys and the JSON file (host only)."""
import json

import pytest

from paper_1512_02818_amd import tuning as T


def test_key_round_trip():
    k = T.key("gfx950", "fp32", 2, False)
    assert k == "gfx950/fp32/D2/plain"
    assert T.parse_key(k) == ("gfx950", "fp32", 2, False, False)
    assert T.parse_key(T.key("gfx950", "fp64", 3, True)) == ("gfx950", "fp64", 3, True, False)
    g = T.key("gfx950", "fp32", 3, True, generic=True)
    assert g == "gfx950/fp32/D3/correction/generic"
    assert T.parse_key(g) == ("gfx950", "fp32", 3, True, True)
    ito = T.key("gfx950", "fp64", 2, 2, generic=True)
    assert ito == "gfx950/fp64/D2/ito/generic"
    assert T.parse_key(ito) == ("gfx950", "fp64", 2, 2, True)
    for bad in ("gfx950/fp16/D2/plain", "gfx950/fp32/2/plain", "gfx950/fp32/D2/cv", "x",
                "gfx950/fp32/D2/plain/special", "gfx950/fp32/D2/plain/generic/x",
                "gfx950/fp32/D2/Ito"):
        with pytest.raises(ValueError):
            T.parse_key(bad)


def test_save_and_read(tmp_path):
    path = str(tmp_path / "cache.json")
    assert T.read(path) == {}
    T.save_entry(path, T.key("gfx950", "fp32", 2, False), (256, 7, 64))
    T.save_entry(path, T.key("gfx950", "fp64", 3, True), (128, 2, 16))
    T.save_entry(path, T.key("gfx950", "fp32", 2, False), (128, 14, 256))  # replaces
    T.save_entry(path, T.key("gfx950", "fp32", 3, 2), (256, 0, 64, 0, 8, 2))
    data = T.read(path)
    assert data == {"gfx950/fp32/D2/plain": [128, 14, 256, 0, 0], "gfx950/fp64/D3/correction": [128, 2, 16, 0, 0],
                    "gfx950/fp32/D3/ito": [256, 0, 64, 8, 2]}
    with open(path, "w") as f:
        json.dump({"gfx950/fp32/D2/plain": [1, 2]}, f)
    with pytest.raises(ValueError):
        T.read(path)


def test_entry_fields():
    """Cache entries map to pdd_tuning fields (block, blocks_per_cu, grab,
    max_launch_paths, refill, bridge); three-field entries take the default
    refill period and bridge form, and max_launch_paths is never cached."""
    assert T.to_fields([256, 0, 64]) == (256, 0, 64, 0, 0, 0)
    assert T.to_fields([128, 3, 16, 4, 1]) == (128, 3, 16, 0, 4, 1)
    assert T.to_entry((128, 3, 16, 999, 4, 1)) == [128, 3, 16, 4, 1]
    assert T.to_entry((256, 0, 64)) == [256, 0, 64, 0, 0]
    assert T.to_fields(T.to_entry((64, 2, 256, 0, 8, 2))) == (64, 2, 256, 0, 8, 2)
    assert T.DEFAULT_SHAPE == (256, 0, 64, 0, 0, 0)


def test_tuning_struct_layout():
    """The binding's pdd_tuning mirrors the C struct: six int32 fields."""
    from paper_1512_02818_amd import pdd
    assert pdd.C.sizeof(pdd.Tuning) == 24
    assert [f[0] for f in pdd.Tuning._fields_] == ["block", "blocks_per_cu", "grab", "max_launch_paths",
                                                   "refill", "bridge"]
    t = pdd.as_tuning((128, 2, 16))
    assert (t.block, t.blocks_per_cu, t.grab, t.max_launch_paths, t.refill, t.bridge) == (128, 2, 16, 0, 0, 0)
    t = pdd.as_tuning((256, 0, 64, 0, 4, 2))
    assert (t.refill, t.bridge) == (4, 2)
    for bad in ((1, 2), (1, 2, 3, 4, 5, 6, 7)):
        with pytest.raises(ValueError):
            pdd.as_tuning(bad)
