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
    data = T.read(path)
    assert data == {"gfx950/fp32/D2/plain": [128, 14, 256], "gfx950/fp64/D3/correction": [128, 2, 16]}
    with open(path, "w") as f:
        json.dump({"gfx950/fp32/D2/plain": [1, 2]}, f)
    with pytest.raises(ValueError):
        T.read(path)
