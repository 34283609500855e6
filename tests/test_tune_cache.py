"""The autotuner's persisted cache (process-wide store of tuned launch shapes
and its JSON file), exercised through the C ABI without a GPU: round trips,
merging, and refusal of files that are not a cache or hold values the
library could not launch."""
import json
import os

import pytest


@pytest.fixture()
def dg():
    import paper_2011_11134_amd as d
    d.tune_cache_clear()
    yield d
    d.tune_cache_clear()


def _entry(key, **kw):
    e = {"key": key, "grid": 0, "cull_mult": 0, "exact_mult": 0, "bwd_mult": 0, "tile_rows": 0,
         "ms": 0.5}
    e.update(kw)
    return e


def _write(path, entries, **top):
    doc = {"format": "dgal-tune-cache", "version": 1, "entries": entries}
    doc.update(top)
    with open(path, "w") as f:
        json.dump(doc, f)


def _lines(dg):
    return sorted(dg.tune_cache_report().strip().splitlines())


def test_round_trip(dg, tmp_path):
    ents = [_entry("gfx950/matrix_fwd/K4/fixed1/z1/seg1/b17.7", cull_mult=16, exact_mult=8,
                   tile_rows=4, ms=0.1234),
            _entry("gfx950/pairs_fwd/K8/fixed0/z0/seg1/b19", grid=4096),
            _entry("gfx950/matrix_bwd/K4/fixed1/z1/seg1/b17.7", bwd_mult=16)]
    src = tmp_path / "in.json"
    _write(src, ents)
    assert dg.tune_cache_load(str(src)) == 3
    lines = _lines(dg)
    assert len(lines) == 3
    assert any("matrix_fwd" in ln and "cull=16" in ln and "exact=8" in ln and "rows=4" in ln
               for ln in lines)
    assert any("pairs_fwd" in ln and "grid=4096" in ln for ln in lines)
    out = tmp_path / "out.json"
    dg.tune_cache_save(str(out))
    doc = json.loads(out.read_text())
    assert doc["format"] == "dgal-tune-cache" and doc["version"] == 1
    got = {e["key"]: e for e in doc["entries"]}
    assert set(got) == {e["key"] for e in ents}
    for e in ents:
        for k in ("grid", "cull_mult", "exact_mult", "bwd_mult", "tile_rows"):
            assert got[e["key"]][k] == e[k], (e["key"], k)
        assert abs(got[e["key"]]["ms"] - e["ms"]) < 1e-6
    # what was saved loads back to the same store
    dg.tune_cache_clear()
    assert dg.tune_cache_report() == ""
    assert dg.tune_cache_load(str(out)) == 3
    assert _lines(dg) == lines
    assert not [p for p in os.listdir(tmp_path) if ".tmp." in p]  # the rename left nothing


def test_merge_replaces_by_key_and_ignores_unknown_fields(dg, tmp_path):
    k1, k2 = "gfx950/pairs_bwd/K4/fixed1/z0/seg0/b20", "gfx942/pairs_bwd/K4/fixed1/z0/seg0/b20"
    f1, f2 = tmp_path / "a.json", tmp_path / "b.json"
    _write(f1, [_entry(k1, grid=1024), _entry(k2, grid=2048)])
    _write(f2, [dict(_entry(k1, grid=512), note="kept out")], comment={"any": [1, 2, None]})
    assert dg.tune_cache_load(str(f1)) == 2
    assert dg.tune_cache_load(str(f2)) == 1
    lines = _lines(dg)
    assert len(lines) == 2
    assert any(ln.startswith(k1) and "grid=512" in ln for ln in lines)
    assert any(ln.startswith(k2) and "grid=2048" in ln for ln in lines)


@pytest.mark.parametrize("text", [
    "",                                                       # empty
    "{",                                                      # truncated
    "[]",                                                     # not an object
    '{"format": "other", "version": 1, "entries": []}',       # foreign format
    '{"format": "dgal-tune-cache", "version": 2, "entries": []}',
    '{"format": "dgal-tune-cache", "version": 1}',            # no entries
    '{"format": "dgal-tune-cache", "version": 1, "entries": [1]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"grid": 0}]}',  # no key
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "a b"}]}',  # bad key
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "k", "tile_rows": 5}]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "k", "cull_mult": -1}]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "k", "exact_mult": 65}]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "k", "grid": 1.5}]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "k", "grid": 1e30}]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "k", "grid": "8"}]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "k", "ms": -1}]}',
    '{"format": "dgal-tune-cache", "version": 1, "entries": []} trailing',
    '{"format": "dgal-tune-cache", "version": 1, "entries": [' + "[" * 40 + "]" * 40 + "]}",
])
def test_malformed_files_are_refused_whole(dg, tmp_path, text):
    good = tmp_path / "good.json"
    _write(good, [_entry("gfx950/pairs_fwd/K4/fixed1/z0/seg0/b10", grid=256)])
    assert dg.tune_cache_load(str(good)) == 1
    before = _lines(dg)
    bad = tmp_path / "bad.json"
    bad.write_text(text)
    with pytest.raises(dg.DgalError) as e:
        dg.tune_cache_load(str(bad))
    assert e.value.status == dg.DGAL_EINVAL
    assert _lines(dg) == before  # nothing merged


def test_file_errors(dg, tmp_path):
    with pytest.raises(dg.DgalError) as e:
        dg.tune_cache_load(str(tmp_path / "missing.json"))
    assert e.value.status == dg.DGAL_EIO
    with pytest.raises(dg.DgalError) as e:
        dg.tune_cache_save(str(tmp_path / "no_such_dir" / "x.json"))
    assert e.value.status == dg.DGAL_EIO
    assert dg.lib.dgal_tune_cache_load(None) == dg.DGAL_EINVAL
    assert dg.lib.dgal_tune_cache_save(b"") == dg.DGAL_EINVAL
    assert dg.lib.dgal_tune_cache_report(None, 5) == dg.DGAL_EINVAL
    assert dg.lib.dgal_tune_cache_report(None, 0) == 0
