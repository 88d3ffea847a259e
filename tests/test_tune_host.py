"""Host-side pieces of the autotuner (no GPU): knob (de)serialisation and
the cache file format."""
from paper_2510_08166_amd import jpt, tune


def test_knobs_round_trip():
    d = {"flags": jpt.TUNE_XCD_TILES, "mark_groups": 1024, "resolve_groups": 0, "decode_groups": 256,
         "idct_groups": 512, "wide_bits": 384}
    assert tune.to_dict(tune.from_dict(d)) == d
    assert tune.to_dict(None) == {k: 0 for k in tune.ORDER}


def test_candidates_start_with_the_default():
    for k in tune.ORDER:
        assert tune.CANDIDATES[k][0] == 0
        assert len(set(tune.CANDIDATES[k])) == len(tune.CANDIDATES[k])


def test_cache_path_env(monkeypatch, tmp_path):
    monkeypatch.setenv("JPT_TUNE_CACHE", str(tmp_path / "x.json"))
    assert tune.default_cache_path() == str(tmp_path / "x.json")
    monkeypatch.setenv("JPT_TUNE_CACHE", str(tmp_path))
    assert tune.default_cache_path() == str(tmp_path / "tune.json")


def test_flag_candidates_are_valid_launches():
    """No candidate forces both forms of resolve's slot lookups (jpt_resolve
    rejects that), and every flag the tuner tries is a declared one."""
    known = jpt.TUNE_XCD_TILES | jpt.TUNE_RESOLVE_PAIRED | jpt.TUNE_RESOLVE_SINGLE
    for f in tune.CANDIDATES["flags"]:
        assert f & ~known == 0
        assert not (f & jpt.TUNE_RESOLVE_PAIRED and f & jpt.TUNE_RESOLVE_SINGLE)
