"""Host logic of the autotuner: candidate sets, cache keys, selection, JSON cache."""
import json

import pytest

from paper_1410_5242_amd import autotune as A


def test_size_bucket_and_keys():
    assert A.size_bucket(1) == 1
    assert A.size_bucket(1_048_576) == 1_048_576
    assert A.size_bucket(1_048_577) == 1_048_576
    assert A.size_bucket(2_097_151) == 1_048_576
    assert A.sweep_key(0, 32, 1_048_576, (64, 64, 64)) == "sweep:c128:R32:N1048576:L64x64x64"
    assert A.batch_key(1, 8, 512, 14_044_416) == "batched:c64:R8:n512:N8388608"
    assert A.width_key(0, 32, 2048) == "width:c128:S32:N2048"


def test_candidates_are_valid_tunings():
    for lat in (False, True):
        cs = A.sweep_candidates(32, lat)
        assert len(cs) == len({json.dumps(c, sort_keys=True) for c in cs}), "duplicates"
        for c in cs:
            assert set(c) == set(A.SWEEP_FIELDS)
            assert all(isinstance(v, int) and v >= 0 for v in c.values())
            assert 0 <= c["stream"] <= 3 and c["lattice"] in (0, 2)
        assert any(c["lattice"] == 2 for c in cs) == lat
    for mw in (8, 16):
        bs = A.batch_candidates(mw)
        assert bs and all(set(b) == set(A.BATCH_FIELDS) for b in bs)
        assert all(b["waves"] <= mw and b["waves"] * b["wg_per_cu"] <= 32 for b in bs)


def test_block_widths():
    assert A.block_widths(32) == [1, 2, 4, 8, 16, 32]
    assert A.block_widths(12) == [1, 2, 4]
    assert A.block_widths(1) == [1]
    assert A.block_widths(128) == [1, 2, 4, 8, 16, 32, 64]


def test_pick_best_takes_fastest_and_first_on_ties():
    t = [A.Trial({"a": 0}, 2.0), A.Trial({"a": 1}, 1.0), A.Trial({"a": 2}, 1.0), A.Trial({"a": 3}, 3.0)]
    assert A.pick_best(t).params == {"a": 1}
    with pytest.raises(ValueError):
        A.pick_best([])


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    c = A.TuningCache(path)
    assert c.get("x") is None
    r = A.TuneResult("sweep:c128:R32:N1024:L-", {"wg_per_cu": 8}, 1e-3, [A.Trial({"wg_per_cu": 8}, 1e-3)])
    c.put(r)
    c.save()
    c2 = A.TuningCache(path)
    assert c2.get("sweep:c128:R32:N1024:L-") == {"wg_per_cu": 8}
    data = json.load(open(path))
    assert data["format"] == 1 and data["entries"]["sweep:c128:R32:N1024:L-"]["trials"][0]["seconds"] == 1e-3


def test_time_call_reports_best_of_repeats():
    calls = []
    s = A.time_call(lambda: calls.append(1), repeats=4)
    assert len(calls) == 5 and s >= 0.0


def test_pick_best_keeps_default_within_margin():
    # the first trial is the library default: kept unless beaten by more than the margin
    t = [A.Trial({"d": 0}, 1.0), A.Trial({"a": 1}, 0.99), A.Trial({"b": 2}, 0.995)]
    assert A.pick_best(t, margin=0.02).params == {"d": 0}
    assert A.pick_best(t, margin=0.0).params == {"a": 1}
    t.append(A.Trial({"c": 3}, 0.95))
    assert A.pick_best(t, margin=0.02).params == {"c": 3}


def test_sell_candidates_are_valid_layouts():
    cands = A.sell_candidates()
    assert cands[0] == {"C": 8, "sigma": 1024}          # the library default first
    assert len({(c["C"], c["sigma"]) for c in cands}) == len(cands)
    for c in cands:
        assert c["C"] in (1, 2, 4, 8, 16, 32, 64)
        assert c["sigma"] == 1 or c["sigma"] % c["C"] == 0
    assert {"C": 1, "sigma": 1} in cands                # CRS is always tried
    assert A.sell_key(0, 32, 1000, 13000) == "sell:c128:R32:N512:nnz8192"
