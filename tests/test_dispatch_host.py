"""Host logic of the measured method choice (no GPU): admissible candidates,
tie-breaking, and the per-signature cache."""
import pytest

from paper_2605_19910_amd import dispatch


def test_candidates():
    c = dispatch.candidates(256, 128, 1, "fp64")
    assert c[0] == ("rgf", 0)
    assert [x[1] for x in c if x[0] == "ddrgf" and len(x) == 2] == [2, 4, 8, 16, 32]
    assert [x[1:] for x in c if len(x) == 3] == [(16, 2), (16, 4), (16, 8), (32, 2), (32, 4), (32, 8)]
    # w = 2: native n-diagonal DDRGF, interiors of at least w layers, one level only
    assert [x for x in dispatch.candidates(512, 64, 2, "fp64") if x[0] == "ddrgf"] == \
        [("ddrgf", m) for m in (2, 4, 8, 16, 32)]
    assert [x for x in dispatch.candidates(512, 64, 2, "fp64") if x[0] == "ddrgf_fused"] == \
        [("ddrgf_fused", m) for m in (2, 4, 8, 16, 32)]
    assert [x[1] for x in dispatch.candidates(511, 100, 2, "fp64") if x[0] == "ddrgf"] == [2, 4, 8, 16, 32]
    assert not [x for x in dispatch.candidates(511, 100, 2, "fp64") if x[0] == "ddrgf_fused"]
    assert not [x for x in dispatch.candidates(512, 100, 2, "fp64") if x[0] == "ddrgf_fused"]
    assert [x[1] for x in dispatch.candidates(30, 64, 3, "fp64") if x[0] == "ddrgf"] == [2, 4]
    assert [x[1] for x in dispatch.candidates(10, 8, 1, "fp64") if x[0] == "ddrgf"] == [2, 4]
    # mixed precision: sequential only; methods filter
    assert dispatch.candidates(256, 128, 1, "fp32") == [("rgf", 0)]
    assert dispatch.candidates(256, 128, 1, "fp64", methods=("ddrgf",))[0] == ("ddrgf", 2)


def test_pick_ties():
    assert dispatch.pick({("ddrgf", 8): 1.0, ("rgf", 0): 1.0}) == ("rgf", 0)
    assert dispatch.pick({("ddrgf", 8): 1.0, ("ddrgf", 4): 1.0}) == ("ddrgf", 4)
    assert dispatch.pick({("ddrgf", 8): 0.5, ("rgf", 0): 1.0}) == ("ddrgf", 8)
    assert dispatch.pick({("ddrgf", 16, 2): 1.0, ("ddrgf", 16): 1.0}) == ("ddrgf", 16)


def test_choose_caches(tmp_path, monkeypatch):
    monkeypatch.setattr(dispatch, "TABLE", str(tmp_path / "table.json"))
    monkeypatch.setattr(dispatch, "_cache", {})
    calls = []

    def measure(method, m, m2=0):
        calls.append((method, m, m2))
        return {"rgf": 10.0}.get(method, 20.0 - m + 0.5 * m2)

    rec = dispatch.choose(40, 32, 1, 8, measure)
    assert (rec["method"], rec["domains"]) == ("ddrgf", 16)
    n = len(calls)
    assert n == len(dispatch.candidates(40, 32, 1))
    again = dispatch.choose(40, 32, 1, 8, measure)
    assert again == rec and len(calls) == n
    # persisted: a fresh process (empty memory cache) reads the table
    monkeypatch.setattr(dispatch, "_cache", {})
    assert dispatch.choose(40, 32, 1, 8, measure) == rec and len(calls) == n
    # restricted choice is a different signature
    rec2 = dispatch.choose(40, 32, 1, 8, measure, methods=("rgf",))
    assert rec2["method"] == "rgf"
    with pytest.raises(ValueError):
        dispatch.choose(40, 32, 1, 8, measure, precision="fp32", methods=("ddrgf",))
