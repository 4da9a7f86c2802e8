"""Measured method choice on the GPU: solve(method="auto") times the sequential
sweep and DDRGF with each admissible domain count on the caller's inputs, keeps
the fastest per workload signature, and its results pass the rule of the method
it chose."""
import numpy as np
import pytest

from parity import check_dd, check_fp64, oracle_results
from test_gpu_rgf import free_gpu, to_dev
from workloads import make_config, make_random

pytestmark = pytest.mark.gpu


@pytest.fixture
def table(tmp_path, monkeypatch):
    from paper_2605_19910_amd import dispatch
    monkeypatch.setattr(dispatch, "TABLE", str(tmp_path / "dispatch.json"))
    monkeypatch.setattr(dispatch, "_cache", {})
    return dispatch


def test_auto_small(lib, table):
    import torch
    wl = make_random(40, 32, 1, 4, seed=5151, eta=1e-3)
    H, sL, sR, E = to_dev(wl)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=0.0, method="auto")
    torch.cuda.synchronize()
    sig = [k for k in table._cache][0]
    rec = table._cache[sig]
    print(f"auto choice for 40 x 32, 4 energies: {rec}", flush=True)
    best = min(rec["timings_ms"].values())
    key = f"{rec['method']}/{rec['domains']}" + (f"/{rec['inner_domains']}" if rec["inner_domains"] else "")
    assert rec["timings_ms"][key] == best
    assert bool((info == 0).all())
    Gn, Tn = G.cpu().numpy(), T.cpu().numpy()
    if rec["method"] == "rgf":
        check_fp64("auto", Gn, Tn, range(4), oracle_results("rgf", wl, range(4)), 1, 32)
    else:
        m = (rec["domains"], rec["inner_domains"]) if rec["inner_domains"] else rec["domains"]
        check_dd("auto", Gn, Tn, range(4), oracle_results("ddrgf", wl, range(4), m=m),
                 oracle_results("dense", wl, range(4)), 1)
    # a second call reuses the choice (no new measurements)
    before = dict(table._cache)
    lib.solve(H, sL, sR, E, eta_d=0.0, method="auto")
    assert table._cache == before


def test_auto_config2_choice(lib, table):
    """The 256 x 128 system: every candidate timed; the choice is the fastest."""
    import torch
    wl = make_config(2)
    H, sL, sR, E = to_dev(wl)
    meas = table.gpu_measure(H, sL, sR, E)
    rec = table.choose(wl.l, wl.b, wl.w, wl.ne, meas, persist=False)
    print(f"auto choice for configuration 2: {rec}", flush=True)
    t = rec["timings_ms"]
    assert "rgf/0" in t and "ddrgf/8" in t and "ddrgf/32/4" in t
    key = f"{rec['method']}/{rec['domains']}" + (f"/{rec['inner_domains']}" if rec["inner_domains"] else "")
    assert t[key] == min(t.values())
    torch.cuda.synchronize()
    free_gpu()


def test_auto_pentadiagonal(lib, table):
    """w = 2: the sequential sweep, native DDRGF and the super-block form are all timed;
    the choice is the fastest and its results pass that method's rule."""
    import torch
    wl = make_random(40, 16, 2, 4, seed=5252, eta=1e-3)
    H, sL, sR, E = to_dev(wl)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=0.0, method="auto")
    torch.cuda.synchronize()
    rec = list(table._cache.values())[0]
    print(f"auto choice for 40 x 16, w = 2, 4 energies: {rec}", flush=True)
    t = rec["timings_ms"]
    assert "rgf/0" in t and "ddrgf/4" in t and "ddrgf_fused/4" in t
    key = f"{rec['method']}/{rec['domains']}"
    assert t[key] == min(t.values())
    assert bool((info == 0).all())
    Gn, Tn = G.cpu().numpy(), T.cpu().numpy()
    if rec["method"] == "rgf":
        check_fp64("auto w=2", Gn, Tn, range(4), oracle_results("nrgf", wl, range(4)), 2, 16)
    else:
        check_dd("auto w=2", Gn, Tn, range(4), oracle_results("ddrgf", wl, range(4), m=rec["domains"]),
                 oracle_results("dense", wl, range(4)), 2)
