"""Two-level DDRGF on the GPU (the reduced separator system solved by DDRGF again)
against the oracle's multi-level DDRGF, under the DDRGF rule of tests/parity.py
(kappa_max over every level, the largest interior of any level, the product of the
levels' rho), and its distance to the exact band printed beside."""
import numpy as np
import pytest

from parity import check_dd, oracle_results
from test_gpu_rgf import free_gpu, to_dev
from workloads import make_config, make_dominant, make_random

pytestmark = pytest.mark.gpu


def run_ml(lib, wl, m, m2, eta_d=None, ne=None):
    import torch
    H, sL, sR, E = to_dev(wl)
    # two levels for w > 1 run on the w-layer super-block form
    plan = lib.Plan(wl.l, wl.b, wl.w, wl.ne, method="ddrgf", domains=m, inner_domains=m2,
                    ddrgf_form="fused" if wl.w > 1 else "native")
    G, T, info = lib.solve(H, sL, sR, E, eta_d=wl.eta_d if eta_d is None else eta_d, plan=plan)
    torch.cuda.synchronize()
    plan.close()
    return G, T, info


@pytest.mark.parametrize("l,b,w,m,m2", [(40, 8, 1, 8, 2), (64, 16, 1, 16, 4), (33, 37, 1, 8, 3), (48, 20, 2, 6, 2),
                                        (100, 64, 1, 20, 5), (30, 128, 1, 6, 2), (12, 4, 1, 2, 1)])
def test_two_level_small(lib, l, b, w, m, m2):
    wl = make_random(l, b, w, 2, seed=6100 + l + b, eta=1e-3)
    G, T, info = run_ml(lib, wl, m, m2)
    assert bool((info == 0).all())
    refs = oracle_results("ddrgf", wl, range(2), m=(m, m2))
    check_dd(f"two-level ddrgf l={l} b={b} w={w} m={m} m2={m2}", G.cpu().numpy(), T.cpu().numpy(), range(2), refs,
             oracle_results("dense", wl, range(2)), w)


def test_two_level_with_broadening(lib):
    wl = make_random(60, 24, 1, 3, seed=61, eta=1e-3)
    G, T, info = run_ml(lib, wl, 12, 3, eta_d=0.05)
    assert bool((info == 0).all())
    refs = oracle_results("ddrgf", wl, range(3), eta_d=0.05, m=(12, 3))
    check_dd("two-level ddrgf eta_d", G.cpu().numpy(), T.cpu().numpy(), range(3), refs,
             oracle_results("dense", wl, range(3), eta_d=0.05), 1)


def test_two_level_dominant_full_size(lib):
    """256 x 128, 64 energies, 32 pairs and 4 inner pairs on the diagonally dominant
    system: every energy within the rule, here the FP64 target."""
    src = ("dominant", 256, 128, 1, 64, 202)
    wl = make_dominant(*src[1:])
    G, T, info = run_ml(lib, wl, 32, 4)
    assert bool((info == 0).all())
    refs = oracle_results("ddrgf", src, range(wl.ne), m=(32, 4))
    rows = check_dd("two-level dominant 256x128", G, T.cpu().numpy(), range(wl.ne), refs,
                    oracle_results("rgf", src, range(wl.ne)), 1)
    assert max(r[3] for r in rows) <= 1e-9
    del G
    free_gpu()


def test_two_level_config2_sampled(lib):
    """The 256 x 128 system with 32 pairs and 4 inner pairs, 9 energies."""
    wl = make_config(2)
    G, T, info = run_ml(lib, wl, 32, 4)
    assert bool((info == 0).all())
    es = [0, 8, 16, 24, 32, 40, 48, 56, 63]
    refs = oracle_results("ddrgf", ("config", 2), es, m=(32, 4))
    check_dd("two-level config2", G, T.cpu().numpy(), es, refs, oracle_results("rgf", ("config", 2), es), 1)
    del G
    free_gpu()


def test_two_level_few_energies_timing(lib):
    """Few energies (4) on 256 x 128: time of one level with 32 pairs (reduced system
    of 32 layers by one sequential sweep per energy) against two levels (32, 4)."""
    import torch
    wl = make_config(2, ne=4)
    H, sL, sR, E = to_dev(wl)
    out = {}
    for label, kw in (("one level", dict(domains=32)), ("two levels", dict(domains=32, inner_domains=4)),
                      ("sequential", dict())):
        method = "ddrgf" if kw else "rgf"
        plan = lib.Plan(wl.l, wl.b, 1, wl.ne, method=method, **kw)
        lib.solve(H, sL, sR, E, plan=plan)
        plan.set_timing(True, 64)
        G, T, info = lib.solve(H, sL, sR, E, plan=plan)
        times = plan.kernel_times()
        plan.close()
        torch.cuda.synchronize()
        assert bool((info == 0).all())
        out[label] = (sum(v[0] for v in times.values()), T.cpu().numpy())
        print(f"4 energies, {label}: {out[label][0]:.2f} ms ({', '.join(f'{k} {v[0]:.2f}' for k, v in times.items())})",
              flush=True)
    assert np.allclose(out["one level"][1], out["two levels"][1], rtol=1e-3, atol=1e-6)
