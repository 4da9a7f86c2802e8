"""Persistent batched launch over (device, energy) instances of uneven size: T and
the diagonal blocks G_ii of every instance against the FP64 oracle; hipGraph
capture replayed several times with eager work between; the 64-device workload."""
import numpy as np
import pytest

import oracle
from workloads import make_config, make_random

from test_gpu_rgf import rel

pytestmark = pytest.mark.gpu


def to_dev(wls):
    import torch
    d = torch.device("cuda:0")
    return [(torch.from_numpy(w.H).to(d), torch.from_numpy(w.sigma_L).to(d),
             torch.from_numpy(w.sigma_R).to(d), torch.from_numpy(w.energies).to(d)) for w in wls]


def check_instance(wl, Gd, T, e, noise=False, tol=1e-10):
    args = (wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], wl.eta_d)
    r = oracle.rgf(*args, extras=True)
    ref = r["G"][1]
    Tref = oracle.transmission(r["row0"][wl.l - 1], wl.sigma_L[e], wl.sigma_R[e])
    if noise:
        # the largest of three perturbed oracle runs (see test_gpu_rgf.check_energies)
        # (drawn until the bound holds: the maximum of three is never below them)
        err0 = rel(Gd, ref)
        terr0 = abs(T - Tref) / max(1.0, abs(Tref))
        for s in range(3):
            rn = oracle.rgf(*args, extras=True, pivot_noise=500 + e + 100000 * s)
            Tn = oracle.transmission(rn["row0"][wl.l - 1], wl.sigma_L[e], wl.sigma_R[e])
            tol = max(tol, 2 * max(rel(rn["G"][1], ref), abs(Tn - Tref) / max(1.0, abs(Tref))))
            if err0 <= tol and terr0 <= tol:
                break
    err = rel(Gd, ref)
    assert err <= tol, (wl.name, e, err, tol)
    assert abs(T - Tref) <= tol * max(1.0, abs(Tref)), (wl.name, e, T, Tref)


def small_batch():
    shapes = [(10, 32, 3), (7, 64, 2), (5, 128, 2), (12, 96, 2), (1, 32, 1), (3, 128, 1)]
    return [make_random(l, b, 1, ne, seed=3000 + 7 * l + b, eta=1e-3) for (l, b, ne) in shapes]


@pytest.mark.parametrize("schedule", ["longest_first", "interleaved", "input_order"])
def test_small_uneven_batch(lib, schedule):
    import torch
    wls = small_batch()
    outs = lib.solve_batched(to_dev(wls), 0.0, schedule=schedule)
    torch.cuda.synchronize()
    for wl, (G, T, info) in zip(wls, outs):
        G, T, info = G.cpu().numpy(), T.cpu().numpy(), info.cpu().numpy()
        assert np.all(info == 0)
        for e in range(wl.ne):
            check_instance(wl, G[e], T[e], e)


def test_graph_replays_match_eager(lib):
    """Captured on a side stream; three replays, eager torch work and host syncs in
    between, each bitwise equal to a direct launch on the default stream."""
    import torch
    wls = small_batch()
    sysd = to_dev(wls)
    shapes = [(w.l, w.b, w.ne) for w in wls]
    plan = lib.BatchedPlan(shapes)
    ref = lib.solve_batched(sysd, 0.0, plan=plan)           # default stream: direct launch
    torch.cuda.synchronize()
    ref = [(G.clone(), T.clone()) for (G, T, _) in ref]
    side = torch.cuda.Stream()
    outs = None
    with torch.cuda.stream(side):
        for rep in range(3):
            if outs is None:
                outs = lib.solve_batched(sysd, 0.0, plan=plan, stream=side)
                entries = [dict(H=H, sigma_L=sL, sigma_R=sR, energies=E, G_diag=o[0], T=o[1], info=o[2])
                           for (H, sL, sR, E), o in zip(sysd, outs)]
                table = lib.device_table(entries, sysd[0][0].device)
                ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=sysd[0][0].device)
            for (G, T, _) in outs:
                G.zero_()
                T.zero_()
            lib.rgf_batched_solve(plan, table, 0.0, ws, side.cuda_stream)
            side.synchronize()
            junk = torch.randn(1 << 20, device=sysd[0][0].device).sum()   # eager work between replays
            torch.cuda.synchronize()
            for (G, T, _), (Gr, Tr) in zip(outs, ref):
                assert torch.equal(G, Gr) and torch.equal(T, Tr), rep
    del junk


def test_config4_full_workload(lib):
    """64 devices, b in {32, 64, 96, 128}, l in [64, 512], 16 energies each: 1024
    instances in one persistent launch; three instances checked block by block."""
    import torch
    wls = make_config(4)
    outs = lib.solve_batched(to_dev(wls), 0.0)
    torch.cuda.synchronize()
    infos = np.concatenate([o[2].cpu().numpy() for o in outs])
    Ts = np.concatenate([o[1].cpu().numpy() for o in outs])
    assert np.all(infos == 0) and np.all(np.isfinite(Ts))
    by_b = {}
    for d, w in enumerate(wls):
        by_b.setdefault(w.b, d)
    for b, d in sorted(by_b.items())[::2]:
        wl = wls[d]
        G = outs[d][0][3].cpu().numpy()
        check_instance(wl, G, float(outs[d][1][3].item()), 3, noise=True)
