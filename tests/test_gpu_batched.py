"""Persistent batched launch over (device, energy) instances of uneven size: T and
the diagonal blocks G_ii of every instance against the FP64 oracle under the fixed
rule of tests/parity.py (the bound's block size is the instance's); hipGraph capture
replayed several times with eager work between; the 64-device workload with one
instance of every block size compared block by block."""
import numpy as np
import pytest

from parity import fp64_bound, pmap, rel, task_rgf, terr
from workloads import make_config, make_random

pytestmark = pytest.mark.gpu


def to_dev(wls):
    import torch
    d = torch.device("cuda:0")
    return [(torch.from_numpy(w.H).to(d), torch.from_numpy(w.sigma_L).to(d),
             torch.from_numpy(w.sigma_R).to(d), torch.from_numpy(w.energies).to(d)) for w in wls]


def check_instances(label, items):
    """items: list of (src, wl, energy, G_ii [l, b, b] host, T host)."""
    refs = pmap(task_rgf, [(src, e, None) for (src, _, e, _, _) in items])
    bad = []
    for (src, wl, e, Gd, T), r in zip(items, refs):
        err = rel(Gd, r["G"][1])
        te = terr(T, r["T"])
        tol = fp64_bound(r["kappa"], wl.b)
        print(f"{label} {wl.name} (l={wl.l}, b={wl.b}) energy {e}: kappa {r['kappa']:.2e} "
              f"|dG_ii|/|G_ii| {err:.2e} dT {te:.2e} bound {tol:.2e}", flush=True)
        if not (err <= tol and te <= tol):
            bad.append((wl.name, e, err, te, tol))
    assert not bad, bad


def small_batch():
    shapes = [(10, 32, 3), (7, 64, 2), (5, 128, 2), (12, 96, 2), (1, 32, 1), (3, 128, 1)]
    return [make_random(l, b, 1, ne, seed=3000 + 7 * l + b, eta=1e-3) for (l, b, ne) in shapes]


@pytest.mark.parametrize("schedule", ["longest_first", "interleaved", "input_order"])
def test_small_uneven_batch(lib, schedule):
    import torch
    wls = small_batch()
    outs = lib.solve_batched(to_dev(wls), 0.0, schedule=schedule)
    torch.cuda.synchronize()
    items = []
    for wl, (G, T, info) in zip(wls, outs):
        G, T, info = G.cpu().numpy(), T.cpu().numpy(), info.cpu().numpy()
        assert np.all(info == 0)
        items += [(wl, wl, e, G[e], T[e]) for e in range(wl.ne)]
    check_instances(f"batched/{schedule}", items)


@pytest.mark.parametrize("waves", [8, 4])
def test_block_sizes_and_tiles(lib, waves):
    """Every padded block size (not only those of the 64-device workload), including
    sizes that are not multiples of 16, with one and with two workgroups per compute
    unit."""
    import torch
    shapes = [(6, 16, 2), (5, 48, 2), (4, 80, 1), (3, 112, 2), (7, 32, 1), (2, 128, 1), (5, 64, 1), (3, 96, 1),
              (4, 5, 2), (6, 37, 1), (3, 100, 2), (2, 127, 1), (2, 20, 1)]
    wls = [make_random(l, b, 1, ne, seed=3500 + l + b, eta=1e-3) for (l, b, ne) in shapes]
    outs = lib.solve_batched(to_dev(wls), 0.0, waves=waves)
    torch.cuda.synchronize()
    items = []
    for wl, (G, T, info) in zip(wls, outs):
        G, T, info = G.cpu().numpy(), T.cpu().numpy(), info.cpu().numpy()
        assert np.all(info == 0)
        items += [(wl, wl, e, G[e], T[e]) for e in range(wl.ne)]
    check_instances(f"batched/waves{waves}", items)


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
    instances in one persistent launch.  Every T finite and in [0, b]; for every
    block size the longest device at two energies compared block by block."""
    import torch
    wls = make_config(4)
    outs = lib.solve_batched(to_dev(wls), 0.0)
    torch.cuda.synchronize()
    infos = np.concatenate([o[2].cpu().numpy() for o in outs])
    Ts = [o[1].cpu().numpy() for o in outs]
    assert np.all(infos == 0)
    for wl, T in zip(wls, Ts):
        assert np.all(np.isfinite(T)) and np.all(T >= -1e-8) and np.all(T <= wl.b + 1e-8)
    pick = {}
    for d, w in enumerate(wls):
        if w.b not in pick or w.l > wls[pick[w.b]].l:
            pick[w.b] = d
    assert sorted(pick) == [32, 64, 96, 128]
    items = []
    for b, d in sorted(pick.items()):
        for e in (3, 12):
            items.append((("config", 4, d), wls[d], e, outs[d][0][e].cpu().numpy(), float(Ts[d][e])))
    del outs
    check_instances("config4", items)
