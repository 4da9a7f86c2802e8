"""Mixed precision path: block products on FP32 MFMA (operands rounded to FP32, FP32
accumulation, widened to FP64 once per product), Schur pivots inverted in FP64 and
refined once in FP64, and the conditioning switch: an energy keeps FP32 products
only while every Schur pivot has kappa_1(S_i) * 2^-24 <= 1e-5; otherwise it is
recomputed with FP64 products and flagged with RGF_INFO_FP64_PRODUCTS.

Bounds, per energy, against the FP64 oracle:
  * energies that stayed mixed: the mixed target, relative band error and
    |dT| / max(1, T) <= 1e-5;
  * flagged energies: the FP64 rule of tests/parity.py.
The FP32-product error is also reported against the oracle's written-out mixed
variant (oracle.rgf_mixed_products, pinned on the CPU), for information.
"""
import numpy as np
import pytest

from parity import TARGET_MIXED, fp64_bound, gpu_energy, oracle_results, rel, terr
from test_gpu_batched import small_batch, to_dev as to_dev_batch
from test_gpu_rgf import free_gpu, run_gpu_dev
from workloads import make_config, make_random

pytestmark = pytest.mark.gpu

FLAG = 0x40000000


def check_mixed(label, G, T, info, energies, refs, b, emul=None):
    bad, n_mixed = [], 0
    for k, (e, r) in enumerate(zip(energies, refs)):
        st = int(info[e])
        assert st & 0x3FFFFFFF == 0, (e, st)
        fell_back = bool(st & FLAG)
        err = rel(gpu_energy(G, e, 1), r["G"])
        te = terr(T[e], r["T"])
        tol = fp64_bound(r["kappa"], b) if fell_back else TARGET_MIXED
        n_mixed += 0 if fell_back else 1
        extra = ""
        if emul is not None:
            extra = f", emulated mixed vs FP64 {rel(emul[k]['G'], r['G']):.2e}"
        print(f"{label} energy {e}: kappa {r['kappa']:.2e} {'FP64 products' if fell_back else 'mixed'}: "
              f"|dG|/|G| {err:.2e} dT {te:.2e} bound {tol:.2e}{extra}", flush=True)
        if not (err <= tol and te <= tol):
            bad.append((e, fell_back, err, te, tol))
    print(f"{label}: {n_mixed} of {len(refs)} energies kept FP32 products", flush=True)
    assert not bad, bad
    return n_mixed


@pytest.mark.parametrize("l,b,eta_d", [(16, 16, 0.0), (20, 48, 4.0), (12, 128, 4.0), (33, 37, 4.0),
                                       (24, 32, 0.0), (20, 48, 0.5)])
def test_mixed_rgf_small(lib, l, b, eta_d):
    """Small systems, some with a large device broadening eta_d = 4 (pivots with
    kappa_1 well below 1e-5 * 2^24, so FP32 products must be kept) and some without."""
    wl = make_config(1, ne=3) if (l, b) == (16, 16) else make_random(l, b, 1, 3, seed=2100 + l + b, eta=1e-3)
    G, T, info = run_gpu_dev(lib, wl, precision="fp32", eta_d=eta_d)
    es = range(wl.ne)
    refs = oracle_results("rgf", wl, es, eta_d=eta_d)
    emul = oracle_results("mixed", wl, es, eta_d=eta_d)
    n = check_mixed(f"mixed l={l} b={b} eta_d={eta_d}", G, T.cpu().numpy(), info.cpu().numpy(), es, refs, b, emul)
    if eta_d >= 4.0:
        assert n == wl.ne   # these are well conditioned: mixed products must be used


def test_mixed_tolerance_forces_fp64(lib):
    """A tolerance below what any FP32 product reaches sends every energy to FP64
    products: the result is then bitwise the FP64 path's."""
    import torch
    from paper_2605_19910_amd import binding
    wl = make_random(12, 32, 1, 3, seed=8, eta=1e-3)
    dev = torch.device("cuda:0")
    H, sL, sR, E = (torch.from_numpy(x).to(dev) for x in (wl.H, wl.sigma_L, wl.sigma_R, wl.energies))
    plan = binding.Plan(wl.l, wl.b, 1, wl.ne, precision="fp32", mixed_tolerance=1e-30)
    G, T, info = binding.solve(H, sL, sR, E, eta_d=0.5, plan=plan)
    G64, T64, info64 = binding.solve(H, sL, sR, E, eta_d=0.5)
    torch.cuda.synchronize()
    assert bool((info == FLAG).all()) and bool((info64 == 0).all())
    assert torch.equal(T, T64)
    from parity import mask_band
    assert np.array_equal(mask_band(G.cpu().numpy(), 1), mask_band(G64.cpu().numpy(), 1))


def test_mixed_config2_all_energies(lib):
    """The 256 x 128 system, all 64 energies: each either within the mixed target
    with FP32 products, or recomputed with FP64 products and within the FP64 rule."""
    wl = make_config(2)
    G, T, info = run_gpu_dev(lib, wl, precision="fp32")
    refs = oracle_results("rgf", ("config", 2), range(wl.ne))
    check_mixed("config2 mixed", G, T.cpu().numpy(), info.cpu().numpy(), range(wl.ne), refs, wl.b)
    del G
    free_gpu()


def test_mixed_batched_small(lib):
    """The persistent batched kernel with FP32 products on the small uneven batch,
    with and without device broadening."""
    import torch
    for eta_d in (0.0, 0.5):
        wls = small_batch()
        outs = lib.solve_batched(to_dev_batch(wls), eta_d, precision="fp32")
        torch.cuda.synchronize()
        for wl, (G, T, info) in zip(wls, outs):
            refs = oracle_results("rgf", wl, range(wl.ne), eta_d=eta_d)
            Gb = np.zeros((wl.ne, 3, wl.l, wl.b, wl.b), dtype=np.complex128)
            Gb[:, 1] = G.cpu().numpy()
            refs_d = [dict(r, G=np.stack([np.zeros_like(r["G"][1]), r["G"][1], np.zeros_like(r["G"][1])]))
                      for r in refs]
            check_mixed(f"batched mixed l={wl.l} b={wl.b} eta_d={eta_d}", Gb, T.cpu().numpy(),
                        info.cpu().numpy(), range(wl.ne), refs_d, wl.b)


def test_mixed_batched_config4(lib):
    """The 64-device batched workload with FP32 products: every instance either kept
    FP32 products (then within the mixed target) or was recomputed with FP64
    products (flagged, then within the FP64 rule); the longest device of each block
    size at two energies against the oracle, and every T finite and in [0, b]."""
    import torch
    from parity import pmap, task_rgf
    wls = make_config(4)
    outs = lib.solve_batched(to_dev_batch(wls), 0.0, precision="fp32")
    torch.cuda.synchronize()
    infos = [o[2].cpu().numpy() for o in outs]
    assert all(np.all(i & 0x3FFFFFFF == 0) for i in infos)
    n_fp32 = sum(int(np.sum((i & FLAG) == 0)) for i in infos)
    print(f"config4 mixed: {n_fp32} of {sum(len(i) for i in infos)} instances kept FP32 products", flush=True)
    for wl, o in zip(wls, outs):
        T = o[1].cpu().numpy()
        assert np.all(np.isfinite(T)) and np.all(T >= -1e-5) and np.all(T <= wl.b + 1e-5)
    pick = {}
    for d, w in enumerate(wls):
        if w.b not in pick or w.l > wls[pick[w.b]].l:
            pick[w.b] = d
    items = [(d, e) for b, d in sorted(pick.items()) for e in (3, 12)]
    refs = pmap(task_rgf, [(("config", 4, d), e, None) for d, e in items])
    bad = []
    for (d, e), r in zip(items, refs):
        wl = wls[d]
        fell_back = bool(infos[d][e] & FLAG)
        err = rel(outs[d][0][e].cpu().numpy(), r["G"][1])
        te = terr(outs[d][1][e].item(), r["T"])
        tol = fp64_bound(r["kappa"], wl.b) if fell_back else TARGET_MIXED
        print(f"config4 mixed device {d} (l={wl.l}, b={wl.b}) energy {e}: kappa {r['kappa']:.2e} "
              f"{'FP64 products' if fell_back else 'mixed'} |dG_ii|/|G_ii| {err:.2e} dT {te:.2e} bound {tol:.2e}",
              flush=True)
        if not (err <= tol and te <= tol):
            bad.append((d, e, err, te, tol))
    assert not bad, bad


def test_mixed_ddrgf_rejected(lib):
    """Mixed DDRGF is refused: the closed interiors' pivots are ill-conditioned at
    most energies of these generators (every interior would fall back to FP64)."""
    with pytest.raises(lib.RgfError) as ei:
        lib.Plan(16, 16, 1, 2, method="ddrgf", domains=2, precision="fp32")
    assert ei.value.code == 2
