"""GPU parity of the sequential RGF path (Algorithm 1) against the FP64 oracle,
through the C ABI.

Bound: the fixed rule of tests/parity.py, max(1e-10, 2 b u kappa_max) per energy
(relative Frobenius error over every band block inside the matrix, and
|dT| / max(1, T)), kappa_max from the oracle's run at that energy.  At small sizes
the pivots are well conditioned and the bound is the 1e-10 target itself.  At the
full 256 x 128 size every one of the 64 energies is compared; four of them are also
compared with an extended-precision run of the same elimination, which measures how
far the GPU and the FP64 oracle each are from the exact selected inverse.
"""
import numpy as np
import pytest

import oracle
from parity import check_fp64, fp64_bound, gpu_energy, mask_band, oracle_results, rel, terr
from workloads import make_config, make_random, make_uniform_chain, surface_sigma

pytestmark = pytest.mark.gpu


def to_dev(wl):
    import torch
    d = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(wl.H)).to(d), torch.from_numpy(wl.sigma_L).to(d),
            torch.from_numpy(wl.sigma_R).to(d), torch.from_numpy(wl.energies).to(d))


def run_gpu_dev(lib, wl, method="rgf", eta_d=None, domains=0, precision="fp64", ddrgf_form="native"):
    """Solve on the GPU; returns (G, T, info) as device tensors."""
    import torch
    H, sL, sR, E = to_dev(wl)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=wl.eta_d if eta_d is None else eta_d, method=method,
                           domains=domains, precision=precision, ddrgf_form=ddrgf_form)
    torch.cuda.synchronize()
    return G, T, info


def run_gpu(lib, wl, method="rgf", eta_d=None, domains=0, precision="fp64", ddrgf_form="native"):
    """Solve on the GPU; returns host arrays (small systems only)."""
    G, T, info = run_gpu_dev(lib, wl, method, eta_d, domains, precision, ddrgf_form)
    return G.cpu().numpy(), T.cpu().numpy(), info.cpu().numpy()


def free_gpu():
    import gc

    import torch
    gc.collect()
    torch.cuda.empty_cache()


def test_config1(lib):
    wl = make_config(1)
    G, T, info = run_gpu(lib, wl)
    assert np.all(info == 0)
    check_fp64("config1", G, T, range(wl.ne), oracle_results("rgf", wl, range(wl.ne)), 1, wl.b)
    # and against the definition itself (dense inverse)
    check_fp64("config1/dense", G, T, range(wl.ne), oracle_results("dense", wl, range(wl.ne)), 1, wl.b)


# ragged block sizes (not multiples of 16) and layer counts, one to eight tiles per side
@pytest.mark.parametrize("l,b,ne", [(1, 5, 2), (2, 16, 2), (3, 1, 2), (7, 20, 3), (13, 37, 2),
                                    (40, 48, 2), (9, 64, 2), (17, 81, 2), (11, 100, 2),
                                    (6, 112, 2), (12, 128, 2), (5, 127, 2)])
def test_ragged_sizes(lib, l, b, ne):
    wl = make_random(l, b, 1, ne, seed=500 + l * 7 + b, eta=1e-3)
    G, T, info = run_gpu(lib, wl)
    assert np.all(info == 0)
    check_fp64(f"ragged l={l} b={b}", G, T, range(ne), oracle_results("rgf", wl, range(ne)), 1, b)


def test_device_broadening(lib):
    wl = make_random(24, 32, 1, 3, seed=9, eta=1e-3)
    G, T, info = run_gpu(lib, wl, eta_d=0.01)
    assert np.all(info == 0)
    check_fp64("eta_d", G, T, range(3), oracle_results("rgf", wl, range(3), eta_d=0.01), 1, wl.b)


def test_config2_all_energies(lib):
    """All 64 energies of the 256-layer, 128-orbital system in the benchmark launch,
    every band block and T compared with the oracle."""
    wl = make_config(2)
    G, T, info = run_gpu_dev(lib, wl)
    assert bool((info == 0).all())
    Th = T.cpu().numpy()
    assert np.all(np.isfinite(Th)) and np.all(Th >= -1e-9) and np.all(Th <= wl.b + 1e-9)
    refs = oracle_results("rgf", ("config", 2), range(wl.ne))
    check_fp64("config2 rgf", G, Th, range(wl.ne), refs, 1, wl.b)
    del G
    free_gpu()


def test_config2_distance_to_exact(lib):
    """Energies 0, 33, 63 and the one with the worst-conditioned pivot: GPU RGF, GPU
    DDRGF (8 domains) and the FP64 oracle, each against the extended-precision run
    of the same elimination (the exact selected inverse to ~kappa * 1e-19).  The GPU
    RGF must be within the FP64 rule of the exact answer; the ratios to the oracle's
    own error are printed."""
    wl = make_config(2)
    kap = [r["kappa"] for r in oracle_results("rgf", ("config", 2), range(wl.ne))]
    worst = int(np.argmax(kap))
    es = sorted({0, 33, 63, worst})
    ext = oracle_results("ext", ("config", 2), es)
    orc = oracle_results("rgf", ("config", 2), es)
    Gr, Tr, info_r = run_gpu_dev(lib, wl)
    assert bool((info_r == 0).all())
    rows = []
    for e, x, o in zip(es, ext, orc):
        eg = rel(gpu_energy(Gr, e, 1), x["G"])
        eo = rel(o["G"], x["G"])
        rows.append((e, eg, eo, terr(Tr[e].item(), x["T"]), terr(o["T"], x["T"])))
    del Gr
    free_gpu()
    Gd, Td, info_d = run_gpu_dev(lib, wl, method="ddrgf", domains=8)
    assert bool((info_d == 0).all())
    for (e, eg, eo, tg, to), x in zip(rows, ext):
        ed = rel(gpu_energy(Gd, e, 1), x["G"])
        print(f"config2 energy {e}: kappa {kap[e]:.2e}  vs exact: GPU RGF {eg:.2e} (T {tg:.2e}), "
              f"oracle RGF {eo:.2e} (T {to:.2e}), ratio {eg / max(eo, 1e-300):.2f}; GPU DDRGF {ed:.2e}",
              flush=True)
        tol = fp64_bound(kap[e], wl.b)
        assert eg <= tol and tg <= tol, (e, eg, tg, tol)
    del Gd
    free_gpu()


def test_uniform_chain_full_size(lib):
    """Uniform chain at the full size: in-band T(E) is the integer number of open
    channels (any size), and with eta_d = eta every block has a closed form."""
    b, l, ne = 128, 256, 64
    wl = make_uniform_chain(l, b, ne, eta=1e-6)
    eps = wl.meta["eps"]
    G, T, info = run_gpu_dev(lib, wl)
    assert bool((info == 0).all())
    n_open = np.array([np.sum(np.abs(E - eps) < 2) for E in wl.energies])
    assert np.max(np.abs(T.cpu().numpy() - n_open)) < 1e-7
    del G
    G, T, info = run_gpu_dev(lib, wl, eta_d=wl.eta)
    V = wl.meta["V"]
    for e in (0, 21, 40, 63):
        Ge = G[e].cpu().numpy()
        z = wl.energies[e] + 1j * wl.eta - eps
        s = np.sqrt(z - 2.0) * np.sqrt(z + 2.0)
        for i in (0, 1, 100, 254, 255):
            for k in (-1, 0, 1):
                j = i + k
                if not (0 <= j < l):
                    continue
                ex = (V * (surface_sigma(z) ** abs(k) / s)[None, :]) @ V.conj().T
                assert np.abs(Ge[1 + k, i] - ex).max() <= 1e-9 * np.abs(ex).max(), (e, i, k)
    del G
    free_gpu()


def test_singular_pivot_reported(lib):
    """Sigma_R = 0 and H_{l-1,l-1} = E I make the first Schur pivot exactly zero."""
    wl = make_random(6, 8, 1, 2, seed=3, eta=1e-3)
    wl.sigma_R[0] = 0.0
    wl.H[1, 5] = wl.energies[0] * np.eye(8)
    G, T, info = run_gpu(lib, wl)
    assert info[0] == 6 and info[1] == 0
    assert np.all(np.isnan(G[0])) and np.isnan(T[0])
    assert np.all(np.isfinite(mask_band(G[1], 1)))


def test_nonfinite_input_reported(lib):
    wl = make_random(5, 8, 1, 1, seed=4, eta=1e-3)
    wl.H[1, 2, 3, 3] = np.nan
    G, T, info = run_gpu(lib, wl)
    assert info[0] != 0 and np.isnan(T[0])


def test_bitwise_deterministic(lib):
    wl = make_random(20, 48, 1, 4, seed=5, eta=1e-3)
    G1, T1, _ = run_gpu(lib, wl)
    G2, T2, _ = run_gpu(lib, wl)
    assert np.array_equal(mask_band(G1, 1), mask_band(G2, 1)) and np.array_equal(T1, T2)
