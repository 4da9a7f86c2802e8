"""GPU parity of the block n-diagonal paths (n = 2w + 1) against the FP64 oracle,
under the fixed rule of tests/parity.py:

* sequential: the native n-diagonal sweep (Sec. 2.3) against the oracle's n-RGF;
* DDRGF with separators of w layers against the oracle's DDRGF (same algorithm)
  under the DDRGF rule of tests/parity.py, its distance to the exact band printed
  beside.
At the full pentadiagonal size (512 layers of 64, 128 energies) 17 energies spread
over the grid are compared for each method, and two of them also against the
extended-precision reference.
"""
import numpy as np
import pytest

from parity import check_dd, check_fp64, fp64_bound, gpu_energy, oracle_results, rel, terr
from test_gpu_rgf import free_gpu, run_gpu, run_gpu_dev
from workloads import make_config, make_dominant, make_random

pytestmark = pytest.mark.gpu

C3_SAMPLE = list(range(0, 128, 8)) + [127]


@pytest.mark.parametrize("l,b,w", [(3, 8, 2), (9, 16, 2), (14, 20, 2), (11, 37, 3), (8, 64, 2),
                                   (6, 100, 2), (10, 5, 4), (7, 128, 2)])
def test_native_ndiagonal(lib, l, b, w):
    wl = make_random(l, b, w, 2, seed=1300 + l * 3 + b + w, eta=1e-3)
    G, T, info = run_gpu(lib, wl)
    assert np.all(info == 0)
    check_fp64(f"nrgf l={l} b={b} w={w}", G, T, range(2), oracle_results("nrgf", wl, range(2)), w, b)


@pytest.mark.parametrize("form", ["native", "fused"])
@pytest.mark.parametrize("l,b,w,m", [(8, 8, 2, 2), (20, 16, 2, 4), (24, 20, 2, 5), (18, 12, 3, 2),
                                     (40, 64, 2, 8), (12, 32, 2, 3)])
def test_ddrgf_ndiagonal(lib, l, b, w, m, form):
    """Both forms of DDRGF with separators of w layers against the oracle's DDRGF (same
    interior layout where l - m w splits into multiples of w) and the dense inverse."""
    wl = make_random(l, b, w, 2, seed=1700 + l + b + w + m, eta=1e-3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=m, ddrgf_form=form)
    assert np.all(info == 0)
    refs = oracle_results("ddrgf", wl, range(2), m=m)
    check_dd(f"ddrgf/{form} l={l} b={b} w={w} m={m}", G, T, range(2), refs, oracle_results("dense", wl, range(2)), w)


@pytest.mark.parametrize("case", ["non_hermitian", "eta_d"])
def test_ddrgf_ndiagonal_native_general_path(lib, case):
    """Native n-diagonal DDRGF on its general interior path: H not Hermitian, or a
    device broadening eta_d > 0 (the Hermitian path needs both), against the oracle's
    DDRGF and the dense inverse."""
    wl = make_random(30, 24, 2, 2, seed=2100, eta=1e-3)
    eta_d = 0.0
    if case == "non_hermitian":
        rng = np.random.default_rng(7)
        wl.H[3, :29] += 0.05 * (rng.standard_normal((29, 24, 24)) + 1j * rng.standard_normal((29, 24, 24)))
        wl.H[0, 9, 2, 3] += 0.1
    else:
        eta_d = 0.02
    wl.eta_d = eta_d
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=4)
    assert np.all(info == 0)
    refs = oracle_results("ddrgf", wl, range(2), m=4)
    check_dd(f"ddrgf/native general ({case})", G, T, range(2), refs, oracle_results("dense", wl, range(2)), 2)


@pytest.mark.parametrize("l,b,w,m", [(16, 100, 2, 3), (21, 128, 2, 2), (26, 40, 4, 3), (17, 7, 3, 2),
                                     (9, 16, 2, 2), (45, 33, 2, 7), (100, 8, 2, 2), (160, 4, 3, 3),
                                     (6, 8, 2, 1), (8, 12, 2, 2), (9, 5, 4, 1)])
def test_ddrgf_ndiagonal_native_only(lib, l, b, w, m):
    """Native n-diagonal DDRGF where the super-block form cannot run (w b > 128 or l
    not a multiple of w), with ragged interiors, interiors of tens of layers (where
    an unstable Hermitian shortcut would show), interiors of exactly w layers and a
    single pair (reduced system of w layers, narrower than its band), against the
    oracle's DDRGF (same layout) and the dense inverse."""
    wl = make_random(l, b, w, 2, seed=1900 + l + b + w + m, eta=1e-3)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=m)
    assert np.all(info == 0)
    refs = oracle_results("ddrgf", wl, range(2), m=m)
    check_dd(f"ddrgf/native l={l} b={b} w={w} m={m}", G, T, range(2), refs,
             oracle_results("dense", wl, range(2)), w)


def test_config3_sequential(lib):
    """Block pentadiagonal, 512 layers x 64, 128 energies, native n-diagonal sweep;
    17 energies spread over the grid against the oracle."""
    wl = make_config(3)
    G, T, info = run_gpu_dev(lib, wl)
    assert bool((info == 0).all())
    refs = oracle_results("nrgf", ("config", 3), C3_SAMPLE)
    check_fp64("config3 nrgf", G, T.cpu().numpy(), C3_SAMPLE, refs, 2, wl.b)
    del G
    free_gpu()


def test_config3_ddrgf(lib):
    """Same system, DDRGF with 16 domains (separators of 2 layers; the reduced system
    is block tridiagonal in 2-layer groups), the same 17 energies against the
    oracle's DDRGF."""
    wl = make_config(3)
    G, T, info = run_gpu_dev(lib, wl, method="ddrgf", domains=16)
    assert bool((info == 0).all())
    refs = oracle_results("ddrgf", ("config", 3), C3_SAMPLE, m=16)
    exact = oracle_results("nrgf", ("config", 3), C3_SAMPLE)
    check_dd("config3 ddrgf", G, T.cpu().numpy(), C3_SAMPLE, refs, exact, 2)
    del G
    free_gpu()


def test_dominant_pentadiagonal_ddrgf(lib):
    """512 x 64 block pentadiagonal, block diagonally dominant (the paper's class of
    test matrices), 16 domains: 9 energies spread over the grid within the DDRGF
    rule, here down to the FP64 target, against the oracle's DDRGF and n-RGF."""
    src = ("dominant", 512, 64, 2, 128, 203)
    wl = make_dominant(*src[1:])
    es = list(range(0, 128, 16)) + [127]
    G, T, info = run_gpu_dev(lib, wl, method="ddrgf", domains=16)
    assert bool((info == 0).all())
    refs = oracle_results("ddrgf", src, es, m=16)
    exact = oracle_results("nrgf", src, es)
    rows = check_dd("dominant 512x64 w=2 ddrgf", G, T.cpu().numpy(), es, refs, exact, 2)
    assert max(r[3] for r in rows) <= 1e-9, "the rule should be tight on a well-conditioned system"
    del G
    free_gpu()


def test_config3_distance_to_exact(lib):
    """Energy 127 and the sampled energy with the worst-conditioned pivot: GPU
    sequential sweep, GPU DDRGF and the FP64 oracle against the extended-precision
    reference."""
    wl = make_config(3)
    kap = [r["kappa"] for r in oracle_results("nrgf", ("config", 3), C3_SAMPLE)]
    worst = C3_SAMPLE[int(np.argmax(kap))]
    es = sorted({127, worst})
    kap_of = dict(zip(C3_SAMPLE, kap))
    ext = oracle_results("ext", ("config", 3), es)
    orc = oracle_results("nrgf", ("config", 3), es)
    Gs, Ts, info = run_gpu_dev(lib, wl)
    assert bool((info == 0).all())
    rows = [(e, rel(gpu_energy(Gs, e, 2), x["G"]), rel(o["G"], x["G"]), terr(Ts[e].item(), x["T"]))
            for e, x, o in zip(es, ext, orc)]
    del Gs
    free_gpu()
    Gd, Td, info = run_gpu_dev(lib, wl, method="ddrgf", domains=16)
    for (e, eg, eo, tg), x in zip(rows, ext):
        ed = rel(gpu_energy(Gd, e, 2), x["G"])
        print(f"config3 energy {e}: kappa {kap_of[e]:.2e}  vs exact: GPU sweep {eg:.2e} (T {tg:.2e}), "
              f"oracle {eo:.2e}, ratio {eg / max(eo, 1e-300):.2f}; GPU DDRGF {ed:.2e}", flush=True)
        tol = fp64_bound(kap_of[e], wl.b)
        assert eg <= tol and tg <= tol, (e, eg, tg, tol)
    del Gd
    free_gpu()


def test_ddrgf_ndiagonal_native_singular_pivot(lib):
    """Native n-diagonal DDRGF, a closed interior whose last layer is exactly E I - H = 0
    at the first energy: that interior's first pivot is singular, its global layer is
    reported, the energy's band and T are NaN, and the other energy is unaffected."""
    wl = make_random(14, 8, 2, 2, seed=9, eta=1e-3)
    # 2 pairs, w = 2: interiors [0..4], [7..11]; separators [5, 6], [12, 13]
    wl.H[2, 11] = wl.energies[0] * np.eye(8)
    G, T, info = run_gpu(lib, wl, method="ddrgf", domains=2)
    assert info[0] == 12 and info[1] == 0
    assert np.all(np.isnan(G[0])) and np.isnan(T[0])
    refs = oracle_results("ddrgf", wl, [1], m=2)
    check_dd("ddrgf/native singular neighbour", G, T, [1], refs, oracle_results("dense", wl, [1]), 2)
