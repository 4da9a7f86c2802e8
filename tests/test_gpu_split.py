"""Sequential sweep with several workgroups per energy (row slabs of every block
product, the pivot inverse on the first workgroup, bounded group barriers):
bitwise the one-workgroup sweep on every output, at small ragged sizes and on the
full 256 x 128 system over its 64 energies, including a singular pivot; and a
tiny spin limit on the group barriers (forced from the host) makes every energy
report RGF_INFO_SYNC_TIMEOUT while every kernel still ends normally.
"""
import numpy as np
import pytest

from parity import check_fp64, mask_band, oracle_results
from test_gpu_rgf import free_gpu, to_dev
from workloads import make_config, make_random

pytestmark = pytest.mark.gpu

TIMEOUT = 0x20000000


def solve_k(lib, dev_inputs, l, b, ne, k, spin=0, w=1):
    import torch
    H, sL, sR, E = dev_inputs
    plan = lib.Plan(l, b, w, ne)
    plan.set_split(k, spin)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=0.0, plan=plan)
    torch.cuda.synchronize()
    used = plan.split_workgroups()
    plan.close()
    return G, T, info, used


def same(lib, a, b, w=1):
    import torch
    Ga, Ta, ia = a[:3]
    Gb, Tb, ib = b[:3]
    return (np.array_equal(mask_band(Ga.cpu().numpy(), w), mask_band(Gb.cpu().numpy(), w))
            and torch.equal(Ta, Tb) and torch.equal(ia, ib))


@pytest.mark.parametrize("l,b,ne", [(40, 128, 8), (33, 120, 5), (24, 64, 16), (17, 50, 3), (1, 128, 2),
                                    (2, 64, 3), (9, 100, 9)])
def test_split_bitwise_equal(lib, l, b, ne):
    wl = make_random(l, b, 1, ne, seed=3100 + l + b, eta=1e-3)
    d = to_dev(wl)
    ref = solve_k(lib, d, l, b, ne, 1)
    assert ref[3] == 1
    bp = (b + 15) // 16 * 16
    for k in (2, 4):
        out = solve_k(lib, d, l, b, ne, k)
        print(f"split l={l} b={b} ne={ne}: asked {k}, used {out[3]}", flush=True)
        assert out[3] == (k if bp in (64, 128) else 1)
        assert same(lib, out, ref), (l, b, ne, k)
    auto = solve_k(lib, d, l, b, ne, 0)
    assert same(lib, auto, ref)
    # and the split result against the oracle
    G, T, info = auto[:3]
    assert bool((info == 0).all())
    check_fp64(f"split l={l} b={b}", G.cpu().numpy(), T.cpu().numpy(), range(min(ne, 3)),
               oracle_results("rgf", wl, range(min(ne, 3))), 1, b)


@pytest.mark.parametrize("l,b,w,ne", [(20, 64, 2, 6), (33, 120, 2, 3), (17, 50, 3, 5), (4, 128, 3, 2)])
def test_split_ndiagonal_bitwise_equal(lib, l, b, w, ne):
    """The n-diagonal sweep with 2 and 4 workgroups per energy: bitwise the
    one-workgroup sweep, and within the FP64 rule of the oracle."""
    from parity import oracle_results as orc
    wl = make_random(l, b, w, ne, seed=3500 + l + b + w, eta=1e-3)
    d = to_dev(wl)
    ref = solve_k(lib, d, l, b, ne, 1, w=w)
    for k in (2, 4):
        out = solve_k(lib, d, l, b, ne, k, w=w)
        print(f"n-diagonal split l={l} b={b} w={w} ne={ne}: asked {k}, used {out[3]}", flush=True)
        assert out[3] == k
        assert same(lib, out, ref, w), (l, b, w, k)
    G, T, info = ref[:3]
    assert bool((info == 0).all())
    check_fp64(f"n-diagonal split l={l} b={b} w={w}", G.cpu().numpy(), T.cpu().numpy(), range(min(ne, 2)),
               orc("nrgf", wl, range(min(ne, 2))), w, b)


def test_split_config3_all_energies(lib):
    """The pentadiagonal 512 x 64 system over its 128 energies: several workgroups per
    energy give bitwise the one-workgroup results."""
    import torch
    wl = make_config(3)
    d = to_dev(wl)
    ref = solve_k(lib, d, wl.l, wl.b, wl.ne, 1, w=2)
    out = solve_k(lib, d, wl.l, wl.b, wl.ne, 0, w=2)
    print(f"config3: {out[3]} workgroups per energy", flush=True)
    assert out[3] in (2, 4)
    for G in (out[0], ref[0]):
        for kk in range(-2, 3):
            if kk < 0:
                G[:, 2 + kk, :(-kk)] = 0
            elif kk > 0:
                G[:, 2 + kk, wl.l - kk:] = 0
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]) and torch.equal(out[2], ref[2])
    del out, ref
    free_gpu()


def test_split_singular_pivot(lib):
    """Sigma_R = 0 and H_{l-1,l-1} = E I at energy 1: the first Schur pivot is exactly
    zero; same info and NaN outputs as one workgroup, the other energies bitwise."""
    wl = make_random(12, 64, 1, 3, seed=5, eta=1e-3)
    wl.sigma_R[1] = 0.0
    wl.H[1, 11] = wl.energies[1] * np.eye(64)
    d = to_dev(wl)
    ref = solve_k(lib, d, 12, 64, 3, 1)
    out = solve_k(lib, d, 12, 64, 3, 4)
    assert out[3] == 4
    info = out[2].cpu().numpy()
    assert info[1] == 12 and info[0] == 0 and info[2] == 0
    assert np.array_equal(info, ref[2].cpu().numpy())
    assert np.all(np.isnan(out[0][1].cpu().numpy())) and np.isnan(out[1][1].item())
    keep = [0, 2]
    assert np.array_equal(mask_band(out[0][keep].cpu().numpy(), 1), mask_band(ref[0][keep].cpu().numpy(), 1))


def test_split_config2_all_energies(lib):
    """The 256 x 128 system over all 64 energies: 4 workgroups per energy fill the
    device and give bitwise the one-workgroup results."""
    import torch
    wl = make_config(2)
    d = to_dev(wl)
    ref = solve_k(lib, d, wl.l, wl.b, wl.ne, 1)
    out = solve_k(lib, d, wl.l, wl.b, wl.ne, 0)
    print(f"config2: {out[3]} workgroups per energy", flush=True)
    assert out[3] == 4
    for G in (out[0], ref[0]):
        # blocks outside the matrix are never written
        G[:, 0, 0] = 0
        G[:, 2, wl.l - 1] = 0
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]) and torch.equal(out[2], ref[2])
    del out, ref
    free_gpu()


def test_split_timeout_reported(lib):
    """Spin limit of one poll: the first workgroups to reach a barrier give up while
    the pivot inverse still runs, so every energy reports RGF_INFO_SYNC_TIMEOUT and
    the launch still ends; the same plan then solves normally with the default
    limit."""
    import torch
    l, b, ne = 10, 128, 4
    wl = make_random(l, b, 1, ne, seed=77, eta=1e-3)
    d = to_dev(wl)
    ref = solve_k(lib, d, l, b, ne, 1)
    H, sL, sR, E = d
    plan = lib.Plan(l, b, 1, ne)
    plan.set_split(4, 1)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=0.0, plan=plan)
    torch.cuda.synchronize()
    assert plan.split_workgroups() == 4
    inf = info.cpu().numpy()
    assert np.all(inf & TIMEOUT), inf
    assert np.all(np.isnan(T.cpu().numpy()))
    plan.set_split(4, 0)
    G, T, info = lib.solve(H, sL, sR, E, eta_d=0.0, plan=plan)
    torch.cuda.synchronize()
    assert same(lib, (G, T, info), ref)
    plan.close()


def test_split_not_used_for_other_plans(lib):
    """Mixed precision and adjoint checkpoints keep one workgroup per energy."""
    import torch
    wl = make_random(8, 64, 1, 2, seed=9, eta=1e-3)
    H, sL, sR, E = to_dev(wl)
    for kw in (dict(precision="fp32"), dict(want_backward=True)):
        plan = lib.Plan(8, 64, 1, 2, **kw)
        plan.set_split(4, 0)
        lib.solve(H, sL, sR, E, eta_d=0.0, plan=plan)
        torch.cuda.synchronize()
        assert plan.split_workgroups() == 1, kw
        plan.close()
