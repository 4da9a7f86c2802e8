"""The benchmark's algorithmic flop counts are the paper's operation counts
(eqs. cost_model_RGF and cost_model_general_RGF), taken from the oracle's own
operation counter, at 8/3 b^3 per LU and 8 b^3 per GETRS or GEMM; the first-row
propagation behind T adds c_i products per layer."""
import pytest

import bench
import oracle as O
from workloads import make_random


@pytest.mark.parametrize("l", [2, 5, 9])
def test_rgf_flops_match_counted_ops(l):
    b = 3
    wl = make_random(l, b, 1, 1, seed=2)
    c = O.OpCounter()
    O.rgf(wl.H, wl.energies[0], wl.sigma_L[0], wl.sigma_R[0], counter=c, extras=False)
    counted = (8.0 / 3.0 * c.lu + 8.0 * c.getrs + 8.0 * c.gemm) * b ** 3
    first_row = 8.0 * (l - 1) * b ** 3
    assert bench.rgf_flops_per_energy(l, b) == pytest.approx(counted + first_row, rel=1e-12)


@pytest.mark.parametrize("l,w", [(9, 2), (13, 3), (5, 2), (8, 1)])
def test_nrgf_flops_match_counted_ops(l, w):
    b = 2
    wl = make_random(l, b, w, 1, seed=3)
    Mb = O.block_accessor(wl.H, w, wl.energies[0], wl.sigma_L[0], wl.sigma_R[0])
    c = O.OpCounter()
    O.nrgf(Mb, l, b, w, counter=c)
    counted = (8.0 / 3.0 * c.lu + 8.0 * c.getrs + 8.0 * c.gemm) * b ** 3
    first_row = 8.0 * sum(min(w, i) for i in range(l)) * b ** 3
    assert bench.nrgf_flops_per_energy(l, b, w) == pytest.approx(counted + first_row, rel=1e-12)


@pytest.mark.parametrize("l,m", [(64, 4), (33, 5), (256, 8)])
def test_native_ndiagonal_ddrgf_counts_reduce_to_tridiagonal(l, m):
    """At w = 1 the native n-diagonal DDRGF counts are those of the tridiagonal
    DDRGF kernels (general interiors)."""
    assert bench.nddrgf_interior_flops(l, 16, 1, m, 3) == bench.ddrgf_interior_flops(l, 16, m, 3)
    assert bench.nddrgf_recover_flops(l, 16, 1, m, 3) == bench.ddrgf_recover_flops(l, 16, m, 3)
    # Hermitian path: the general count less the row transfer products (one per layer
    # after the first) on every interior but the first
    base, rem = divmod(l - m, m)
    saved = sum(base + (1 if k < rem else 0) - 1 for k in range(1, m))
    assert bench.nddrgf_interior_flops(l, 16, 1, m, 3, True) == \
        bench.nddrgf_interior_flops(l, 16, 1, m, 3) - 8.0 * 16 ** 3 * saved * 3


def test_hermitian_band_check():
    from workloads import make_random
    wl = make_random(9, 4, 2, 1, seed=5)
    assert bench.is_hermitian_band(wl.H)
    wl.H[0, 4, 1, 2] += 1e-3
    assert not bench.is_hermitian_band(wl.H)
    wl3 = make_random(7, 3, 1, 1, seed=6)
    assert bench.is_hermitian_band(wl3.H)
