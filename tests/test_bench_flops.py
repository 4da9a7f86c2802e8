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
