"""The allocation-free sequential solve (rgf_solve_noalloc, workspace in the
library's static device array) against rgf_solve with a caller workspace: two
calls in a row, the second on a smaller system, each bitwise equal to rgf_solve
(same kernels on the same inputs) and within the FP64 rule of the oracle; plans
larger than the array and adjoint plans are refused without GPU work."""
import numpy as np
import pytest

from parity import check_fp64, mask_band, oracle_results
from workloads import make_random

pytestmark = pytest.mark.gpu


def test_noalloc_matches_workspace_solve(lib):
    import torch
    from paper_2605_19910_amd import binding
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    for (l, b, ne, seed) in [(24, 48, 3, 61), (9, 16, 2, 62)]:
        wl = make_random(l, b, 1, ne, seed=seed, eta=1e-3)
        H, sL, sR, E = (torch.from_numpy(x).to(dev) for x in (wl.H, wl.sigma_L, wl.sigma_R, wl.energies))
        plan = binding.Plan(l, b, 1, ne)
        assert plan.workspace_bytes <= 64 << 20
        G0, T0, info0 = binding.solve(H, sL, sR, E, plan=plan)
        G = torch.full_like(G0, float("nan"))
        T = torch.full_like(T0, float("nan"))
        info = torch.full_like(info0, 7)
        binding.rgf_solve_noalloc(plan, H, sL, sR, E, 0.0, G, T, info, stream)
        torch.cuda.synchronize()
        assert bool((info == 0).all()) and bool((info0 == 0).all())
        Gh, G0h = mask_band(G.cpu().numpy(), 1), mask_band(G0.cpu().numpy(), 1)
        assert np.array_equal(Gh, G0h) and torch.equal(T, T0)
        check_fp64(f"noalloc l={l} b={b}", Gh, T.cpu().numpy(), range(ne), oracle_results("rgf", wl, range(ne)),
                   1, b)
        plan.close()


def test_noalloc_refuses_large_and_adjoint_plans(lib):
    import ctypes
    from paper_2605_19910_amd import binding
    lib_ = binding.load()
    f = ctypes.c_void_p(16)
    big = binding.Plan(256, 128, 1, 64)                 # 13 GB of workspace
    assert lib_.rgf_solve_noalloc(big.handle, f, f, f, f, 0.0, f, None, f, None) == 4
    adj = binding.Plan(8, 16, 1, 2, want_backward=True)
    assert lib_.rgf_solve_noalloc(adj.handle, f, f, f, f, 0.0, f, None, f, None) == 2
    assert lib_.rgf_solve_noalloc(None, f, f, f, f, 0.0, f, None, f, None) == 1
