"""The C-ABI library loads and exports every entry point of include/rgf.h, and its
host-side plan validation behaves as documented (no GPU needed: plan creation
and validation are pure host code)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2605_19910_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return binding


def declared_symbols():
    syms = []
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not name.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", name)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        syms += re.findall(r"^\s*(?:[A-Za-z_][A-Za-z0-9_]*\s+\**)+([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(syms))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("rgf_plan_create", "rgf_plan_destroy", "rgf_solve", "ddrgf_solve", "rgf_batched_plan_create",
              "rgf_batched_solve", "rgf_backward", "rgf_plan_checkpoint_bytes", "rgf_plan_set_timing",
              "rgf_plan_kernel_times"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    b = _lib()
    lib = ctypes.CDLL(b.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_version_and_status_strings():
    lib = _lib().load()
    assert lib.rgf_version() >= 100
    assert lib.rgf_status_string(0) == b"ok"
    assert lib.rgf_status_string(4).startswith(b"workspace")


@pytest.mark.parametrize("l,b,w,ne", [(16, 16, 1, 4), (256, 128, 1, 64), (1, 5, 1, 1), (7, 37, 1, 3)])
def test_plan_workspace_size(l, b, w, ne):
    binding = _lib()
    p = binding.Plan(l, b, w, ne)
    bp = ((b + 15) // 16) * 16
    sweep = (3 * l + 10) * bp * bp * 16 * ne
    # plus one 64-byte group counter per energy for the split sweep, 256-byte aligned
    assert p.workspace_bytes == (sweep + 255) // 256 * 256 + 64 * ne
    p.close()


@pytest.mark.parametrize("args,code", [
    (dict(l=0, b=4, w=1, ne=1), 1),
    (dict(l=4, b=0, w=1, ne=1), 1),
    (dict(l=4, b=4, w=1, ne=0), 1),
    (dict(l=4, b=129, w=1, ne=1), 2),
    (dict(l=4, b=4, w=4, ne=1), 1),
    (dict(l=4, b=4, w=1, ne=1, precision="bf16x3"), 2),
    (dict(l=8, b=4, w=2, ne=1, precision="fp32"), 2),
    (dict(l=8, b=4, w=1, ne=1, method="ddrgf", domains=2, precision="fp32"), 2),
    (dict(l=9, b=4, w=2, ne=1, method="ddrgf", domains=2, ddrgf_form="fused"), 2),
    (dict(l=8, b=80, w=2, ne=1, method="ddrgf", domains=2, ddrgf_form="fused"), 2),
    (dict(l=7, b=4, w=2, ne=1, method="ddrgf", domains=2), 1),
    (dict(l=32, b=4, w=2, ne=1, method="ddrgf", domains=4, inner_domains=2), 2),
    (dict(l=8, b=4, w=1, ne=1, method="ddrgf", domains=2, ddrgf_form="fused"), 1),
    (dict(l=8, b=4, w=2, ne=1, ddrgf_form="fused"), 1),
    (dict(l=8, b=4, w=1, ne=1, method="ddrgf", domains=5), 1),
    (dict(l=8, b=4, w=1, ne=1, method="ddrgf", domains=2, want_backward=True), 2),
    (dict(l=8, b=4, w=1, ne=1, precision="fp32", want_backward=True), 2),
    (dict(l=8, b=4, w=1, ne=1, precision="fp32", mixed_tolerance=-1.0), 1),
    (dict(l=8, b=4, w=1, ne=1, inner_domains=1), 1),
    (dict(l=16, b=4, w=1, ne=1, method="ddrgf", domains=4, inner_domains=3), 1),
    (dict(l=16, b=4, w=1, ne=1, method="ddrgf", domains=4, inner_domains=-1), 1),
])
def test_plan_validation_errors(args, code):
    binding = _lib()
    with pytest.raises(binding.RgfError) as ei:
        binding.Plan(**args)
    assert ei.value.code == code


def test_solve_rejects_null_and_small_workspace():
    binding = _lib()
    lib = binding.load()
    p = binding.Plan(4, 4, 1, 1)
    V = ctypes.c_void_p
    # null inputs: rejected synchronously before any GPU work
    assert lib.rgf_solve(p.handle, None, None, None, None, 0.0, None, None, None, None, 0, None) == 1
    fake = V(16)
    assert lib.rgf_solve(p.handle, fake, fake, fake, fake, 0.0, fake, None, fake, fake, 1, None) == 4
    # a sequential plan used with the DDRGF entry point
    assert lib.ddrgf_solve(p.handle, fake, fake, fake, fake, 0.0, fake, None, fake, fake, 1 << 40, None) == 6
    p.close()


def test_backward_plan_workspace_and_mismatch():
    """The adjoint's plan: checkpoints (4 nd + 1 blocks per energy) at the front of the
    workspace, then scratch large enough for the forward sweep and for the adjoint;
    argument and plan errors are rejected on the host."""
    binding = _lib()
    lib = binding.load()
    l, b, ne, nd = 256, 64, 4, 8
    p = binding.Plan(l, b, 1, ne, want_backward=True, checkpoint_domains=nd)
    pb = binding.Plan(l, b, 1, ne, want_backward=binding.BACKWARD_BAND, checkpoint_domains=nd)
    plain = binding.Plan(l, b, 1, ne)
    bpbp = b * b
    ck = (4 * nd + 1) * bpbp * 16 * ne
    assert p.checkpoint_bytes == ck and plain.checkpoint_bytes == 0
    assert p.workspace_bytes >= ck + plain.workspace_bytes
    # the band gradient's per-chunk partial sums (min(nE, 64) chunks of a band of H)
    assert pb.workspace_bytes >= ck + ne * 3 * l * bpbp * 16
    f = ctypes.c_void_p(16)
    big = 1 << 44
    # a plan without want_backward cannot run the adjoint
    assert lib.rgf_backward(plain.handle, f, f, f, f, 0.0, f, 0, f, None, f, f, big, None) == 6
    # a band gradient needs a plan made for it
    assert lib.rgf_backward(p.handle, f, f, f, f, 0.0, f, 0, f, f, None, f, big, None) == 6
    # missing inputs, no output at all, negative stride, small workspace
    assert lib.rgf_backward(p.handle, None, f, f, f, 0.0, f, 0, f, None, f, f, big, None) == 1
    assert lib.rgf_backward(p.handle, f, f, f, f, 0.0, f, 0, f, None, None, f, big, None) == 1
    assert lib.rgf_backward(p.handle, f, f, f, f, 0.0, f, -1, f, None, f, f, big, None) == 1
    assert lib.rgf_backward(p.handle, f, f, f, f, 0.0, f, 0, f, None, f, f, 16, None) == 4
    with pytest.raises(binding.RgfError):
        binding.Plan(8, 4, 1, 1, want_backward=4)


def test_lesser_and_lead_argument_errors():
    """Host-side checks of the lesser and lead entry points (no HIP call is made)."""
    binding = _lib()
    lib = binding.load()
    size = ctypes.c_size_t(0)
    assert lib.rgf_lead_workspace_bytes(16, 3, ctypes.byref(size)) == 0
    assert size.value == 8 * 16 * 16 * 16 * 3
    assert lib.rgf_lead_workspace_bytes(0, 3, ctypes.byref(size)) == 1
    assert lib.rgf_lead_workspace_bytes(129, 3, ctypes.byref(size)) == 2
    assert lib.rgf_lead_workspace_bytes(16, 3, None) == 1
    dummy = ctypes.c_void_p(16)
    # null pointers, bad tolerance / steps / eta, small workspace
    assert lib.rgf_lead_self_energy(4, 1, None, dummy, dummy, dummy, 1e-3, 1e-14, 10, dummy, dummy, dummy, 1 << 20,
                                    None) == 1
    assert lib.rgf_lead_self_energy(4, 1, dummy, dummy, dummy, dummy, 1e-3, 0.0, 10, dummy, dummy, dummy, 1 << 20,
                                    None) == 1
    assert lib.rgf_lead_self_energy(4, 1, dummy, dummy, dummy, dummy, 1e-3, 1e-14, 0, dummy, dummy, dummy, 1 << 20,
                                    None) == 1
    assert lib.rgf_lead_self_energy(4, 1, dummy, dummy, dummy, dummy, -1.0, 1e-14, 10, dummy, dummy, dummy, 1 << 20,
                                    None) == 1
    assert lib.rgf_lead_self_energy(4, 1, dummy, dummy, dummy, dummy, 1e-3, 1e-14, 10, dummy, dummy, dummy, 16,
                                    None) == 4
    # lesser: DDRGF plan -> plan mismatch; mixed / backward plans -> unsupported; null occupations
    f = [dummy] * 4
    p = binding.Plan(8, 4, 1, 1, method="ddrgf", domains=2)
    assert lib.rgf_solve_lesser(p.handle, *f, 0.0, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 1 << 20,
                                None) == 6
    p.close()
    for kw in (dict(precision="fp32"), dict(want_backward=True)):
        p = binding.Plan(8, 4, 1, 1, **kw)
        assert lib.rgf_solve_lesser(p.handle, *f, 0.0, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 1 << 20,
                                    None) == 2
        p.close()
    p = binding.Plan(8, 4, 1, 1)
    assert lib.rgf_solve_lesser(p.handle, *f, 0.0, None, dummy, dummy, dummy, dummy, dummy, dummy, 1 << 20,
                                None) == 1
    p.close()


def test_split_arguments():
    """Workgroups per energy: 0, 1, 2, 4 accepted, anything else and negative spin
    limits rejected on the host; before any solve the plan reports 1."""
    binding = _lib()
    lib = binding.load()
    p = binding.Plan(8, 64, 1, 2)
    for k in (0, 1, 2, 4):
        assert lib.rgf_plan_set_split(p.handle, k, 0) == 0
    for k in (-1, 3, 5, 8):
        assert lib.rgf_plan_set_split(p.handle, k, 0) == 1
    assert lib.rgf_plan_set_split(p.handle, 0, -5) == 1
    assert lib.rgf_plan_set_split(None, 0, 0) == 1
    assert p.split_workgroups() == 1
    assert lib.rgf_plan_split_workgroups(p.handle, None) == 1
    p.close()


def test_timing_argument_errors():
    """Timing queries on a plan without timing, and a pool too small to hold a
    start and an end mark, are rejected on the host (no HIP call is made)."""
    binding = _lib()
    lib = binding.load()
    p = binding.Plan(4, 4, 1, 1)
    n = ctypes.c_int32(-1)
    out = (binding.KernelTime * 4)()
    assert lib.rgf_plan_kernel_times(p.handle, out, 4, ctypes.byref(n), None) == 1
    assert lib.rgf_plan_kernel_times(None, out, 4, ctypes.byref(n), None) == 1
    assert lib.rgf_plan_set_timing(p.handle, 1, 1) == 1
    assert lib.rgf_plan_set_timing(None, 1, 16) == 1
    assert lib.rgf_plan_set_timing(p.handle, 0, 0) == 0     # disabling is always fine
    with pytest.raises(binding.RgfError):
        p.kernel_times()
    p.close()


@pytest.mark.parametrize("l,b,w,m,ne", [(9, 4, 2, 2, 3), (40, 64, 2, 8, 2), (26, 100, 3, 3, 1), (33, 128, 4, 2, 2)])
def test_native_ndiagonal_ddrgf_workspace(l, b, w, m, ne):
    """Native n-diagonal DDRGF plans (no l % w or w b <= 128 condition): interiors of
    (2w^2 + 8w + 2) nmax + 2w blocks each, reduced band and inverse (half bandwidth
    2w - 1 over m w layers), w last-column rows, the reduced sweep, scratch, status."""
    binding = _lib()
    p = binding.Plan(l, b, w, ne, method="ddrgf", domains=m)
    bp = (b + 15) // 16 * 16
    B = bp * bp * 16
    al = lambda x: (x + 255) // 256 * 256
    nmax = (l - m * w) // m + 1
    lr, wr = m * w, 2 * w - 1
    chain = ((2 * w * w + 8 * w + 2) * nmax + 2 * w) * B
    red_chain = ((4 * wr + 3) * lr + 3 + (w - 1) * lr) * B
    band = (2 * wr + 1) * lr * b * b * 16 * ne
    want = (al(chain * ne * m) + 2 * al(band) + al(ne * w * b * b * 16) + al(red_chain * ne)
            + al(ne * 4 * B) + al(ne * m * 4) + al(ne * 4) + al(4) + al(64 * ne))
    assert p.workspace_bytes == want
    p.close()


def test_dos_density_argument_errors():
    """Invalid arguments are rejected before any GPU work."""
    lib = _lib().load()
    fake = ctypes.c_void_p(16)
    assert lib.rgf_dos(None, 4, 4, 1, 2, fake, None) == 1
    assert lib.rgf_dos(fake, 0, 4, 1, 2, fake, None) == 1
    assert lib.rgf_dos(fake, 4, 4, 0, 2, fake, None) == 1
    assert lib.rgf_dos(fake, 4, 4, 1, 0, fake, None) == 1
    assert lib.rgf_density(fake, 4, 4, 1, 2, None, fake, None) == 1
    assert lib.rgf_density(fake, 4, 0, 1, 2, fake, fake, None) == 1
    assert lib.rgf_bond_current(fake, fake, 1, 4, 2, fake, None) == 1
    assert lib.rgf_bond_current(None, fake, 4, 4, 2, fake, None) == 1
    assert lib.rgf_bond_current(fake, fake, 4, 4, 0, fake, None) == 1
