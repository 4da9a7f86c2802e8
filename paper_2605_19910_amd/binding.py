"""Thin ctypes binding of the C ABI in include/rgf.h (argument marshalling only).

Names follow the C entry points.  Tensors are torch tensors on the GPU; only their
device pointers cross the boundary.  Every step of the computation runs in the HIP
library: if it is missing, loading fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "librgf.so")

RGF_OK = 0
BACKWARD_ONSITE = 1                 # want_backward flags (RGF_BACKWARD_ONSITE / _BAND)
BACKWARD_BAND = 2
INFO_FP64_PRODUCTS = 0x40000000     # RGF_INFO_FP64_PRODUCTS: a mixed solve recomputed the energy in FP64
INFO_STATUS_MASK = 0x3fffffff
INFO_SYNC_TIMEOUT = 0x20000000
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported configuration", 3: "out of host memory",
          4: "workspace missing or too small", 5: "HIP runtime error",
          6: "plan does not match the entry point"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2}
METHOD = {"rgf": 0, "sequential": 0, "ddrgf": 1}
DDRGF_FORM = {"native": 0, "fused": 1}


class RgfDesc(ctypes.Structure):
    _fields_ = [
        ("num_layers", ctypes.c_int64),
        ("block_size", ctypes.c_int64),
        ("half_bandwidth", ctypes.c_int64),
        ("num_energies", ctypes.c_int64),
        ("precision", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("num_domains", ctypes.c_int64),
        ("separator_layers", ctypes.c_int64),
        ("want_transmission", ctypes.c_int32),
        ("want_backward", ctypes.c_int32),
        ("checkpoint_domains", ctypes.c_int64),
        ("mixed_tolerance", ctypes.c_double),
        ("inner_domains", ctypes.c_int64),
        ("ddrgf_form", ctypes.c_int64),
    ]


class BatchShape(ctypes.Structure):
    _fields_ = [("num_layers", ctypes.c_int64), ("block_size", ctypes.c_int64),
                ("num_energies", ctypes.c_int64)]


# layout of rgf_batch_device_t: seven device pointers and two int32
BATCH_DEVICE_DTYPE = [("H", "<u8"), ("sigma_L", "<u8"), ("sigma_R", "<u8"), ("energies", "<u8"),
                      ("G_diag", "<u8"), ("T", "<u8"), ("info", "<u8"), ("num_layers", "<i4"),
                      ("block_size", "<i4")]
SCHEDULE = {"longest_first": 0, "input_order": 1, "interleaved": 2}


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("total_ms", ctypes.c_double), ("launches", ctypes.c_int64)]


class RgfError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn}: {STATUS.get(code, 'unknown status')} (code {code})")
        self.code = code


_lib = None

_VP = ctypes.c_void_p
_SOLVE_ARGS = [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]


def load() -> ctypes.CDLL:
    """Load the built library (build it first with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.rgf_plan_create.argtypes = [ctypes.POINTER(RgfDesc), ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_size_t)]
    lib.rgf_plan_create.restype = ctypes.c_int
    lib.rgf_plan_destroy.argtypes = [_VP]
    lib.rgf_plan_destroy.restype = ctypes.c_int
    for fn in ("rgf_solve", "ddrgf_solve"):
        f = getattr(lib, fn)
        f.argtypes = list(_SOLVE_ARGS)
        f.restype = ctypes.c_int
    lib.rgf_batched_plan_create.argtypes = [ctypes.c_int64, ctypes.POINTER(BatchShape), ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_VP),
                                            ctypes.POINTER(ctypes.c_size_t)]
    lib.rgf_batched_plan_create.restype = ctypes.c_int
    lib.rgf_batched_solve.argtypes = [_VP, _VP, ctypes.c_double, _VP, ctypes.c_size_t, _VP]
    lib.rgf_batched_solve.restype = ctypes.c_int
    lib.rgf_backward.argtypes = [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP, ctypes.c_int64, _VP, _VP, _VP,
                                 _VP, ctypes.c_size_t, _VP]
    lib.rgf_backward.restype = ctypes.c_int
    lib.rgf_plan_checkpoint_bytes.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
    lib.rgf_plan_checkpoint_bytes.restype = ctypes.c_int
    lib.rgf_plan_workspace_bytes.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
    lib.rgf_plan_workspace_bytes.restype = ctypes.c_int
    lib.rgf_solve_noalloc.argtypes = [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP]
    lib.rgf_solve_noalloc.restype = ctypes.c_int
    lib.rgf_solve_lesser.argtypes = [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                     ctypes.c_size_t, _VP]
    lib.rgf_solve_lesser.restype = ctypes.c_int
    lib.rgf_lead_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    lib.rgf_lead_workspace_bytes.restype = ctypes.c_int
    lib.rgf_lead_self_energy.argtypes = [ctypes.c_int64, ctypes.c_int64, _VP, _VP, _VP, _VP, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t, _VP]
    lib.rgf_lead_self_energy.restype = ctypes.c_int
    lib.rgf_dos.argtypes = [_VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _VP, _VP]
    lib.rgf_dos.restype = ctypes.c_int
    lib.rgf_density.argtypes = [_VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _VP, _VP, _VP]
    lib.rgf_density.restype = ctypes.c_int
    lib.rgf_bond_current.argtypes = [_VP, _VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _VP, _VP]
    lib.rgf_bond_current.restype = ctypes.c_int
    lib.rgf_plan_set_split.argtypes = [_VP, ctypes.c_int32, ctypes.c_int64]
    lib.rgf_plan_set_split.restype = ctypes.c_int
    lib.rgf_plan_split_workgroups.argtypes = [_VP, ctypes.POINTER(ctypes.c_int32)]
    lib.rgf_plan_split_workgroups.restype = ctypes.c_int
    lib.rgf_plan_set_timing.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32]
    lib.rgf_plan_set_timing.restype = ctypes.c_int
    lib.rgf_plan_kernel_times.argtypes = [_VP, ctypes.POINTER(KernelTime), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.rgf_plan_kernel_times.restype = ctypes.c_int
    lib.rgf_status_string.argtypes = [ctypes.c_int]
    lib.rgf_status_string.restype = ctypes.c_char_p
    lib.rgf_version.argtypes = []
    lib.rgf_version.restype = ctypes.c_int
    _lib = lib
    return lib


class Plan:
    """Owning wrapper of an rgf_plan_t."""

    def __init__(self, l: int, b: int, w: int, ne: int, method: str = "rgf", precision: str = "fp64",
                 domains: int = 0, separator_layers: int = 0, want_transmission: bool = True,
                 want_backward: bool = False, checkpoint_domains: int = 0, mixed_tolerance: float = 0.0,
                 inner_domains: int = 0, ddrgf_form: str = "native"):
        self.lib = load()
        wb = int(want_backward) if not isinstance(want_backward, bool) else (BACKWARD_ONSITE if want_backward else 0)
        self.desc = RgfDesc(l, b, w, ne, PRECISION[precision], METHOD[method], domains,
                            separator_layers, 1 if want_transmission else 0, wb,
                            checkpoint_domains, float(mixed_tolerance), int(inner_domains),
                            DDRGF_FORM[ddrgf_form])
        self.handle = _VP()
        ws = ctypes.c_size_t(0)
        st = self.lib.rgf_plan_create(ctypes.byref(self.desc), ctypes.byref(self.handle), ctypes.byref(ws))
        if st != RGF_OK:
            raise RgfError("rgf_plan_create", st)
        self.workspace_bytes = int(ws.value)
        ck = ctypes.c_size_t(0)
        st = self.lib.rgf_plan_checkpoint_bytes(self.handle, ctypes.byref(ck))
        if st != RGF_OK:
            raise RgfError("rgf_plan_checkpoint_bytes", st)
        self.checkpoint_bytes = int(ck.value)
        self.method = method
        self.l, self.b, self.w, self.ne = l, b, w, ne

    def set_split(self, workgroups_per_energy: int = 0, spin_limit: int = 0) -> None:
        """Workgroups per energy of the sequential sweep (0 = automatic, 1 = off, 2, 4)."""
        st = self.lib.rgf_plan_set_split(self.handle, int(workgroups_per_energy), int(spin_limit))
        if st != RGF_OK:
            raise RgfError("rgf_plan_set_split", st)

    def split_workgroups(self) -> int:
        """Workgroups per energy used by the last rgf_solve."""
        k = ctypes.c_int32(0)
        st = self.lib.rgf_plan_split_workgroups(self.handle, ctypes.byref(k))
        if st != RGF_OK:
            raise RgfError("rgf_plan_split_workgroups", st)
        return int(k.value)

    def set_timing(self, enable: bool = True, max_marks: int = 256) -> None:
        """Record a HIP event after every kernel this plan's solves launch."""
        st = self.lib.rgf_plan_set_timing(self.handle, 1 if enable else 0, int(max_marks) if enable else 0)
        if st != RGF_OK:
            raise RgfError("rgf_plan_set_timing", st)

    def kernel_times(self, max_entries: int = 32) -> dict:
        """{kernel name: (total ms, launches)} since the previous call (blocks the host)."""
        out = (KernelTime * max_entries)()
        n = ctypes.c_int32(0)
        dropped = ctypes.c_int32(0)
        st = self.lib.rgf_plan_kernel_times(self.handle, out, max_entries, ctypes.byref(n), ctypes.byref(dropped))
        if st != RGF_OK:
            raise RgfError("rgf_plan_kernel_times", st)
        if dropped.value:
            raise RuntimeError(f"{dropped.value} timing marks dropped: enlarge max_marks")
        return {out[i].name.decode(): (out[i].total_ms, int(out[i].launches)) for i in range(min(n.value, max_entries))}

    def close(self):
        if self.handle:
            self.lib.rgf_plan_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def rgf_solve(plan: Plan, H, sigma_L, sigma_R, energies, eta_d: float, G, T, info, workspace,
              stream: int = 0) -> None:
    st = plan.lib.rgf_solve(plan.handle, _ptr(H), _ptr(sigma_L), _ptr(sigma_R), _ptr(energies),
                            float(eta_d), _ptr(G), _ptr(T), _ptr(info), _ptr(workspace),
                            workspace.numel() * workspace.element_size() if workspace is not None else 0,
                            stream)
    if st != RGF_OK:
        raise RgfError("rgf_solve", st)


def rgf_solve_noalloc(plan: Plan, H, sigma_L, sigma_R, energies, eta_d: float, G, T, info, stream: int = 0) -> None:
    """rgf_solve with the library's static device workspace (allocates nothing)."""
    st = plan.lib.rgf_solve_noalloc(plan.handle, _ptr(H), _ptr(sigma_L), _ptr(sigma_R), _ptr(energies),
                                    float(eta_d), _ptr(G), _ptr(T), _ptr(info), stream)
    if st != RGF_OK:
        raise RgfError("rgf_solve_noalloc", st)


def rgf_solve_lesser(plan: Plan, H, sigma_L, sigma_R, energies, eta_d: float, occupation_L, occupation_R, G,
                     G_lesser, T, info, workspace, stream: int = 0) -> None:
    st = plan.lib.rgf_solve_lesser(plan.handle, _ptr(H), _ptr(sigma_L), _ptr(sigma_R), _ptr(energies), float(eta_d),
                                   _ptr(occupation_L), _ptr(occupation_R), _ptr(G), _ptr(G_lesser), _ptr(T),
                                   _ptr(info), _ptr(workspace), workspace.numel() * workspace.element_size(), stream)
    if st != RGF_OK:
        raise RgfError("rgf_solve_lesser", st)


def solve_lesser(H, sigma_L, sigma_R, energies, occupation_L, occupation_R, eta_d: float = 0.0,
                 plan: Optional[Plan] = None) -> Tuple:
    """Allocate outputs and run rgf_solve_lesser on the current stream.  Returns
    (G [nE, 2w+1, l, b, b], G_lesser [nE, 2w+1, l, b, b], T [nE], info [nE])."""
    import torch
    nb, l, b, _ = H.shape
    w = (nb - 1) // 2
    ne = energies.shape[0]
    if plan is None:
        plan = Plan(l, b, w, ne)
    dev = H.device
    G = torch.empty((ne, nb, l, b, b), dtype=torch.complex128, device=dev)
    Gl = torch.empty_like(G)
    T = torch.empty((ne,), dtype=torch.float64, device=dev)
    info = torch.empty((ne,), dtype=torch.int32, device=dev)
    ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=dev)
    for t, name in ((occupation_L, "occupation_L"), (occupation_R, "occupation_R")):
        if t.dtype != torch.float64 or not t.is_cuda or t.shape[0] != ne:
            raise ValueError(f"{name} must be a float64 GPU tensor of one value per energy")
    rgf_solve_lesser(plan, H, sigma_L, sigma_R, energies, eta_d, occupation_L, occupation_R, G, Gl, T, info, ws,
                     torch.cuda.current_stream(dev).cuda_stream)
    return G, Gl, T, info


def lead_self_energy(H00, H01, Hc, energies, eta: float, tolerance: float = 1e-14, max_steps: int = 100,
                     stream: Optional[int] = None) -> Tuple:
    """Retarded self-energies of a semi-infinite lead at every energy (rgf_lead_self_energy).
    H00, H01, Hc: complex128 [b, b] GPU tensors; energies: float64 [nE].
    Returns (sigma [nE, b, b], steps [nE])."""
    import torch
    lib = load()
    b = H00.shape[0]
    ne = energies.shape[0]
    for t, name in ((H00, "H00"), (H01, "H01"), (Hc, "Hc")):
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (b, b):
            raise ValueError(f"{name} must be a contiguous complex128 [b, b] GPU tensor")
    if energies.dtype != torch.float64 or not energies.is_cuda:
        raise ValueError("energies must be a float64 GPU tensor")
    ws_bytes = ctypes.c_size_t(0)
    st = lib.rgf_lead_workspace_bytes(b, ne, ctypes.byref(ws_bytes))
    if st != RGF_OK:
        raise RgfError("rgf_lead_workspace_bytes", st)
    dev = H00.device
    sigma = torch.empty((ne, b, b), dtype=torch.complex128, device=dev)
    steps = torch.empty((ne,), dtype=torch.int32, device=dev)
    ws = torch.empty((int(ws_bytes.value),), dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream(dev).cuda_stream if stream is None else stream
    st = lib.rgf_lead_self_energy(b, ne, _ptr(H00), _ptr(H01), _ptr(Hc), _ptr(energies), float(eta), float(tolerance),
                                  int(max_steps), _ptr(sigma), _ptr(steps), _ptr(ws), int(ws_bytes.value), s)
    if st != RGF_OK:
        raise RgfError("rgf_lead_self_energy", st)
    return sigma, steps


def dos(G, stream: Optional[int] = None):
    """Orbital-resolved density of states -(1/pi) Im G^R_{ii,ss} of every energy
    (rgf_dos).  G: complex128 band [nE, 2w+1, l, b, b] on the GPU; returns [nE, l b]."""
    import torch
    lib = load()
    ne, nb, l, b, _ = G.shape
    if G.dtype != torch.complex128 or not G.is_cuda or not G.is_contiguous():
        raise ValueError("G must be a contiguous complex128 GPU tensor")
    out = torch.empty((ne, l * b), dtype=torch.float64, device=G.device)
    st = lib.rgf_dos(_ptr(G), l, b, (nb - 1) // 2, ne, _ptr(out),
                     torch.cuda.current_stream(G.device).cuda_stream if stream is None else stream)
    if st != RGF_OK:
        raise RgfError("rgf_dos", st)
    return out


def density(G_lesser, weights, stream: Optional[int] = None):
    """Orbital-resolved electron density sum_e weights[e] Im G^<_{ii,ss}(E_e) / 2pi
    (rgf_density).  G_lesser: complex128 band [nE, 2w+1, l, b, b] on the GPU; weights:
    float64 [nE] on the GPU; returns [l b]."""
    import torch
    lib = load()
    ne, nb, l, b, _ = G_lesser.shape
    if G_lesser.dtype != torch.complex128 or not G_lesser.is_cuda or not G_lesser.is_contiguous():
        raise ValueError("G_lesser must be a contiguous complex128 GPU tensor")
    if weights.dtype != torch.float64 or not weights.is_cuda or weights.shape[0] != ne:
        raise ValueError("weights must be a float64 GPU tensor of one value per energy")
    out = torch.empty((l * b,), dtype=torch.float64, device=G_lesser.device)
    st = lib.rgf_density(_ptr(G_lesser), l, b, (nb - 1) // 2, ne, _ptr(weights), _ptr(out),
                         torch.cuda.current_stream(G_lesser.device).cuda_stream if stream is None else stream)
    if st != RGF_OK:
        raise RgfError("rgf_density", st)
    return out


def bond_current(H, G_lesser, stream: Optional[int] = None):
    """Spectral particle current through every bond (rgf_bond_current), w = 1.
    H: complex128 band [3, l, b, b]; G_lesser: [nE, 3, l, b, b] (GPU); returns [nE, l-1]."""
    import torch
    lib = load()
    ne, nb, l, b, _ = G_lesser.shape
    for t, name in ((H, "H"), (G_lesser, "G_lesser")):
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex128 GPU tensor")
    if nb != 3 or tuple(H.shape) != (3, l, b, b):
        raise ValueError("block tridiagonal bands of matching shape are required")
    out = torch.empty((ne, l - 1), dtype=torch.float64, device=H.device)
    st = lib.rgf_bond_current(_ptr(H), _ptr(G_lesser), l, b, ne, _ptr(out),
                              torch.cuda.current_stream(H.device).cuda_stream if stream is None else stream)
    if st != RGF_OK:
        raise RgfError("rgf_bond_current", st)
    return out


def rgf_backward(plan: Plan, H, sigma_L, sigma_R, energies, eta_d: float, G_diag, g_diag_stride: int, dL_dT,
                 dH, d_onsite, workspace, stream: int = 0) -> None:
    st = plan.lib.rgf_backward(plan.handle, _ptr(H), _ptr(sigma_L), _ptr(sigma_R), _ptr(energies), float(eta_d),
                               _ptr(G_diag), int(g_diag_stride), _ptr(dL_dT), _ptr(dH), _ptr(d_onsite),
                               _ptr(workspace), workspace.numel() * workspace.element_size(), stream)
    if st != RGF_OK:
        raise RgfError("rgf_backward", st)


def ddrgf_solve(plan: Plan, H, sigma_L, sigma_R, energies, eta_d: float, G, T, info, workspace,
                stream: int = 0) -> None:
    st = plan.lib.ddrgf_solve(plan.handle, _ptr(H), _ptr(sigma_L), _ptr(sigma_R), _ptr(energies),
                              float(eta_d), _ptr(G), _ptr(T), _ptr(info), _ptr(workspace),
                              workspace.numel() * workspace.element_size() if workspace is not None else 0,
                              stream)
    if st != RGF_OK:
        raise RgfError("ddrgf_solve", st)


def solve(H, sigma_L, sigma_R, energies, eta_d: float = 0.0, method: str = "rgf",
          precision: str = "fp64", domains: int = 0, want_transmission: bool = True,
          plan: Optional[Plan] = None, workspace=None, out=None, ddrgf_form: str = "native") -> Tuple:
    """Allocate outputs (torch, on H's device) and run one solve on the current stream.
    method "auto" times the sequential sweep and DDRGF with each admissible domain
    count on these inputs once per workload signature and uses the fastest
    (paper_2605_19910_amd.dispatch).  ddrgf_form: "native" (n-diagonal interiors) or
    "fused" (w-layer super-blocks), for DDRGF with w > 1.

    H: complex128 [2w+1, l, b, b]; sigma_L, sigma_R: complex128 [nE, b, b];
    energies: float64 [nE].  Returns (G [nE, 2w+1, l, b, b], T [nE], info [nE])."""
    import torch
    nb, l, b, _ = H.shape
    w = (nb - 1) // 2
    ne = energies.shape[0]
    for t, name in ((H, "H"), (sigma_L, "sigma_L"), (sigma_R, "sigma_R")):
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex128 GPU tensor")
    if energies.dtype != torch.float64 or not energies.is_cuda:
        raise ValueError("energies must be a float64 GPU tensor")
    if plan is None:
        if method == "auto":
            # measured choice between the sequential sweep and DDRGF, cached per workload
            from . import dispatch
            rec = dispatch.choose(l, b, w, ne, dispatch.gpu_measure(H, sigma_L, sigma_R, energies, eta_d, precision),
                                  precision=precision, device=f"cuda{H.device.index or 0}")
            method, domains, inner = rec["method"], rec["domains"], rec.get("inner_domains", 0)
            if method == "ddrgf_fused":
                method, ddrgf_form = "ddrgf", "fused"
        else:
            inner = 0
        plan = Plan(l, b, w, ne, method=method, precision=precision, domains=domains,
                    want_transmission=want_transmission, inner_domains=inner,
                    ddrgf_form=ddrgf_form if (method == "ddrgf" and w > 1) else "native")
    dev = H.device
    if out is None:
        G = torch.empty((ne, nb, l, b, b), dtype=torch.complex128, device=dev)
        T = torch.empty((ne,), dtype=torch.float64, device=dev)
        info = torch.empty((ne,), dtype=torch.int32, device=dev)
    else:
        G, T, info = out
    if workspace is None:
        workspace = torch.empty((max(plan.workspace_bytes, 1),), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    if plan.method == "ddrgf":
        ddrgf_solve(plan, H, sigma_L, sigma_R, energies, eta_d, G, T, info, workspace, stream)
    else:
        rgf_solve(plan, H, sigma_L, sigma_R, energies, eta_d, G, T, info, workspace, stream)
    return G, T, info


# ----------------------------------------------------------------------------
# Batched launch over devices of uneven size
# ----------------------------------------------------------------------------

class BatchedPlan:
    """Owning wrapper of a batched rgf_plan_t (rgf_batched_plan_create).

    schedule="auto" takes the queue order, grid and waves per workgroup that the
    autotuner stored for this workload (block-size histogram, precision) and the
    defaults (longest first, one workgroup of 8 waves per compute unit) when it has
    not tuned it."""

    def __init__(self, shapes, precision: str = "fp64", schedule: str = "longest_first", grid: int = 0,
                 waves: int = 0):
        self.lib = load()
        if schedule == "auto":
            from . import autotune
            rec = autotune.lookup(shapes, precision)
            schedule, grid, waves = ((rec["schedule"], rec["grid"], rec.get("waves", 8)) if rec
                                     else ("longest_first", 0, 0))
        arr = (BatchShape * len(shapes))(*[BatchShape(int(l), int(b), int(ne)) for (l, b, ne) in shapes])
        self.handle = _VP()
        ws = ctypes.c_size_t(0)
        st = self.lib.rgf_batched_plan_create(len(shapes), arr, PRECISION[precision], SCHEDULE[schedule],
                                              int(grid), int(waves), ctypes.byref(self.handle), ctypes.byref(ws))
        if st != RGF_OK:
            raise RgfError("rgf_batched_plan_create", st)
        self.workspace_bytes = int(ws.value)
        self.shapes = [tuple(int(v) for v in sh) for sh in shapes]
        self.precision, self.schedule, self.grid, self.waves = precision, schedule, grid, waves

    def close(self):
        if self.handle:
            self.lib.rgf_plan_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_table(entries, device):
    """Device array of rgf_batch_device_t from a list of dicts with torch tensors
    H, sigma_L, sigma_R, energies, G_diag, T (or None), info."""
    import numpy as np
    import torch
    rec = np.zeros(len(entries), dtype=BATCH_DEVICE_DTYPE)
    for k, d in enumerate(entries):
        rec[k] = (d["H"].data_ptr(), d["sigma_L"].data_ptr(), d["sigma_R"].data_ptr(),
                  d["energies"].data_ptr(), d["G_diag"].data_ptr(),
                  0 if d.get("T") is None else d["T"].data_ptr(), d["info"].data_ptr(),
                  d["H"].shape[1], d["H"].shape[2])
    return torch.from_numpy(rec.view(np.uint8).copy()).to(device)


def rgf_batched_solve(plan: BatchedPlan, table, eta_d: float, workspace, stream: int = 0) -> None:
    st = plan.lib.rgf_batched_solve(plan.handle, table.data_ptr(), float(eta_d), workspace.data_ptr(),
                                    workspace.numel() * workspace.element_size(), stream)
    if st != RGF_OK:
        raise RgfError("rgf_batched_solve", st)


def solve_batched(systems, eta_d: float = 0.0, precision: str = "fp64", schedule: str = "longest_first",
                  grid: int = 0, plan: Optional[BatchedPlan] = None, stream=None, waves: int = 0):
    """systems: list of (H [3, l, b, b], sigma_L [nE, b, b], sigma_R, energies [nE]) GPU tensors.
    Runs every (system, energy) instance in one persistent launch; returns a list of
    (G_diag [nE, l, b, b], T [nE], info [nE]) per system."""
    import torch
    dev = systems[0][0].device
    shapes = [(H.shape[1], H.shape[2], E.shape[0]) for (H, _, _, E) in systems]
    if plan is None:
        plan = BatchedPlan(shapes, precision=precision, schedule=schedule, grid=grid, waves=waves)
    outs, entries = [], []
    for (H, sL, sR, E) in systems:
        l, b, ne = H.shape[1], H.shape[2], E.shape[0]
        G = torch.empty((ne, l, b, b), dtype=torch.complex128, device=dev)
        T = torch.empty((ne,), dtype=torch.float64, device=dev)
        info = torch.empty((ne,), dtype=torch.int32, device=dev)
        outs.append((G, T, info))
        entries.append(dict(H=H, sigma_L=sL, sigma_R=sR, energies=E, G_diag=G, T=T, info=info))
    table = device_table(entries, dev)
    ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    rgf_batched_solve(plan, table, eta_d, ws, s.cuda_stream)
    return outs
