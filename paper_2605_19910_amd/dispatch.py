"""Automatic choice between the sequential sweep and DDRGF for one workload.

The paper plans a dispatcher that picks, per workload, between sequential RGF over
energies and the domain-decomposed method (DDRGF) according to where the
parallelism is.  Here the choice is measured rather than modelled: every candidate
(the sequential sweep, which itself gives each energy 1, 2 or 4 workgroups, and
DDRGF with each admissible number of domains) is timed on the caller's own inputs
with the library's kernel timing, and the fastest is kept per workload signature
(sizes, precision, device) in memory and in a JSON table next to this module.

Accuracy: both methods are exact in exact arithmetic, but in FP64 DDRGF inverts
closed interiors, whose conditioning can cost many digits on systems that are not
diagonally dominant; ``methods=("rgf",)`` restricts the choice to the sequential
sweep.
"""
from __future__ import annotations

import json
import os
import threading
from typing import Callable, Dict, Iterable, List, Optional, Tuple

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dispatch_table.json")
DOMAIN_CANDIDATES = (2, 4, 8, 16, 32)
_lock = threading.Lock()
_cache: Dict[str, dict] = {}


def signature(l: int, b: int, w: int, ne: int, precision: str, device: str) -> str:
    return f"l{l}_b{b}_w{w}_ne{ne}_{precision}_{device}"


def candidates(l: int, b: int, w: int, precision: str = "fp64",
               methods: Iterable[str] = ("rgf", "ddrgf")) -> List[Tuple]:
    """Admissible candidates: ("rgf", 0), the sequential sweep; ("ddrgf", m), DDRGF
    (FP64 only) with separators of w layers and interiors of at least w layers (native
    n-diagonal interiors for w > 1); ("ddrgf_fused", m), for w > 1 the same on w-layer
    super-blocks (l divisible by w, w b <= 128); ("ddrgf", m, m2), two-level DDRGF with
    m2 inner pairs, for w = 1, m >= 16 and m2 in {2, 4, 8} with m >= 2 m2."""
    out: List[Tuple] = []
    if "rgf" in methods:
        out.append(("rgf", 0))
    if "ddrgf" in methods and precision == "fp64":
        for m in DOMAIN_CANDIDATES:
            if l - m * w < m * w:
                continue
            out.append(("ddrgf", m))
            if w > 1 and l % w == 0 and w * b <= 128 and l // w - m >= m:
                out.append(("ddrgf_fused", m))
            if m >= 16 and w == 1:
                out += [("ddrgf", m, m2) for m2 in (2, 4, 8) if m >= 2 * m2]
    return out


def pick(timings: Dict[Tuple, float]) -> Tuple:
    """Fastest candidate; ties go to the sequential sweep, then to fewer levels and
    fewer domains."""
    return min(timings, key=lambda k: (timings[k], 0 if k[0] == "rgf" else 1, len(k), k[1:]))


def _load_table() -> dict:
    try:
        with open(TABLE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(sig: str, rec: dict) -> None:
    tab = _load_table()
    tab[sig] = rec
    tmp = TABLE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    os.replace(tmp, TABLE)


def lookup(sig: str) -> Optional[dict]:
    with _lock:
        if sig in _cache:
            return _cache[sig]
        rec = _load_table().get(sig)
        if rec is not None:
            _cache[sig] = rec
        return rec


def choose(l: int, b: int, w: int, ne: int, measure: Callable[..., float], precision: str = "fp64",
           device: str = "cuda0", methods: Iterable[str] = ("rgf", "ddrgf"), retune: bool = False,
           persist: bool = True) -> dict:
    """Time every candidate with measure(method, domains[, inner_domains]) ->
    milliseconds and keep the fastest.  Returns {"method", "domains",
    "inner_domains", "timings_ms"}; cached per signature."""
    methods = tuple(methods)
    sig = signature(l, b, w, ne, precision, device) + "_" + "+".join(sorted(methods))
    if not retune:
        rec = lookup(sig)
        if rec is not None:
            return rec
    cands = candidates(l, b, w, precision, methods)
    if not cands:
        raise ValueError("no admissible method for this workload")
    timings = {c: float(measure(*c)) for c in cands}
    best = pick(timings)
    rec = {"method": best[0], "domains": best[1], "inner_domains": best[2] if len(best) > 2 else 0,
           "timings_ms": {"/".join(str(x) for x in k): round(v, 4) for k, v in timings.items()}}
    with _lock:
        _cache[sig] = rec
    if persist:
        _store(sig, rec)
    return rec


def gpu_measure(H, sigma_L, sigma_R, energies, eta_d: float = 0.0, precision: str = "fp64",
                reps: int = 2) -> Callable[..., float]:
    """measure() for choose(): one untimed solve, then the summed kernel time of the
    best of reps solves, from the library's events on the launch stream."""
    import torch

    from . import binding
    nb, l, b, _ = H.shape
    w = (nb - 1) // 2
    ne = energies.shape[0]

    def measure(method: str, m: int, m2: int = 0) -> float:
        form = "fused" if method == "ddrgf_fused" else "native"
        plan = binding.Plan(l, b, w, ne, method="ddrgf" if method == "ddrgf_fused" else method,
                            precision=precision, domains=m, inner_domains=m2, ddrgf_form=form)
        ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=H.device)
        G = torch.empty((ne, nb, l, b, b), dtype=torch.complex128, device=H.device)
        T = torch.empty((ne,), dtype=torch.float64, device=H.device)
        info = torch.empty((ne,), dtype=torch.int32, device=H.device)
        binding.solve(H, sigma_L, sigma_R, energies, eta_d, plan=plan, workspace=ws, out=(G, T, info))
        best = float("inf")
        plan.set_timing(True, 64)
        for _ in range(reps):
            binding.solve(H, sigma_L, sigma_R, energies, eta_d, plan=plan, workspace=ws, out=(G, T, info))
            best = min(best, sum(v[0] for v in plan.kernel_times().values()))
        plan.set_timing(False)
        plan.close()
        del ws, G
        torch.cuda.empty_cache()
        return best

    return measure
