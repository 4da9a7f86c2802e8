#!/usr/bin/env python3
"""Benchmark: energy points per second of selected G^R + T(E) on one MI355X.

Workload (default): the 256-layer block-tridiagonal system with 128 x 128 complex
blocks, random Hermitian H, closed-form 1D-lead self-energies with eta = 1e-6 and
64 energies at the midpoints of [-2, 2].  One step = one solve over the whole
energy grid: every band block of G^R written plus T(E) for all 64 energies, with
inputs already resident in HBM.

Prints ONE JSON line.  ``roofline`` describes the dominant kernel (the sweep
kernel: one launch per step), timed with HIP events on the stream it runs on;
``cpu_baseline`` is the FP64 oracle on the host cores over a bounded sample of
the same energy grid.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 MFMA
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a kernel, from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) scaled by what the same counters read for a plain copy of
# known size.  Valid only for the kernel sources the counters were taken on: their sha256
# is stored with the figure, and a mismatch reports null.
TRAFFIC_SOURCES = ("paper_2605_19910_amd/csrc/block_engine.h", "paper_2605_19910_amd/csrc/kernels.h",
                   "paper_2605_19910_amd/csrc/ddrgf.hip", "paper_2605_19910_amd/csrc/rgf_sweep.hip",
                   "paper_2605_19910_amd/csrc/split_engine.h", "paper_2605_19910_amd/csrc/rgf_split.hip")
MEASURED_TRAFFIC = {
    # sequential sweep with 4 workgroups per energy, l=256, b=128, 64 energies: FETCH_SIZE
    # 2.94817e+07 KiB x 2.00 + WRITE_SIZE 3.40240e+07 KiB x 1.00 (copy calibration: a 1 GiB copy
    # reads 5.2431e+05 and writes 1.0486e+06 KiB); profiles/rgf_split_kernel_b128_l256_e64_counters.txt
    ("rgf_split_kernel", "c2/rgf_fp64"): {
        "sha256": "08b7a0d0b028b380cbbc1a7d4ca07569955716f4ea74e9166821577456aaa711",
        "bytes": 9.521683e+10},
}


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_for(kernel: str, workload: str):
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None or rec["sha256"] != sources_digest():
        return None
    return rec["bytes"]


def rgf_flops_per_energy(l: int, b: int) -> float:
    """Algorithmic flops of one RGF energy point: the paper's op counts (l LU,
    3l-2 GETRS, 4(l-1) GEMM; eq. cost_model_RGF) at 8/3 b^3, 8 b^3 and 8 b^3 complex
    flops each, plus 8 b^3 per layer for the first-row propagation behind T."""
    b3 = float(b) ** 3
    return (8.0 / 3.0 * l + 8.0 * (3 * l - 2) + 8.0 * 4 * (l - 1) + 8.0 * (l - 1)) * b3


def ddrgf_interior_flops(l: int, b: int, m: int, ne: int, hermitian: bool = False) -> float:
    """Flops executed by the DDRGF interior kernel (closed-interior RGF plus the
    halo products), 8 b^3 per complex product or Gauss-Jordan inversion: per
    interior of n layers, n inversions, 5(n-1) upward products (L, U, the two
    last-row/column propagators, the Schur update), 3(n-1) downward products, and
    2n (last row/column) + 2n (first row/column, all but the first interior).
    With ``hermitian`` (H Hermitian, eta_d = 0) the interiors that hold no lead run
    the Hermitian path: n inversions, 3(n-1) upward products (L, P, Schur update),
    2 + 4(n-1) downward (X_{i,i-1}, X_ii, first and last column)."""
    base, rem = divmod(l - m, m)
    tot = 0.0
    for k in range(m):
        n = base + (1 if k < rem else 0)
        if hermitian and k > 0:
            ops = n + 3 * (n - 1) + 2 + 4 * (n - 1)
        else:
            ops = n + 5 * (n - 1) + 3 * (n - 1) + 2 * n + (2 * n if k > 0 else 0)
        tot += ops
    return tot * 8.0 * float(b) ** 3 * ne


def fused_band(H, w: int):
    """The w-layer super-block (tridiagonal) form of a band [2w+1, l, b, b] (host
    copy, used only to decide which interior path the library takes)."""
    import numpy as np
    _, l, b, _ = H.shape
    lf, B = l // w, w * b
    out = np.zeros((3, lf, B, B), dtype=H.dtype)
    for I in range(lf):
        for kf in (-1, 0, 1):
            J = I + kf
            if not 0 <= J < lf:
                continue
            for r in range(w):
                for c in range(w):
                    i, j = I * w + r, J * w + c
                    if abs(j - i) <= w:
                        out[1 + kf, I, r * b:(r + 1) * b, c * b:(c + 1) * b] = H[w + j - i, i]
    return out


def is_hermitian_band(H) -> bool:
    """H (band [2w+1, l, b, b], block (i, i+d-w) at [d, i]) exactly Hermitian, as the
    library's device check decides."""
    import numpy as np
    w = (H.shape[0] - 1) // 2
    for d in range(w + 1):
        k = w - d                      # block (i, i-k) against block (i-k, i)
        lo = H[d][k:]
        up = H[2 * w - d][:H.shape[1] - k]
        if not np.array_equal(lo, np.conj(np.swapaxes(up, 1, 2))):
            return False
    return True


def ddrgf_recover_flops(l: int, b: int, m: int, ne: int) -> float:
    """Flops executed by the DDRGF recovery kernel, 8 b^3 per complex product: per
    interior of n layers with a left separator, 4 products per layer for
    V^L_i, V^R_i, 2 per recovered band block (3n - 2 of them) and 4 for the
    separator couplings; the first interior (no left separator) needs 1, 1 and 1."""
    base, rem = divmod(l - m, m)
    tot = 0
    for k in range(m):
        n = base + (1 if k < rem else 0)
        left = k > 0
        tot += n * (4 if left else 1) + (3 * n - 2) * (2 if left else 1) + (4 if left else 1)
    return tot * 8.0 * float(b) ** 3 * ne


def nddrgf_interior_flops(l: int, b: int, w: int, m: int, ne: int, hermitian: bool = False) -> float:
    """Flops executed by the native n-diagonal DDRGF interior kernel, 8 b^3 per complex
    product or Gauss-Jordan inversion, counted per interior of n layers as the kernel
    runs them: upward step i (c = min(w, i) coupled layers): 1 inversion, 2c multipliers,
    c^2 Schur products, 2 w c transfer products; downward step i >= 1: 2c^2 + c band
    products; last-column/row halos 2 w min(w, i + 1) per layer; with a left separator
    the first w rows/columns w^2 (w + 1) once and 2 w^2 per layer from layer w on.
    With ``hermitian`` (H Hermitian, eta_d = 0) the interiors without a lead skip the
    row transfer products (Q = P^H): w c fewer per upward step."""
    base, rem = divmod(l - m * w, m)
    ops = 0
    for k in range(m):
        n = base + (1 if k < rem else 0)
        herm = hermitian and k > 0
        for i in range(n):
            c = min(w, i)
            if herm:
                ops += 1 + 2 * c + c * c + w * c               # upward, Hermitian
            else:
                ops += 1 + 2 * c + c * c + 2 * w * c           # upward
            if i >= 1:
                ops += 2 * c * c + c                          # band of X
            ops += 2 * w * min(w, i + 1)                      # CR, RR
            if k > 0 and i >= w:
                ops += 2 * w * w                              # CL, RL recursions
        if k > 0:
            ops += w * w * (w + 1)                            # CL, RL of the first w layers
    return 8.0 * float(b) ** 3 * ops * ne


def nddrgf_recover_flops(l: int, b: int, w: int, m: int, ne: int) -> float:
    """Flops executed by the native n-diagonal DDRGF recovery kernel, 8 b^3 per
    product: per interior layer (g = 2 separator groups, 1 for the first interior)
    (g w)^2 for V_i and g w per band block of the interior row, plus g w per
    separator-row block next to the interior and w^2 (no products) for the
    separator's own blocks."""
    base, rem = divmod(l - m * w, m)
    ops = 0
    for k in range(m):
        n = base + (1 if k < rem else 0)
        g = 2 if k > 0 else 1
        a = k * (base + w) + min(k, rem)
        seps = ([a - w + s for s in range(w)] if k > 0 else []) + [a + n + s for s in range(w)]
        for i in range(n):
            ops += (g * w) ** 2 + g * w * (min(n - 1, i + w) - max(0, i - w) + 1)
            ops += g * w * sum(1 for q in seps if abs(q - (a + i)) <= w)
    return 8.0 * float(b) ** 3 * ops * ne


def nrgf_flops_per_energy(l: int, b: int, w: int) -> float:
    """The paper's op counts for the block n-diagonal sweep (eq. cost_model_general_RGF):
    with c_i = min(w, i) coupled layers above layer i, the upward pass costs l LU,
    2 c_i GETRS and c_i^2 GEMM per layer, the downward pass 1 GETRS and 2 c_i^2 + c_i
    GEMM per layer; the first-row propagation behind T adds c_i GEMM per layer.
    8/3 b^3 per LU, 8 b^3 per GETRS or GEMM."""
    b3 = float(b) ** 3
    tot = 0.0
    for i in range(l):
        c = min(w, i)
        tot += 8.0 / 3.0 + 8.0 * (2 * c + c * c) + 8.0 * (1 + 2 * c * c + c) + 8.0 * c
    return tot * b3


def adjoint_flops(l: int, b: int, ne: int, nd: int) -> float:
    """Flops of the adjoint kernel (on-site gradient), 8 b^3 per complex product or
    Gauss-Jordan inversion: per (energy, domain of n layers starting at i0), the
    upward sweep re-run from the domain's checkpointed pivot (n inversions, n
    multipliers U_i but none for layer 0, n - 1 multipliers L_i and n - 1 Schur
    updates), X = Gamma_R R^H Gamma_L (2), P rebuilt inside the domain (n - 1), and
    per layer R_i (all but the domain's first), X R_i and G_ii P_i."""
    dlen = -(-l // nd)
    per = 0
    for k in range(nd):
        i0 = k * dlen
        if i0 >= l:
            continue
        n = min(dlen, l - i0)
        per += n + (n - (1 if i0 == 0 else 0)) + 2 * (n - 1) + 2 + (n - 1) + (n - 1) + 2 * n
    return per * 8.0 * float(b) ** 3 * ne


def algorithmic_bytes(l: int, b: int, ne: int, w: int = 1) -> float:
    """H read once, Sigma_L/R and E read once, G band written once, T written once."""
    blk = 16.0 * b * b
    return (2 * w + 1) * l * blk + 2 * ne * blk + 8.0 * ne + ne * (2 * w + 1) * l * blk + 8.0 * ne


# ----------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, energies spread over worker processes
# ----------------------------------------------------------------------------

_W = None


def _worker_init(cfg: int):
    global _W
    from workloads import make_config
    _W = make_config(cfg)


def _noop(_):
    return 0


def _oracle_one(e: int) -> float:
    import oracle
    wl = _W
    _, T = oracle.solve_energy(wl.H, wl.w, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], wl.eta_d,
                               method="rgf")
    return T


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_info() -> dict:
    """CPU model and the BLAS NumPy uses, for the baseline's record."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = ""
    try:
        import numpy as np
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = f"{b.get('name', '')} {b.get('version', '')}".strip()
    except Exception:
        pass
    return {"cpu_model": model, "blas": blas, "affinity_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(wl, workers: int, cfg: int = 2, runs: int = 3):
    """The oracle over the whole energy grid, one energy per worker process (fresh
    interpreters, one BLAS thread each), median wall time of ``runs`` runs."""
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["OMP_NUM_THREADS"] = "1"
    idx = list(range(wl.ne))
    ctx = mp.get_context("spawn")
    walls = []
    with ctx.Pool(workers, initializer=_worker_init, initargs=(cfg,)) as pool:
        pool.map(_noop, range(workers), chunksize=1)
        log(f"cpu baseline: {workers} workers ready, timing {len(idx)} oracle energies x {runs} runs")
        for _ in range(runs):
            t0 = time.perf_counter()
            pool.map(_oracle_one, idx, chunksize=1)
            walls.append(time.perf_counter() - t0)
    dt = float(sorted(walls)[len(walls) // 2])
    log(f"cpu baseline: median {dt:.1f} s of {[round(w, 1) for w in walls]}")
    out = {"value": len(idx) / dt, "unit": "energy points/s", "cores": workers, "kind": "oracle",
           "sample": f"all {len(idx)} energies of the same system (sequential RGF + T), one energy per "
                     f"worker process, {workers} processes with 1 BLAS thread each, median wall of {runs} "
                     f"runs {dt:.1f} s"}
    out.update(cpu_info())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="both", choices=["rgf", "ddrgf", "mixed", "both"])
    ap.add_argument("--domains", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--config", type=int, default=2, choices=[2, 3, 4, 5],
                    help="2: the 256 x 128 system (default); 3: the pentadiagonal 512 x 64 system; "
                         "4: the batched 64-device workload; 5: transmission + adjoint gradient, 256 x 64")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones((1 << 27,), dtype=torch.float64, device="cuda:0")   # 1 GiB
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": x.numel() * 8}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU sharding is "
                                   "design-only (energies shard with no exchange)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_19910_amd import binding
    from workloads import make_config

    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    if args.config == 4:
        return bench_batched(args)
    if args.config == 3:
        return bench_ndiag(args)
    if args.config == 5:
        return bench_adjoint(args)
    wl = make_config(2)
    l, b, w, ne = wl.l, wl.b, wl.w, wl.ne
    # the CPU leg runs first, in forked workers, before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        cpu = cpu_baseline(wl, workers)
    dev = torch.device("cuda:0")
    H = torch.from_numpy(wl.H).to(dev)
    sL = torch.from_numpy(wl.sigma_L).to(dev)
    sR = torch.from_numpy(wl.sigma_R).to(dev)
    E = torch.from_numpy(wl.energies).to(dev)
    G = torch.empty((ne, 2 * w + 1, l, b, b), dtype=torch.complex128, device=dev)
    T = torch.empty((ne,), dtype=torch.float64, device=dev)
    info = torch.empty((ne,), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def run_leg(leg: str):
        method, prec = leg.split("_")
        if method == "rgf":
            plan = binding.Plan(l, b, w, ne, method="rgf", precision=prec)
            fn = binding.rgf_solve
        else:
            plan = binding.Plan(l, b, w, ne, method="ddrgf", domains=args.domains, precision=prec)
            fn = binding.ddrgf_solve
        ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=dev)

        def step():
            fn(plan, H, sL, sR, E, wl.eta_d, G, T, info, ws, stream.cuda_stream)

        log(f"{leg}: inputs on the GPU; warmup")
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        status = info & binding.INFO_STATUS_MASK
        if not bool((status == 0).all()) or not bool(torch.isfinite(T).all()):
            print(json.dumps({"error": f"{leg} solve reported a failure",
                              "info": info.cpu().tolist()}), flush=True)
            sys.exit(1)
        n_fp64 = int(((info & binding.INFO_FP64_PRODUCTS) != 0).sum().item())
        log(f"{leg}: warmup done; timing")
        plan.set_timing(True, 16 * args.steps + 16)
        events = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            step()
            e1.record(stream)
            events.append((e0, e1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        step_ms = float(np.mean([a.elapsed_time(c) for a, c in events]))
        res = {"value": ne * args.steps / wall, "ms_per_step": 1000.0 * wall / args.steps,
               "gpu_ms_per_step": step_ms}
        if prec != "fp64":
            res["energies_with_fp32_products"] = ne - n_fp64
        # per-kernel durations from the library's HIP events on the launch stream
        times = plan.kernel_times()
        plan.set_timing(False)
        res["kernel_ms_avg"] = {k: v[0] / v[1] for k, v in times.items()}
        if method == "rgf":
            res["workgroups_per_energy"] = plan.split_workgroups()
        herm = is_hermitian_band(wl.H) and wl.eta_d == 0.0
        rgf_fl = rgf_flops_per_energy(l, b) * ne if method == "rgf" else None
        flops_of = {"rgf_sweep_kernel": rgf_fl, "rgf_split_kernel": rgf_fl,
                    "ddrgf_interior_kernel": ddrgf_interior_flops(l, b, args.domains, ne, herm),
                    "ddrgf_recover_kernel": ddrgf_recover_flops(l, b, args.domains, ne)}
        dom = max(times, key=lambda k: times[k][0])
        res["kernel"] = dom
        res["kernel_ms"] = times[dom][0] / times[dom][1]
        res["flops_per_launch"] = flops_of.get(dom)
        del ws, plan
        torch.cuda.empty_cache()
        if leg != "rgf_fp64" and ref_G is not None:
            res["err_vs_fp64"] = rel_err_stats(G, T, ref_G, ref_T)
        log(f"{leg}: {res['value']:.2f} energy points/s, {step_ms:.2f} ms per step")
        return res

    def rel_err_stats(Gx, Tx, Gr, Tr):
        # per-energy relative Frobenius error of every band block inside the matrix, and of T
        errs = []
        for e in range(ne):
            d = torch.linalg.vector_norm((Gx[e] - Gr[e])[band_mask]).item()
            n = torch.linalg.vector_norm(Gr[e][band_mask]).item()
            errs.append(d / n)
        terr = ((Tx - Tr).abs() / torch.clamp(Tr.abs(), min=1.0)).cpu().numpy()
        return {"G_rel_max": float(np.max(errs)), "G_rel_median": float(np.median(errs)),
                "T_rel_max": float(np.max(terr)), "T_rel_median": float(np.median(terr))}

    band_mask = torch.ones((2 * w + 1, l, b, b), dtype=torch.bool, device=dev)
    band_mask[0, 0] = False
    band_mask[2 * w, l - 1] = False
    ref_G = ref_T = None
    names = {"rgf": ["rgf_fp64"], "ddrgf": ["ddrgf_fp64"], "mixed": ["rgf_fp64", "rgf_fp32"],
             "both": ["rgf_fp64", "ddrgf_fp64", "rgf_fp32"]}[args.method]
    legs = {}
    for leg in names:
        legs[leg] = run_leg(leg)
        if leg == "rgf_fp64":
            ref_G, ref_T = G.clone(), T.clone()
    best = max(legs, key=lambda k: legs[k]["value"])
    lead = legs[best]
    value = legs[best]["value"]
    ms_per_step = legs[best]["ms_per_step"]
    kern_ms = lead["kernel_ms"]
    flops = lead["flops_per_launch"]
    achieved = flops / (kern_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
                "kernel": f"{lead['kernel']} ({best})", "kernel_ms": round(kern_ms, 3),
                "flops_per_launch": flops}
    roofline["traffic"] = traffic_for(lead["kernel"], f"c2/{best}")

    out = {
        "metric": "energy points/sec (selected G^R + T(E))",
        "value": round(value, 3),
        "unit": "energy points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (f64)" if best.endswith("fp64") else "c128 storage, f32 products / f64 pivots",
        "data": "synthetic: seeded random Hermitian block band, closed-form lead self-energies",
        "config": {"workload": "block-tridiagonal, l=256 layers, b=128, 64 energies in [-2,2], "
                               "eta=1e-6, seed 102",
                   "method": {"rgf": "sequential RGF (Algorithm 1)",
                              "ddrgf": f"DDRGF (Algorithm 2), {args.domains} domains"}[best.split("_")[0]],
                   "precision": {"fp64": "fp64", "fp32": "mixed: FP32-MFMA products, FP64 pivots + refinement"}[
                       best.split("_")[1]],
                   "parallelism": "one workgroup per energy (RGF) / per (energy, domain) (DDRGF)"},
        "roofline": roofline,
        "legs": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                 for k, v in legs.items()},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """The batched uneven workload: 64 devices (b in {32,64,96,128}, l in [64,512]),
    16 energies each = 1024 instances in one persistent launch; T and G_ii out."""
    import numpy as np
    import torch

    from paper_2605_19910_amd import autotune, binding
    from workloads import make_config

    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    wls = make_config(4)
    dev = torch.device("cuda:0")
    systems = [(torch.from_numpy(w.H).to(dev), torch.from_numpy(w.sigma_L).to(dev),
                torch.from_numpy(w.sigma_R).to(dev), torch.from_numpy(w.energies).to(dev)) for w in wls]
    shapes = [(w.l, w.b, w.ne) for w in wls]
    n_inst = sum(ne for (_, _, ne) in shapes)
    flops = sum((rgf_flops_per_energy(l, b) - 8.0 * (l - 1) * float(b) ** 3) * ne for (l, b, ne) in shapes)
    log(f"batched: {len(wls)} devices, {n_inst} instances, {flops:.3e} algorithmic flops")
    stream = torch.cuda.current_stream(dev)
    legs = {}
    ref = None
    for prec in ("fp64", "fp32"):
        tuned = autotune.tune(systems, 0.0, precision=prec, log=log)
        # the plan reads the autotuner's table for this workload (schedule, grid, waves)
        plan = binding.BatchedPlan(shapes, precision=prec, schedule="auto")
        outs = binding.solve_batched(systems, 0.0, plan=plan)
        entries = [dict(H=H, sigma_L=sL, sigma_R=sR, energies=E, G_diag=o[0], T=o[1], info=o[2])
                   for (H, sL, sR, E), o in zip(systems, outs)]
        table = binding.device_table(entries, dev)
        ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            binding.rgf_batched_solve(plan, table, 0.0, ws, stream.cuda_stream)
        torch.cuda.synchronize()
        ok = all(bool(((o[2] & binding.INFO_STATUS_MASK) == 0).all()) for o in outs)
        n_fp32 = sum(int(((o[2] & binding.INFO_FP64_PRODUCTS) == 0).sum().item()) for o in outs)
        evs = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.rgf_batched_solve(plan, table, 0.0, ws, stream.cuda_stream)
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = float(np.mean([a.elapsed_time(c) for a, c in evs]))
        res = {"value": n_inst * args.steps / wall, "ms_per_step": 1000.0 * wall / args.steps,
               "kernel_ms": kms, "achieved_tflops": flops / (kms * 1e-3) / 1e12, "all_info_zero": ok,
               "autotune": tuned}
        if prec != "fp64":
            res["instances_with_fp32_products"] = n_fp32
        if prec == "fp64":
            ref = [(o[0].clone(), o[1].clone()) for o in outs]
        else:
            eg, et = [], []
            for (G, T, _), (Gr, Tr) in zip(outs, ref):
                for e in range(G.shape[0]):
                    eg.append((torch.linalg.vector_norm(G[e] - Gr[e]) / torch.linalg.vector_norm(Gr[e])).item())
                et += ((T - Tr).abs() / torch.clamp(Tr.abs(), min=1.0)).cpu().tolist()
            res["err_vs_fp64"] = {"G_diag_rel_max": max(eg), "G_diag_rel_median": float(np.median(eg)),
                                  "T_rel_max": max(et), "T_rel_median": float(np.median(et))}
        legs["batched_" + prec] = res
        log(f"batched {prec}: {res['value']:.1f} instances/s, {kms:.1f} ms per launch")
        del ws, plan, outs, table
        torch.cuda.empty_cache()
    lead = legs["batched_fp64"]
    out = {
        "metric": "energy points/sec (T(E) + diagonal blocks of G^R), batched uneven workload",
        "value": round(lead["value"], 3), "unit": "energy points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(lead["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128 (f64)",
        "data": "synthetic: 64 seeded random Hermitian block-tridiagonal devices",
        "config": {"workload": "64 devices, b in {32,64,96,128}, l in [64,512], 16 energies each "
                               "(1024 instances), eta=1e-6, seed 104",
                   "method": "persistent batched sequential RGF, one hipGraph-capturable launch"},
        "roofline": {"bound": "mfma", "achieved": round(lead["achieved_tflops"], 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(lead["achieved_tflops"] / FP64_PEAK_TFLOPS, 4),
                     "traffic": None, "kernel": "rgf_batched_kernel<0>", "kernel_ms": round(lead["kernel_ms"], 3),
                     "flops_per_launch": flops},
        "legs": legs,
    }
    print(json.dumps(out), flush=True)


def _timed_steps(args, step, plan, stream, n_points, label):
    """Warm up, then time args.steps steps between synchronisations; per-kernel
    durations come from the library's HIP events on the launch stream."""
    import numpy as np
    import torch
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True, 16 * args.steps + 16)
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step()
        e1.record(stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = plan.kernel_times()
    plan.set_timing(False)
    res = {"value": n_points * args.steps / wall, "ms_per_step": 1000.0 * wall / args.steps,
           "gpu_ms_per_step": float(np.mean([a.elapsed_time(c) for a, c in evs])),
           "kernel_ms_avg": {k: v[0] / v[1] for k, v in times.items()}}
    log(f"{label}: {res['value']:.2f} energy points/s, {res['ms_per_step']:.1f} ms per step")
    return res, times


def _roofline(times, flops_of, label):
    dom = max(times, key=lambda k: times[k][0])
    kms = times[dom][0] / times[dom][1]
    fl = flops_of.get(dom)
    ach = fl / (kms * 1e-3) / 1e12 if fl else None
    return {"bound": "mfma", "achieved": round(ach, 3) if ach else None, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4) if ach else None, "traffic": None,
            "kernel": f"{dom} ({label})", "kernel_ms": round(kms, 3), "flops_per_launch": fl}


def bench_ndiag(args):
    """The pentadiagonal system (w = 2, 512 layers of 64, 128 energies): native
    n-diagonal sequential sweep and DDRGF with 16 domains."""
    import torch

    from paper_2605_19910_amd import binding
    from workloads import make_config

    wl = make_config(3)
    l, b, w, ne, m = wl.l, wl.b, wl.w, wl.ne, wl.domains
    Hf_np = fused_band(wl.H, w)
    dev = torch.device("cuda:0")
    H, sL, sR, E = (torch.from_numpy(x).to(dev) for x in (wl.H, wl.sigma_L, wl.sigma_R, wl.energies))
    G = torch.empty((ne, 2 * w + 1, l, b, b), dtype=torch.complex128, device=dev)
    T = torch.empty((ne,), dtype=torch.float64, device=dev)
    info = torch.empty((ne,), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    legs, rooflines, Ts = {}, {}, {}
    for leg in ("nrgf_fp64", "ddrgf_fp64", "ddrgf_fused_fp64"):
        if leg.startswith("nrgf"):
            plan = binding.Plan(l, b, w, ne, method="rgf")
            fn = binding.rgf_solve
        else:
            plan = binding.Plan(l, b, w, ne, method="ddrgf", domains=m,
                                ddrgf_form="fused" if "fused" in leg else "native")
            fn = binding.ddrgf_solve
        ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=dev)
        log(f"{leg}: workspace {plan.workspace_bytes / 2**30:.1f} GiB")

        def step():
            fn(plan, H, sL, sR, E, wl.eta_d, G, T, info, ws, stream.cuda_stream)

        res, times = _timed_steps(args, step, plan, stream, ne, leg)
        res["all_info_zero"] = bool((info == 0).all())
        if leg.startswith("nrgf"):
            res["workgroups_per_energy"] = plan.split_workgroups()
        Ts[leg] = T.clone()
        flops_of = {"nrgf_sweep_kernel": nrgf_flops_per_energy(l, b, w) * ne,
                    "nrgf_split_kernel": nrgf_flops_per_energy(l, b, w) * ne,
                    # DDRGF runs on the w-layer super-block form (l/w layers of w b)
                    "ddrgf_interior_kernel": ddrgf_interior_flops(l // w, w * b, m, ne,
                                                                  is_hermitian_band(Hf_np) and wl.eta_d == 0.0),
                    "ddrgf_recover_kernel": ddrgf_recover_flops(l // w, w * b, m, ne),
                    "nddrgf_interior_kernel": nddrgf_interior_flops(l, b, w, m, ne,
                                                                    is_hermitian_band(wl.H) and wl.eta_d == 0.0),
                    "nddrgf_recover_kernel": nddrgf_recover_flops(l, b, w, m, ne)}
        rooflines[leg] = _roofline(times, flops_of, leg)
        legs[leg] = res
        del ws, plan
        torch.cuda.empty_cache()
    dT = {leg: ((Ts[leg] - Ts["nrgf_fp64"]).abs() / torch.clamp(Ts["nrgf_fp64"].abs(), min=1.0)).max().item()
          for leg in ("ddrgf_fp64", "ddrgf_fused_fp64")}
    best = max(legs, key=lambda k: legs[k]["value"])
    out = {
        "metric": "energy points/sec (selected G^R + T(E))", "value": round(legs[best]["value"], 3),
        "unit": "energy points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(legs[best]["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128 (f64)",
        "data": "synthetic: seeded random Hermitian block pentadiagonal band, closed-form lead self-energies",
        "config": {"workload": f"block pentadiagonal (w=2, next-nearest blocks x0.3), l={l}, b={b}, "
                               f"{ne} energies in [-2,2], eta=1e-4, seed 103",
                   "method": {"nrgf_fp64": "native block n-diagonal sweep",
                              "ddrgf_fp64": f"DDRGF, {m} domains, separators of w layers, n-diagonal interiors",
                              "ddrgf_fused_fp64": f"DDRGF, {m} domains, on w-layer super-blocks"}[best]},
        "roofline": rooflines[best],
        "legs": legs, "rooflines": rooflines, "T_rel_diff_ddrgf_vs_sequential": dT,
    }
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Transmission and its gradient with respect to every on-site energy: the
    256 x 64 system over 256 energies, forward sweep with 8 checkpoint domains,
    then the adjoint kernel (L = sum_E T(E))."""
    import torch

    from paper_2605_19910_amd import binding
    from workloads import make_config

    wl = make_config(5)
    l, b, ne = wl.l, wl.b, wl.ne
    nd = wl.domains or 8
    dev = torch.device("cuda:0")
    H, sL, sR, E = (torch.from_numpy(x).to(dev) for x in (wl.H, wl.sigma_L, wl.sigma_R, wl.energies))
    G = torch.empty((ne, 3, l, b, b), dtype=torch.complex128, device=dev)
    T = torch.empty((ne,), dtype=torch.float64, device=dev)
    info = torch.empty((ne,), dtype=torch.int32, device=dev)
    dLdT = torch.ones((ne,), dtype=torch.float64, device=dev)
    grad = torch.empty((l * b,), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    plan = binding.Plan(l, b, 1, ne, method="rgf", want_backward=True, checkpoint_domains=nd)
    ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=dev)
    log(f"adjoint: workspace {plan.workspace_bytes / 2**30:.1f} GiB")

    Gd = G[:, 1]      # diagonal blocks read in place from the output band

    def step():
        binding.rgf_solve(plan, H, sL, sR, E, wl.eta_d, G, T, info, ws, stream.cuda_stream)
        binding.rgf_backward(plan, H, sL, sR, E, wl.eta_d, Gd, 3 * l * b * b, dLdT, None, grad, ws,
                             stream.cuda_stream)

    res, times = _timed_steps(args, step, plan, stream, ne, "forward+adjoint")
    res["all_info_zero"] = bool((info == 0).all())
    res["grad_finite"] = bool(torch.isfinite(grad).all())
    flops_of = {"rgf_sweep_kernel": rgf_flops_per_energy(l, b) * ne,
                "rgf_adjoint_kernel": adjoint_flops(l, b, ne, nd)}
    roof = _roofline(times, flops_of, "forward+adjoint")
    adj = {k: v for k, v in times.items() if k == "rgf_adjoint_kernel"}
    out = {
        "metric": "energy points/sec (T(E) + dT/d(on-site energies) via the adjoint)",
        "value": round(res["value"], 3), "unit": "energy points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(res["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128 (f64)",
        "data": "synthetic: seeded random Hermitian block-tridiagonal band, closed-form lead self-energies",
        "config": {"workload": f"block-tridiagonal, l={l}, b={b}, {ne} energies in [-2,2], eta=1e-6, "
                               f"seed 105; gradient w.r.t. {l * b} on-site energies, {nd} checkpoint domains",
                   "method": "sequential RGF forward + adjoint kernel"},
        "roofline": roof,
        "adjoint_roofline": _roofline(adj, flops_of, "adjoint only") if adj else None,
        "legs": {"forward_adjoint_fp64": res},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
