"""Shared parity rule and oracle worker pool for the GPU tests.

Parity rule for the FP64 paths, fixed before any full-size run
---------------------------------------------------------------
The GPU and the oracle run the same block elimination, without pivoting across
blocks (partial row pivoting inside each block only), so both carry the rounding
error of each Schur pivot's inversion amplified by that pivot's condition number.
The classical forward-error bound for inverting (or solving with) a b x b matrix of
1-norm condition number kappa with partial pivoting is of order gamma_b * kappa with
gamma_b = b u / (1 - b u) ~ b u, u = 2^-53.  Both sides err, hence per energy

    tol = max(1e-10, 2 * b * u * kappa_max)

where kappa_max is the largest kappa_1 over the Schur pivots met by the oracle's
run of the same method at that energy (for DDRGF: interior pivots and the reduced
system's pivots, whose blocks have w b rows).  The bound applies to the relative
Frobenius error over all band blocks inside the matrix and to |dT| / max(1, T).
1e-10 is the target figure; it is the bound wherever the pivots are well
conditioned (kappa_max < ~1e3 at b = 128).

DDRGF is compared element by element with the oracle's DDRGF, and both with the
exact band, under a rule of its own.  Algorithm 2 inverts closed interiors (no lead,
no broadening) by elimination and then recovers G_{D2,D2} = X + X T21 G_S T12 X,
cancelling the interior inverse X against the correction wherever the energy is
close to an interior eigenvalue.  The normwise forward-error bound of inverting an
n x n matrix by elimination is of order n u kappa, so an interior of n_int = s2 b
rows (the largest one) is known to about n_int u kappa_max relative to ||X||; the
recovery turns that into an error relative to ||G|| larger by
rho = ||X||_F / ||G||_F (Frobenius norms over the interiors' bands and over the
output band).  Both sides err, hence per energy

    tol = max(1e-10, 2 * n_int * u * kappa_max * max(1, rho)),

for the band against the oracle's DDRGF, T against it, and the band against the
exact band (dense inverse on small systems, the oracle's sequential RGF at the
full size, itself within the FP64 rule of the exact band).  kappa_max, rho and
n_int come from the oracle's DDRGF run at that energy.

An earlier rule, max(2 b u kappa_max, 8 e_method) with e_method the oracle DDRGF's
own distance to the exact band, used one sample of the rounding error as the
error scale; at one of 17 sampled energies of the 512-layer pentadiagonal system
the oracle's rounding landed 12 times closer to the exact band than the GPU's and
the rule failed there.  On the same runs (256 x 128, 64 energies; 512 x 64, 17
energies) the GPU-oracle differences stay within 0.30 of the rule above.  Where
kappa_max rho is huge the rule is loose (DDRGF in FP64 has no more digits there,
whichever implementation runs it), so the full-size DDRGF parity is also checked on
block diagonally dominant systems, the class of test matrices of the paper's
experiments, where the rule comes down to the 1e-10 target.

Oracle work runs in a pool of fresh interpreters (one BLAS thread each), so the
full-size comparisons over every energy take seconds to a few minutes.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from typing import Dict

import numpy as np

U64 = 2.0 ** -53
TARGET_FP64 = 1e-10
TARGET_MIXED = 1e-5


def fp64_bound(kappa: float, b: int) -> float:
    k = float(kappa)
    if not np.isfinite(k):
        k = 0.0          # no pivot conditioning known (dense reference): the target itself
    return max(TARGET_FP64, 2.0 * b * U64 * k)


def dd_bound(kappa: float, n_int: int, rho: float) -> float:
    """DDRGF rule (module docstring)."""
    return max(TARGET_FP64, 2.0 * n_int * U64 * float(kappa) * max(1.0, float(rho)))


def mask_band(G: np.ndarray, w: int) -> np.ndarray:
    """Zero the band entries that fall outside the matrix (never written by the
    library); G is [..., 2w+1, l, b, b]."""
    G = np.array(G, copy=True)
    l = G.shape[-3]
    for k in range(-w, w + 1):
        if k < 0:
            G[..., w + k, :(-k), :, :] = 0
        elif k > 0:
            G[..., w + k, l - k:, :, :] = 0
    return G


def rel(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def terr(T, Tref) -> float:
    return abs(float(T) - float(Tref)) / max(1.0, abs(float(Tref)))


# ----------------------------------------------------------------------------
# worker pool
# ----------------------------------------------------------------------------

_POOL = None


def pool():
    global _POOL
    if _POOL is None:
        os.environ["OPENBLAS_NUM_THREADS"] = "1"
        os.environ["OMP_NUM_THREADS"] = "1"
        n = max(1, min(16, len(os.sched_getaffinity(0))))
        _POOL = mp.get_context("spawn").Pool(n)
    return _POOL


def pmap(fn, items):
    """Ordered parallel map over the oracle pool."""
    items = list(items)
    if len(items) <= 1:
        return [fn(x) for x in items]
    return pool().map(fn, items, chunksize=1)


_WL: Dict = {}


def _workload(src):
    """src: a Workload, ("config", n) regenerated (and cached) in the worker,
    ("config", 4, d) for device d of the batched workload, or
    ("dominant", l, b, w, ne, seed) for workloads.make_dominant."""
    if isinstance(src, tuple):
        if src[0] == "dominant":
            if src not in _WL:
                from workloads import make_dominant
                _WL[src] = make_dominant(*src[1:])
            return _WL[src]
        key = src[:2]
        if key not in _WL:
            from workloads import make_config
            _WL[key] = make_config(src[1])
        return _WL[key][src[2]] if len(src) > 2 else _WL[key]
    return src


def _args(src, e, eta_d):
    wl = _workload(src)
    eta = wl.eta_d if eta_d is None else eta_d
    return wl, (wl.H, wl.energies[e], wl.sigma_L[e], wl.sigma_R[e], eta)


# Each task returns {"G": band, "T": transmission, "kappa": worst pivot kappa_1}.

def task_rgf(spec):
    import oracle
    src, e, eta_d = spec
    wl, a = _args(src, e, eta_d)
    r = oracle.rgf(*a, extras=True, pivot_cond=True)
    return {"G": r["G"], "T": oracle.transmission(r["row0"][wl.l - 1], a[2], a[3]), "kappa": r["pivot_cond"]}


def task_nrgf(spec):
    import oracle
    src, e, eta_d = spec
    wl, a = _args(src, e, eta_d)
    Mb = oracle.block_accessor(wl.H, wl.w, *a[1:])
    r = oracle.nrgf(Mb, wl.l, wl.b, wl.w, halo=1, pivot_cond=True)
    return {"G": r["G"], "T": oracle.transmission(r["first_rows"][0, wl.l - 1], a[2], a[3]),
            "kappa": r["pivot_cond"]}


def task_ddrgf(spec):
    """spec: (src, e, eta_d, m) with m the number of pairs, or (m, m2, ...) for
    multi-level DDRGF.  Returns the band, T, kappa_max over every level, and the
    DDRGF rule's n_int and rho (for several levels: the largest interior over the
    levels and the product of the levels' rho)."""
    import oracle
    src, e, eta_d, m = spec
    inner = ()
    if isinstance(m, (tuple, list)):
        m, inner = m[0], tuple(m[1:])
    wl, a = _args(src, e, eta_d)
    r = oracle.ddrgf(wl.H, wl.w, *a[1:], n_pairs=m, pivot_cond=True, return_parts=True, inner_pairs=inner)
    rho, n_int = 1.0, 0
    lev, band, blk = r, mask_band(r["G"], wl.w), wl.b
    while True:
        xn = np.sqrt(sum(np.linalg.norm(x["G"]) ** 2 for x in lev["X"]))
        rho *= max(1.0, xn / np.linalg.norm(band))
        n_int = max(n_int, blk * max(e1 - a1 + 1 for (a1, e1, p1) in lev["layout"]))
        if "inner" not in lev:
            break
        blk = wl.w * wl.b
        band = mask_band(lev["GS"], 1)
        lev = lev["inner"]
    return {"G": r["G"], "T": oracle.transmission(r["G_0_last"], a[2], a[3]), "kappa": r["pivot_cond"],
            "rho": rho, "n_int": n_int}


def task_ext(spec):
    import oracle
    src, e, eta_d = spec
    wl, a = _args(src, e, eta_d)
    G, T = oracle.solve_energy_ext(wl.H, wl.w, *a[1:])
    return {"G": np.asarray(G, dtype=np.complex128), "T": T, "kappa": float("nan")}


def task_dense(spec):
    import oracle
    src, e, eta_d = spec
    wl, a = _args(src, e, eta_d)
    band, Gf = oracle.dense_selected(wl.H, wl.w, *a[1:], full=True)
    b, n = wl.b, wl.l * wl.b
    return {"G": band, "T": oracle.transmission(Gf[:b, n - b:], a[2], a[3]), "kappa": float("nan")}


def task_mixed(spec):
    import oracle
    src, e, eta_d = spec
    wl, a = _args(src, e, eta_d)
    r = oracle.rgf_mixed_products(*a)
    return {"G": r["G"], "T": oracle.transmission(r["G_0_last"], a[2], a[3]), "kappa": float("nan")}


def task_lesser(spec):
    """spec: (src, e, eta_d, (f_L, f_R)); the band of G^< and the sweep's kappa."""
    import oracle
    src, e, eta_d, occ = spec
    wl, a = _args(src, e, eta_d)
    G, Gl = oracle.lesser(*a[:4], occ[0], occ[1], a[4])
    r = oracle.rgf(*a, extras=False, pivot_cond=True)
    return {"G": Gl, "GR": G, "kappa": r["pivot_cond"]}


TASKS = {"rgf": task_rgf, "nrgf": task_nrgf, "ddrgf": task_ddrgf, "ext": task_ext, "dense": task_dense,
         "mixed": task_mixed, "lesser": task_lesser}


def oracle_results(kind: str, src, energies, eta_d=None, m=None, occ=None):
    """occ (kind "lesser"): per energy (f_L, f_R)."""
    fn = TASKS[kind]
    if kind == "lesser":
        specs = [(src, int(e), eta_d, tuple(o)) for e, o in zip(energies, occ)]
        return pmap(fn, specs)
    specs = [(src, int(e), eta_d, m) if kind == "ddrgf" else (src, int(e), eta_d) for e in energies]
    return pmap(fn, specs)


# ----------------------------------------------------------------------------
# comparisons
# ----------------------------------------------------------------------------

def gpu_energy(G, e, w):
    """Band of one energy from a GPU (torch) or host array, masked to the matrix."""
    x = G[e]
    if hasattr(x, "cpu"):
        x = x.cpu().numpy()
    return mask_band(x, w)


def check_dd(label, G, T, energies, refs_dd, refs_exact, w):
    """DDRGF rule (module docstring): per energy, band and T within dd_bound of the
    oracle's DDRGF and the band within it of the exact band.  Prints every energy's
    figures, asserts after all of them are printed."""
    rows, bad = [], []
    for e, r, x in zip(energies, refs_dd, refs_exact):
        Ge = gpu_energy(G, e, w)
        err = rel(Ge, r["G"])
        te = terr(T[e], r["T"])
        e_method = rel(r["G"], x["G"])
        e_gpu = rel(Ge, x["G"])
        tol = dd_bound(r["kappa"], r["n_int"], r["rho"])
        rows.append((e, err, te, tol, e_method, e_gpu))
        print(f"{label} energy {e}: kappa {r['kappa']:.2e} rho {r['rho']:.2e} |dG|/|G| vs oracle DDRGF {err:.2e} "
              f"dT {te:.2e} bound {tol:.2e}; vs exact: GPU {e_gpu:.2e} oracle DDRGF {e_method:.2e}", flush=True)
        if not (err <= tol and te <= tol and e_gpu <= tol):
            bad.append((e, err, te, e_gpu, tol))
    eg = np.array([x[5] for x in rows])
    em = np.array([x[4] for x in rows])
    print(f"{label}: {len(rows)} energies, distance to the exact band: GPU median {np.median(eg):.2e} max "
          f"{eg.max():.2e}; oracle DDRGF median {np.median(em):.2e} max {em.max():.2e}", flush=True)
    assert not bad, bad
    return rows


def check_fp64(label, G, T, energies, refs, w, b, extra_bound=None):
    """Per energy: band and T within fp64_bound(kappa, b) of the reference.  Prints
    every energy's figures, asserts after all of them are printed.  Returns the
    list of (e, err, terr, tol, kappa)."""
    rows, bad = [], []
    for e, r in zip(energies, refs):
        err = rel(gpu_energy(G, e, w), r["G"])
        te = terr(T[e], r["T"])
        tol = fp64_bound(r["kappa"], b)
        if extra_bound is not None:
            tol = max(tol, extra_bound)
        rows.append((e, err, te, tol, r["kappa"]))
        print(f"{label} energy {e}: kappa {r['kappa']:.2e} |dG|/|G| {err:.2e} dT {te:.2e} bound {tol:.2e}",
              flush=True)
        if not (err <= tol and te <= tol):
            bad.append((e, err, te, tol))
    errs = np.array([x[1] for x in rows])
    print(f"{label}: {len(rows)} energies, band error median {np.median(errs):.2e} max {errs.max():.2e}",
          flush=True)
    assert not bad, bad
    return rows
