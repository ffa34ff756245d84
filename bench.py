"""Benchmark of the hyperbolic self-gravity hot path on one MI355X.

One step = one hydrodynamical step of the method: multipole moments of rho and
the Dirichlet ghost shell, `nsub` leapfrog substeps of Eq. (2) with rho frozen,
and the acceleration g = -grad phi.  Workload: 512^3 cell-centred grid on
[-1, 1]^3, FP32 storage with the substeps in the FP32 increment form (moments,
ghosts, gradient and norms in FP64), rho a mixture of 16 Gaussian
blobs (seed 1) rigidly rotating about z at 0.1 c_g, multipole degree 4,
4 substeps per hydro step, dt = 0.4 dx / c_g.  Every hydro step gets its own
rotated density, generated into HBM before the timed region.

Prints one JSON line: Gcell-updates/s (cells x substeps / s) with the
stencil kernel's roofline, measured with HIP events on the solver's stream,
and the FP64 CPU oracle timed on the host cores over one hydro step of the
same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


CONVERGE_SUBSTEPS = 3600  # critically damped 512^3: R_b ~ e^-15 of its zero-start value
SETTLE_STEPS = 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tile_desc(storage: str, tblock: int, tile: int):
    """The fused launch's tile as reported: index and shape (rows per thread,
    waves, planes in flight); None when the depth has no fused launch."""
    from paper_1602_05700_amd import hgs

    if tblock < 2:
        return None
    r, w, pf = hgs.tile_shape(storage, tblock, tile if tile < hgs.tile_count(tblock) else 0)
    return {"index": tile, "rows_per_thread": r, "waves": w, "planes_in_flight": pf,
            "extended_tile": [64, r * w]}


KERNEL_SOURCES = {
    # sources that define each timed stencil kernel (the counter file is valid
    # only while they are unchanged)
    "leapfrog_tblock": ("common.hpp", "k_tblock.hpp"),
    "leapfrog_stream": ("common.hpp", "k_stencil.hpp"),
}


def kernel_source_hash(kernel: str = "leapfrog_tblock") -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1602_05700_amd", "csrc")
    for f in KERNEL_SOURCES["leapfrog_stream" if kernel.startswith("leapfrog_stream") else "leapfrog_tblock"]:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(kernel: str, launches_cells: int, tile: int = 0):
    """HBM bytes per launch from the committed rocprofv3 counter summary (one
    entry per tile shape: kernel, kernel_tile1, ...), if it was taken on the
    current kernel sources, workload and tile shape; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(kernel if tile == 0 else f"{kernel}_tile{tile}")
        if (not e or e.get("source_hash") != kernel_source_hash(kernel) or e.get("cells") != launches_cells
                or e.get("tile", 0) != tile):
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def host_cpu() -> str:
    """Model name and logical CPU count of the host, from /proc/cpuinfo."""
    try:
        names = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")]
        return f"{names[0]} ({len(names)} logical CPUs)" if names else "unknown"
    except OSError:
        return "unknown"


def cpu_baseline(rho_host, n, nsub, dt, phi0_host=None, gpu=None):
    """The FP64 oracle, as it stands, over one hydro step of the same workload
    (from phi0 when given, else from zero).  gpu = (phi, gx, gy, gz) of the
    same hydro step from the same state, as host arrays: their error against
    the oracle, max |a - b| / max |b| per field, is reported as well."""
    import numpy as np

    from oracle import core
    from oracle.core import Grid, Oracle

    g = Grid.cube(n)
    o = Oracle(g, lmax=4, eta=0.0)
    r = np.ascontiguousarray(rho_host, dtype=np.float64)
    if phi0_host is not None:
        o.set_state(np.asarray(phi0_host, dtype=np.float64), None, dt)
    t0 = time.perf_counter()
    o.step(r, 1.0, dt, nsub)
    acc = o.accel()
    t = time.perf_counter() - t0
    out = {
        "value": nsub * n ** 3 / t / 1e9,
        "unit": "Gcell-updates/s",
        "cores": core.max_threads(),
        "kind": "oracle",
        "sample": f"one hydro step ({n}^3, moments+ghosts, {nsub} substeps, gradient) in {t:.2f} s",
    }
    # the same oracle on one thread, over a smaller sample of the workload
    nt = core.max_threads()
    stride = max(1, n // 256)
    r1 = np.ascontiguousarray(r[::stride, ::stride, ::stride])
    m = r1.shape[0]
    g1 = Grid.cube(m)
    o1 = Oracle(g1, lmax=4, eta=0.0)
    core.set_threads(1)
    try:
        t1 = time.perf_counter()
        o1.step(r1, 1.0, 0.4 * g1.dx, nsub)
        o1.accel()
        t1 = time.perf_counter() - t1
    finally:
        core.set_threads(nt)
    out["one_thread"] = {"value": nsub * m ** 3 / t1 / 1e9, "unit": "Gcell-updates/s", "cores": 1,
                         "sample": f"one hydro step ({m}^3, the density sampled every {stride} cells) in {t1:.2f} s"}
    out["host_cpu"] = host_cpu()
    if gpu is not None:
        rel = lambda a, b: float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b)) / np.max(np.abs(b)))
        out["gpu_vs_oracle"] = {"phi": rel(gpu[0], o.potential()[0]),
                                "accel": max(rel(a, b) for a, b in zip(gpu[1:], acc)),
                                "metric": "max|gpu - oracle| / max|oracle| per field, FP32 storage",
                                "tolerance": 1e-4}
    return out


def run_batched(dev, nsub=500, seed=2, count=64):
    """64 independent cube grids, N in {32, 48, ..., 160} drawn with the seed,
    each with its own 4-12 blob density, FP32 storage, lmax 4; one hydro step
    of 500 substeps (dt = 0.4 dx_g) for all grids together, replayed from a
    captured graph.  Returns total cell updates per second of the default
    launch form (one workgroup per work item, grid-ordered), and the
    persistent form's beside it."""
    import torch

    import workloads
    from paper_1602_05700_amd import hgs

    spec = workloads.batch_spec(seed=seed, count=count)
    rhos = [workloads.blob_density_torch(n, workloads.blob_params(s, k), dev, torch.float32)
            for n, k, s in zip(spec.sizes, spec.nblobs, spec.seeds)]
    b = hgs.Batch(list(spec.sizes), storage="f32", lmax=4, eta=0.0, device=dev)
    dts = [0.4 * 2.0 / n for n in spec.sizes]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(launch, reps=2):
        b.set_launch(launch)
        b.step(rhos, 1.0, dts, nsub)  # warm-up: captures the graph of this launch form
        torch.cuda.synchronize()
        log(f"[bench]   batched {launch}: warmed up")
        e0.record(b.stream)
        for _ in range(reps):
            b.step(rhos, 1.0, dts, nsub)
        e1.record(b.stream)
        torch.cuda.synchronize()
        log(f"[bench]   batched {launch}: timed")
        return e0.elapsed_time(e1) / reps

    ms_persistent = timed("persistent")
    ms = timed("per_item")  # the default launch form, timed last
    cells = sum(n ** 3 for n in spec.sizes)
    T = b.grids[0].tblock
    # algorithmic bytes of the substeps: per fused launch each cell's phi^n,
    # phi^{n-1} and rho are read and two levels written (FP32), per streaming
    # substep three reads and one write; the moments and ghosts once per step
    # are counted in the time but not in the bytes
    launches = nsub // T if T > 1 else nsub
    stencil_bytes = (20.0 if T > 1 else 16.0) * cells * launches + 16.0 * cells * (nsub - launches * max(T, 1))
    gbps = stencil_bytes / (ms / 1e3) / 1e9
    return {"grids": count, "cells": cells, "substeps": nsub, "ms_per_hydro_step": round(ms, 3),
            "value": round(cells * nsub / (ms / 1e3) / 1e9, 3), "unit": "Gcell-updates/s",
            "graph": b.used_graph, "tblock": T, "launch": b.launch, "stencil_GBps_algorithmic": round(gbps, 1),
            "hbm_frac": round(gbps / PEAK_HBM_GBS, 4),
            "persistent_launch": {"ms_per_hydro_step": round(ms_persistent, 3),
                                  "value": round(cells * nsub / (ms_persistent / 1e3) / 1e9, 3)}}


def run_configs(dev):
    """Throughput of the two smaller configurations, besides the headline one:
    the 64^3 uniform sphere (FP64, lmax 0, zero start, 2000 substeps, eta = 0
    as in Eq. 2 and critically damped) and the 256^3 rotating 8-blob mixture
    (seed 0, speed 0.1 c_g at radius 1, lmax 4, 4 substeps per hydro step,
    250 hydro steps, FP64 and FP32 storage, moments + ghosts + substeps +
    gradient timed; 64 rotated densities generated beforehand and cycled).
    Each run takes the fused depth the library's autotuner picks for it."""
    import math

    import torch

    import workloads
    from paper_1602_05700_amd import hgs

    out = {}
    n = 64
    dx = 2.0 / n
    dt = 0.4 * dx
    rho = torch.from_numpy(workloads.sphere_density(n, 0.25)).to(dev)
    lam = 3 * (4 / dx ** 2) * math.sin(math.pi / (2 * (n + 1))) ** 2  # slowest Dirichlet mode
    for label, eta in (("eta_0", 0.0), ("eta_critical", 2.0 * math.sqrt(lam))):
        # fused depth and tile by the library's autotuner (timed on 200-substep
        # steps, so the per-step moment and ghost launches weigh as in the run):
        # at 64^3 a fused launch is bound by its pipeline fill, not by HBM
        tb, tile, _ = hgs.autotune(n, rho, 1.0, dt, 200, storage="f64", lmax=0, eta=eta, device=dev)
        s = hgs.Solver(n, storage="f64", lmax=0, eta=eta, tblock=tb, tile=tile, device=dev)
        s.step(rho, 1.0, dt, 8)  # warm-up
        s2 = hgs.Solver(n, storage="f64", lmax=0, eta=eta, tblock=tb, tile=tile, device=dev)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s2.stream)
        s2.step(rho, 1.0, dt, 2000)
        e1.record(s2.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out.setdefault("sphere_64_f64", {})[label] = {
            "substeps": 2000, "tblock": tb, "tile": tile_desc("f64", tb, tile), "ms": round(ms, 3),
            "Gcell_updates_per_s": round(n ** 3 * 2000 / (ms / 1e3) / 1e9, 2),
            "R_f": float(s2.residual(rho)[1])}
        s.close()
        s2.close()
    n, nsub, steps = 256, 4, 250
    dx = 2.0 / n
    dt = 0.4 * dx
    blobs = workloads.blob_params(0, 8)
    for storage, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        rhos = [workloads.blob_density_torch(n, blobs.rotated(0.1 * nsub * dt * h), dev, tdt) for h in range(64)]
        tb, tile, _ = hgs.autotune(n, rhos[0], 1.0, dt, nsub, storage=storage, lmax=4, eta=0.0, device=dev)
        s = hgs.Solver(n, storage=storage, lmax=4, eta=0.0, tblock=tb, tile=tile, device=dev)
        g = [torch.empty((n, n, n), dtype=tdt, device=dev) for _ in range(3)]
        for h in range(3):
            s.step(rhos[h], 1.0, dt, nsub)
            s.accel(g)
        torch.cuda.synchronize()
        s.timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        for h in range(steps):
            s.step(rhos[h % 64], 1.0, dt, nsub)
            s.accel(g)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        kinds = {k: s.timing_read(k) for k in ("stencil", "multipole", "gradient")}
        s.timing(False)
        out.setdefault("rotating_256", {})[storage] = {
            "hydro_steps": steps, "tblock": s.tblock, "tile": tile_desc(storage, s.tblock, s.tile),
            "ms_per_hydro_step": round(ms / steps, 4),
            "Gcell_updates_per_s": round(n ** 3 * nsub * steps / (ms / 1e3) / 1e9, 2),
            "us_per_launch": {k: round(d["ms"] / max(d["launches"], 1) * 1e3, 1) for k, d in kinds.items()},
            "stencil_GBps_algorithmic": round(kinds["stencil"]["bytes"] / kinds["stencil"]["ms"] / 1e6, 0)}
        s.close()
        del rhos, g
        torch.cuda.empty_cache()
    out["tracking_256"] = run_tracking(dev)
    out["next_rows_256_f32"] = run_next_rows(dev)
    return out


def run_tracking(dev, n=256, nsub=4, steps=250, every=5, omega=0.1):
    """Tracking accuracy of the 256^3 rotating configuration (8 blobs, seed 0,
    speed 0.1 c_g at radius 1, l <= 4, 4 substeps per hydro step, eta = 0)
    over 250 hydro steps from the converged potential of the first density
    with the rigid-rotation phidot, in FP64 and FP32 storage: the paper's
    average relative error (Eq. 6, the volume RMS of (phi_H - phi_P) / phi_P,
    Eq. 5) against the Poisson solution phi_P of the density of the last hydro
    step, every `every` hydro steps.  phi_P is the solver's own damped
    relaxation (FP64, critical damping) carried from checkpoint to checkpoint:
    the damped iteration's fixed point is the discrete Poisson solution, and
    its residual R_b is reported with the errors."""
    import math

    import torch

    import workloads
    from paper_1602_05700_amd import hgs

    dx = 2.0 / n
    dt = 0.4 * dx
    lam = 3 * (4 / dx ** 2) * math.sin(math.pi / (2 * (n + 1))) ** 2
    eta_c = 2.0 * math.sqrt(lam)
    blobs = workloads.blob_params(0, 8)
    dens = lambda h, tdt: workloads.blob_density_torch(n, blobs.rotated(omega * nsub * dt * h), dev, tdt)
    ref = hgs.Solver(n, storage="f64", lmax=4, eta=eta_c, device=dev)
    r0 = dens(0, torch.float64)
    ref.step(r0, 1.0, dt, 4000)
    start_rb = float(ref.residual(r0)[0])
    phi0 = ref.potential(with_phidot=False)[0]
    ax = -1.0 + (torch.arange(n, device=dev, dtype=torch.float64) + 0.5) * dx
    dpy, dpx = torch.gradient(phi0, spacing=dx, dim=(1, 2))
    pd0 = (-omega * (ax[None, None, :] * dpy - ax[None, :, None] * dpx)).contiguous()
    del dpy, dpx
    runs = {}
    for storage, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        s = hgs.Solver(n, storage=storage, lmax=4, eta=0.0, device=dev)
        s.set_state(phi0.to(tdt), pd0.to(tdt), dt)
        runs[storage] = s
    eq6 = {"f64": [], "f32": []}
    ref_rb = []
    t0 = time.time()
    for h in range(1, steps + 1):
        rho64 = dens(h - 1, torch.float64)
        runs["f64"].step(rho64, 1.0, dt, nsub)
        runs["f32"].step(rho64.float(), 1.0, dt, nsub)
        if h % every == 0:
            ref.step(rho64, 1.0, dt, 1600)  # relax the Poisson reference to this density
            ref_rb.append(float(ref.residual(rho64)[0]))
            phi_p = ref.potential(with_phidot=False)[0]
            for storage, sv in runs.items():
                d = (sv.potential(with_phidot=False)[0].double() - phi_p) / phi_p
                eq6[storage].append(float(torch.sqrt(torch.mean(d * d))))
    fin = {k: v.potential(with_phidot=False)[0].double() for k, v in runs.items()}
    diff = float((fin["f32"] - fin["f64"]).abs().max() / fin["f64"].abs().max())
    for v in runs.values():
        v.close()
    ref.close()
    log(f"[bench] tracking 256^3: {steps} hydro steps in {time.time() - t0:.1f} s, "
        f"Eq. 6 max f64 {max(eq6['f64']):.3e} f32 {max(eq6['f32']):.3e}")
    return {"hydro_steps": steps, "every": every, "metric": "Eq. 6 (volume RMS of (phi_H - phi_P)/phi_P)",
            "reference": "FP64 damped relaxation, 1600 critically damped substeps per checkpoint",
            "start_R_b": start_rb, "reference_R_b_max": max(ref_rb),
            "eq6_f64": {"max": max(eq6["f64"]), "final": eq6["f64"][-1], "mean": sum(eq6["f64"]) / len(eq6["f64"])},
            "eq6_f32": {"max": max(eq6["f32"]), "final": eq6["f32"][-1], "mean": sum(eq6["f32"]) / len(eq6["f32"])},
            "eq6_at": {str(h): [round(a, 8), round(b, 8)] for h, a, b in
                       zip(range(every, steps + 1, every), eq6["f64"], eq6["f32"])
                       if h in (every, 25, 50, 100, 150, 200, steps)},
            "f32_vs_f64_phi_maxrel_final": diff}


def run_next_rows(dev, n=256, nsub=4, steps=20):
    """Throughput of the parts built beyond the multipole path, at 256^3 FP32
    on the same 8-blob density (eta = 0, dt = 0.4 dx): the local boundaries
    (the faster, over whole hydro steps, of the autotuner's depth and tile
    and one substep per launch; all three can fuse substeps), the three
    again at 512^3 with one and with four substeps per launch, the
    extended grid (32 vacuum
    cells on every side, outgoing boundary, rho embedded every hydro step, g on
    the hydrodynamics region; updates counted over the whole wider grid), the
    nested coarse outer levels (Robin at the outermost faces; one level 16 or
    64 coarse cells beyond the fine grid, or two levels of 16 cells each;
    coarse sources, coarse substeps, interpolated ghosts and the fine substeps
    at the fused depth; fine updates counted) and
    the hydro-coupled driver (signal-speed reduction over c_s and v, k_g = 5,
    Courant numbers 0.3: 5 substeps per hydro step).  Each entry: ms per
    hydro step (step + gradient) and cell updates per second."""
    import torch

    import workloads
    from paper_1602_05700_amd import hgs

    dx = 2.0 / n
    dt = 0.4 * dx
    rho = workloads.blob_density_torch(n, workloads.blob_params(0, 8), dev, torch.float32)
    res = {}

    def timed(label, run, updates):
        for _ in range(3):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[label] = {"ms_per_hydro_step": round(ms, 4), "Gcell_updates_per_s": round(updates / (ms / 1e3) / 1e9, 2)}

    g = [torch.empty((n, n, n), dtype=torch.float32, device=dev) for _ in range(3)]
    for bc in ("robin", "outgoing", "periodic"):
        # the depth and tile the autotuner picks for this boundary and size
        # (it times hgs_step alone), against one substep per launch, both over
        # whole hydro steps (gradient included: at 256^3 it runs slower after a
        # fused launch, whose outputs push phi^n out of the last-level cache);
        # the faster is the entry
        best, tile, _ = hgs.autotune((n, n, n), rho, 1.0, dt, nsub, storage="f32", bc=bc, device=dev)
        runs = {}
        for T, tl in {(best, tile), (1, 0)}:
            sv = hgs.Solver(n, storage="f32", lmax=4, eta=0.0, bc=bc, device=dev, tblock=T, tile=tl)
            timed(bc, lambda: (sv.step(rho, 1.0, dt, nsub), sv.accel(g)), n ** 3 * nsub)
            runs[(T, tl)] = res.pop(bc)
            sv.close()
        pick = min(runs, key=lambda k: runs[k]["ms_per_hydro_step"])
        res[bc] = dict(runs[pick], substeps_per_launch=pick[0], tile=pick[1],
                       autotuner_pick={"substeps_per_launch": best, "tile": tile,
                                       "ms_per_hydro_step": runs[(best, tile)]["ms_per_hydro_step"]},
                       one_per_launch_ms_per_hydro_step=runs[(1, 0)]["ms_per_hydro_step"])
    # the local boundaries at 512^3, where a streamed substep is bound by HBM
    # (at 256^3 a field fits the last-level cache and streaming gains from
    # it): one substep per launch against four fused
    n5 = 512
    rho5 = workloads.blob_density_torch(n5, workloads.blob_params(0, 8), dev, torch.float32)
    g5 = [torch.empty((n5, n5, n5), dtype=torch.float32, device=dev) for _ in range(3)]
    dt5 = 0.4 * 2.0 / n5
    for bc in ("robin", "outgoing", "periodic"):
        for T, tile in ((1, 0), (4, 1)):
            sv = hgs.Solver(n5, storage="f32", lmax=4, eta=0.0, bc=bc, device=dev, tblock=T, tile=tile)
            label = f"{bc}_512_t{T}"
            timed(label, lambda: (sv.step(rho5, 1.0, dt5, nsub), sv.accel(g5)), n5 ** 3 * nsub)
            res[label]["substeps_per_launch"] = T
            sv.close()
    del rho5, g5
    e = 32
    ex = hgs.ExtendedSolver(n, e, bc="outgoing", storage="f32", lmax=4, eta=0.0, device=dev)
    timed("extended_outgoing_ext32", lambda: (ex.step(rho, 1.0, dt, nsub), ex.accel()), (n + 2 * e) ** 3 * nsub)
    res["extended_outgoing_ext32"]["grid"] = n + 2 * e
    ex.close()
    for ec, lv in ((16, 2), (64, 2), (16, 3)):
        ns = hgs.NestedSolver(n, ec, bc="robin", storage="f32", eta=0.0, device=dev, levels=lv)
        label = f"nested_robin_ext{ec}" if lv == 2 else f"nested{lv}_robin_ext{ec}"
        timed(label, lambda: (ns.step(rho, 1.0, dt, nsub), ns.accel(g)), n ** 3 * nsub)
        res[label]["coarse_grids"] = [t.shape[0] for t in ns.solvers[1:]]
        ns.close()
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    cs = 0.05 + 0.05 * torch.rand((n, n, n), device=dev, generator=gen)
    v = [0.05 * torch.randn((n, n, n), device=dev, generator=gen) for _ in range(3)]
    sv = hgs.Solver(n, storage="f32", lmax=4, eta=0.0, device=dev)
    info = {}

    def driver():
        info["step"] = sv.hydro_step(rho, cs, v, k_g=5.0, courant_hydro=0.3, courant_grav=0.3)
        sv.accel(g)

    driver()
    timed("driver_kg5", driver, n ** 3 * info["step"][1])
    res["driver_kg5"]["nsub"] = info["step"][1]
    sv.close()
    return res


def run_domain_study(dev, n=128):
    """Sec. 4 / Table I style: error of the converged potential against the
    closed-form free-space one, for the outer boundary at the hydro faces
    (Robin), pushed out by an extended gravity-only grid or by one to three
    nested coarse levels, and for the multipole Dirichlet boundary.  Two Gaussians off the
    expansion centre on n^3 over [-1, 1]^3, FP64 storage, each run damped
    (eta for the slowest mode of its outermost grid) for 60 e-folds of that
    mode.  Reported per run: the paper's average relative error (Eq. 6) and
    the largest relative error over the hydro region, R_b of the final state,
    the substeps and the GPU time."""
    import math

    import torch

    from paper_1602_05700_amd import hgs

    dx = 2.0 / n
    dt = 0.4 * dx
    ax = -1.0 + (torch.arange(n, device=dev, dtype=torch.float64) + 0.5) * dx
    Z, Y, X = torch.meshgrid(ax, ax, ax, indexing="ij")
    rho = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    exact = torch.zeros_like(rho)
    for (cx, cy, cz), a0, sg in (((0.35, 0.1, 0.0), 1.0, 0.2), ((-0.3, -0.2, 0.15), 0.6, 0.16)):
        r = torch.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2)
        rho += a0 * torch.exp(-0.5 * r ** 2 / sg ** 2)
        mass = a0 * (2.0 * math.pi) ** 1.5 * sg ** 3
        exact += -mass * torch.erf(r / (math.sqrt(2.0) * sg)) / r
    del X, Y, Z

    def errors(phi):
        d = (phi - exact) / exact
        return float(torch.sqrt(torch.mean(d * d))), float(torch.max(torch.abs(d)))

    def robin_eta(half):  # slowest Robin mode of a box of half-width `half`, critically damped
        return 2.0 * math.sqrt(0.66) * math.pi / (2.0 * half)

    out = {}

    def record(label, run, potential, residual, substeps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        eq6, mx = errors(potential())
        out[label] = {"eq6": eq6, "max_rel": mx, "R_b": float(residual()[0]), "substeps": substeps,
                      "ms": round(e0.elapsed_time(e1), 2)}

    lam = 3.0 * (4.0 / dx ** 2) * math.sin(math.pi / (2 * (n + 1))) ** 2
    eta = 2.0 * math.sqrt(lam)
    steps = int(60.0 / (eta * dt))
    sv = hgs.Solver(n, storage="f64", lmax=4, eta=eta, bc="multipole", device=dev)
    record("multipole_dirichlet", lambda: sv.step(rho, 1.0, dt, steps), lambda: sv.potential(False)[0],
           lambda: sv.residual(rho), steps)
    sv.close()
    for e in (0, 16, 32, 64):
        eta = robin_eta(1.0 + e * dx)
        steps = int(60.0 / (eta * dt))
        ex = hgs.ExtendedSolver(n, e, bc="robin", storage="f64", eta=eta, device=dev)
        record("robin_at_faces" if e == 0 else f"extended_e{e}", lambda: ex.step(rho, 1.0, dt, steps),
               lambda: ex.potential(False)[0], lambda: ex.residual(rho), steps)
        ex.close()
    half = {"robin_at_faces": 1.0, **{f"extended_e{e}": 1.0 + e * dx for e in (16, 32, 64)}}
    for ec, lv in ((8, 2), (16, 2), (32, 2), (16, 3), (16, 4)):
        hw = 1.0 + sum(ec * 2 ** (k + 1) * dx for k in range(lv - 1))  # half-width of the outermost level
        label = f"nested_e{ec}" if lv == 2 else f"nested{lv}_e{ec}"
        half[label] = hw
        eta = robin_eta(hw)
        calls = int(60.0 / (eta * dt)) // 8 + 1
        ns = hgs.NestedSolver(n, ec, bc="robin", storage="f64", eta=eta, device=dev, levels=lv)

        def run_nested():
            for _ in range(calls):
                ns.step(rho, 1.0, dt, 8)

        record(label, run_nested, lambda: ns.potential(False)[0], lambda: ns.fine.residual(rho), calls * 8)
        ns.close()
    return {"grid": n, "storage": "f64", "reference": "closed-form free-space potential of two Gaussians",
            "boundary_half_width": half, "runs": out}


def run_warmstart(dev, count=8, n=128, tol=1e-4):
    """Substeps of the critically damped FP32 solver to R_b < tol on 128^3
    blob mixtures (held-out seeds 20000..), from the zero start and from the
    learned start with the committed weights (zero start as fallback); the
    coarse cue that feeds the network (the direct Poisson solve on the n/4
    grid) is counted in fine-substep equivalents.  Wall time as well: one
    density's prediction (restriction, coarse solve, features, network,
    prolongation; replayed from a captured graph), the fallback check
    (start_solver: ghosts, residual, the decision on the device) and the median learned
    substep count, against the median zero-start count, each timed with
    events from the first launch to the last."""
    import numpy as np
    import torch

    import workloads
    from paper_1602_05700_amd import hgs, warmstart as ws

    if not os.path.exists(ws.WEIGHTS):
        return {"skipped": "no trained weights in the package"}
    net = ws.Net.load(ws.WEIGHTS, dev)
    feats = ws.Features(n, dev, coarse_steps=net.coarse_steps)
    seeds = list(range(20000, 20000 + count))
    rho = torch.stack([workloads.blob_density_torch(n, workloads.warmstart_blobs(s), dev, torch.float32)
                       for s in seeds])
    planar, phi2, scale = feats.inputs(rho)
    phi, pd = ws.predict_fine(net, planar, phi2, scale, n)
    zero, learned, fallback = [], [], 0
    for i in range(count):
        z = ws.steps_to_tolerance(rho[i], n, tol)
        # the start goes through start_solver: on a fallback the substeps are
        # counted from the zero start, and the prediction is counted either way
        w = ws.steps_to_tolerance(rho[i], n, tol, start=(phi[i], pd[i]))
        zero.append(z[0])
        fallback += 0 if w[3] else 1
        learned.append(w[0] + feats.coarse_cost_fine_steps)
    mz, ml = float(np.median(zero)), float(np.median(learned))

    # wall time, density 0: prediction for one density, then the substeps
    dx = 2.0 / n
    dt = 0.4 * dx
    eta = ws.eta_critical(n, dx)
    r0 = rho[0].contiguous()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def solve(start, nsub):
        s = hgs.Solver(n, storage="f32", lmax=4, eta=eta, device=dev)
        if start is not None:
            s.set_state(start[0], start[1], dt)
        return s

    n_l = int(round(np.median([v - feats.coarse_cost_fine_steps for v in learned])))
    predictor = ws.Predictor(net, n, B=1, device=dev)  # the prediction captured in a graph
    for rep in range(3):  # the first passes warm up
        s = solve(None, 0)  # created outside the timed region, as for the zero start
        torch.cuda.synchronize()
        e[0].record()
        f_phi, f_pd = predictor(r0[None])
        e[1].record()
        # the fallback check (ghosts, residual, the decision on the device) is timed too
        kept = ws.start_solver(s, r0, f_phi[0].contiguous(), f_pd[0].contiguous(), dt)
        e[2].record()
        s.step(r0, 1.0, dt, n_l)
        e[3].record()
        torch.cuda.synchronize()
        assert kept.item() == 1, "the timed density fell back to the zero start"
        s.close()
    predict_ms = e[0].elapsed_time(e[1])
    check_ms = e[1].elapsed_time(e[2])
    learned_ms = e[0].elapsed_time(e[3])
    s = solve(None, 0)
    torch.cuda.synchronize()
    e[0].record()
    s.step(r0, 1.0, dt, int(mz))
    e[1].record()
    torch.cuda.synchronize()
    zero_ms = e[0].elapsed_time(e[1])
    s.close()
    return {"grid": n, "densities": count, "seeds": f"{seeds[0]}..{seeds[-1]}", "tol_Rb": tol,
            "steps_zero_median": mz, "steps_learned_median": round(ml, 2), "ratio": round(mz / ml, 3),
            "fallback": fallback, "coarse_cue": feats.coarse, "coarse_cost_fine_steps": feats.coarse_cost_fine_steps,
            "wall_ms_zero": round(zero_ms, 3), "wall_ms_learned": round(learned_ms, 3),
            "wall_ms_predict": round(predict_ms, 3), "wall_ms_fallback_check": round(check_ms, 3),
            "wall_ratio": round(zero_ms / learned_ms, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nsub", type=int, default=4)
    ap.add_argument("--tblock", type=int, default=0, help="substeps per fused launch (0 = autotune)")
    ap.add_argument("--tile", type=int, default=0, help="tile shape index with --tblock (hgs_tile_shape)")
    ap.add_argument("--storage", choices=("f32", "f64"), default="f32",
                    help="storage of the headline run (f32: the headline configuration; f64 for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-grid batched measurement")
    ap.add_argument("--batch-substeps", type=int, default=500,
                    help="substeps per hydro step of the batched measurement (fewer for profiler runs)")
    ap.add_argument("--no-warmstart", action="store_true", help="skip the steps-to-1e-4 warm-start measurement")
    ap.add_argument("--no-configs", action="store_true", help="skip the 64^3 sphere and 256^3 rotating-blob runs")
    ap.add_argument("--no-study", action="store_true", help="skip the boundary-placement error study")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy five times (for scaling HBM counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch

        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4, "copies": 5}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition is "
              "described in the design notes but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_1602_05700_amd import hgs

    dev = torch.device("cuda:0")
    n, nsub, K, W = args.n, args.nsub, args.steps, args.warmup
    dx = 2.0 / n
    c_g = 1.0
    dt = 0.4 * dx / c_g
    omega = 0.1 * c_g / 1.0  # speed 0.1 c_g at cylindrical radius 1
    blobs = workloads.blob_params(1, 16)
    storage = args.storage
    tdt = torch.float32 if storage == "f32" else torch.float64
    log(f"[bench] generating {W + K} rotated densities {n}^3 {storage} on the GPU")
    rhos = [workloads.blob_density_torch(n, blobs.rotated(omega * nsub * dt * h), dev, tdt)
            for h in range(W + K)]
    tune = None
    tblock, tile = args.tblock, args.tile
    if tblock == 0:
        best, best_tile, times = hgs.autotune(n, rhos[0], c_g, dt, nsub, storage=storage, lmax=4, device=dev)
        tune = {"best_tblock": best, "best_tile": tile_desc(storage, best, best_tile), "ms_per_substep": times}
        tblock, tile = best, best_tile
        log(f"[bench] autotune: depth {best}, tile {tune['best_tile']}, ms per substep {times}")
    s = hgs.Solver(n, storage=storage, lmax=4, eta=0.0, tblock=tblock, tile=tile, device=dev)
    out = [torch.empty((n, n, n), dtype=tdt, device=dev) for _ in range(3)]
    stream = s.stream
    # start: the converged potential of the first density (critically damped
    # relaxation) and the time derivative of rigid rotation about z,
    # dphi/dt = -omega (x d/dy - y d/dx) phi; then the undamped Eq. (2)
    log(f"[bench] converged start: {CONVERGE_SUBSTEPS} critically damped substeps")
    lam = 3 * (4 / dx ** 2) * math.sin(math.pi / (2 * (n + 1))) ** 2
    sc = hgs.Solver(n, storage=storage, lmax=4, eta=2.0 * c_g * math.sqrt(lam), device=dev)
    sc.step(rhos[0], c_g, dt, CONVERGE_SUBSTEPS)
    start_res = sc.residual(rhos[0])
    phi_c = sc.potential(with_phidot=False)[0]
    sc.close()
    ax = -1.0 + (torch.arange(n, device=dev, dtype=tdt) + 0.5) * dx
    dpy, dpx = torch.gradient(phi_c, spacing=dx, dim=(1, 2))
    pd0 = -omega * (ax[None, None, :] * dpy - ax[None, :, None] * dpx)
    pd0 = pd0.contiguous()
    s.set_state(phi_c, pd0, dt)
    # settle: after the set-up's host-side work (tens of ms of light load) the
    # first dozen or so fused launches ran up to 30% slower in a kernel trace
    # (992 us falling to a steady 752 us over about 15 launches), so
    # SETTLE_STEPS untimed hydro steps run first and the start state is then
    # restored
    log(f"[bench] settle {SETTLE_STEPS} hydro steps, start state restored")
    for _ in range(SETTLE_STEPS):
        s.step(rhos[0], c_g, dt, nsub)
        s.accel(out)
    s.set_state(phi_c, pd0, dt)
    del phi_c, dpy, dpx, pd0

    log(f"[bench] warmup {W} hydro steps, tblock {s.tblock}")
    for h in range(W):
        s.step(rhos[h], c_g, dt, nsub)
        s.accel(out)
    torch.cuda.synchronize()

    s.timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for h in range(K):
        s.step(rhos[W + h], c_g, dt, nsub)
        s.accel(out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    end_res = s.residual(rhos[W + K - 1])
    st = s.timing_read("stencil")
    mp = s.timing_read("multipole")
    gr = s.timing_read("gradient")
    s.timing(False)
    log(f"[bench] {K} hydro steps: events {ms:.3f} ms, wall {wall * 1e3:.3f} ms")
    for name, d in (("stencil", st), ("multipole", mp), ("gradient", gr)):
        if d["launches"]:
            log(f"[bench]   {name}: {d['launches']} launches, {d['ms'] / d['launches'] * 1e3:.1f} us avg, "
                f"{d['bytes'] / d['ms'] / 1e6:.0f} GB/s algorithmic")

    updates = K * nsub * n ** 3
    value = updates / (ms / 1e3) / 1e9
    per_launch_bytes = st["bytes"] / st["launches"]
    avg_s = st["ms"] / st["launches"] / 1e3
    achieved = per_launch_bytes / avg_s / 1e9
    kname = ("leapfrog_stream" if s.tblock == 1 else f"leapfrog_tblock{s.tblock}") + ("_f64" if storage == "f64" else "")
    traffic = counter_traffic(kname, n ** 3, s.tile if s.tblock > 1 else 0)
    line = {
        "metric": "Gcell-updates/s + %HBM roofline; steps to 1e-4 residual, plain vs learned",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 (storage and substeps; f64 moments, boundary and gradient)" if storage == "f32"
                  else "f64"),
        "data": "synthetic",
        "config": {
            "workload": f"hyperbolic gravity, {n}^3 grid, 16 rotating Gaussian blobs, {storage.upper()} storage, lmax 4, "
                        f"{nsub} substeps per hydro step, moments+ghosts+substeps+gradient, from the converged "
                        "potential with the rotation's time derivative",
            "grid": n, "nsub": nsub, "tblock": s.tblock, "tile": tile_desc(storage, s.tblock, s.tile), "lmax": 4,
            "blobs": 16,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": per_launch_bytes,
            "avg_launch_us": round(avg_s * 1e6, 2),
        },
        "autotune": tune,
        "state": {
            "start_R_b": float(start_res[0]), "start_R_f": float(start_res[1]),
            "end_R_b": float(end_res[0]), "end_R_f": float(end_res[1]),
            "note": "residuals of the discrete Eq. (1) for the current density: after the converged start, and "
                    "after the timed hydro steps of the undamped wave equation tracking the rotating density",
        },
        "kernels_us_per_step": {
            "stencil": round(st["ms"] / K * 1e3, 1),
            "multipole": round(mp["ms"] / K * 1e3, 1),
            "gradient": round(gr["ms"] / K * 1e3, 1),
        },
    }
    # the timed block again, five times, for its run-to-run spread (same
    # densities in the same order; the work does not depend on the values)
    reps = []
    for _ in range(5):
        torch.cuda.synchronize()
        e0.record(stream)
        for h in range(K):
            s.step(rhos[W + h], c_g, dt, nsub)
            s.accel(out)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(round(updates / (e0.elapsed_time(e1) / 1e3) / 1e9, 3))
    line["repeat_blocks"] = {"blocks": len(reps), "steps_each": K, "Gcell_updates_per_s": reps,
                             "median": sorted(reps)[len(reps) // 2]}
    log(f"[bench] five more blocks of {K} hydro steps: {reps} Gcell-updates/s")
    del rhos
    if not args.no_batched:
        log(f"[bench] batched: 64 uneven grids, {args.batch_substeps} substeps")
        line["batched"] = run_batched(dev, nsub=args.batch_substeps)
        log(f"[bench]   {line['batched']}")
    if not args.no_configs:
        log("[bench] smaller configurations: 64^3 sphere (FP64), 256^3 rotating blobs (FP64, FP32)")
        line["configs"] = run_configs(dev)
        log(f"[bench]   {line['configs']}")
    if not args.no_study:
        log("[bench] boundary study at 128^3: converged error against the free-space potential")
        line["domain_study"] = run_domain_study(dev)
        log(f"[bench]   {line['domain_study']}")
    if not args.no_warmstart:
        log("[bench] warm start: steps to R_b < 1e-4 at 128^3, zero vs learned")
        line["warm_start"] = run_warmstart(dev)
        log(f"[bench]   {line['warm_start']}")
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle, one hydro step) and the GPU's error against it")
        rho0 = workloads.blob_density_torch(n, blobs.rotated(omega * nsub * dt * W), dev, torch.float32)
        # the same hydro step on the GPU from the same smooth non-zero start
        ax = -1.0 + (torch.arange(n, device=dev, dtype=torch.float64) + 0.5) * dx
        phi0 = (-1.0 / torch.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2
                                  + 0.09)).to(torch.float32)
        v = hgs.Solver(n, storage="f32", lmax=4, eta=0.0, tblock=s.tblock, device=dev)
        v.set_state(phi0, None, dt)
        v.step(rho0, c_g, dt, nsub)
        gpu = [v.potential(with_phidot=False)[0].cpu().numpy()] + [a.cpu().numpy() for a in v.accel()]
        v.close()
        line["cpu_baseline"] = cpu_baseline(rho0.cpu().numpy(), n, nsub, dt, phi0.cpu().numpy(), gpu)
        log(f"[bench]   {line['cpu_baseline']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
