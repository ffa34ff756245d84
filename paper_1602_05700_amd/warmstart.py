"""Learned warm start for the hyperbolic solver (orchestration only: every
array operation runs in libhgs.so kernels through the hgs binding).

The paper starts its runs from a Poisson solution or an interpolated exact one
(Sec. 2).  Here a start for (phi, dphi/dt) on a fine grid is predicted instead:

  1. rho (fine, n^3) is restricted to n/2 and n/4 (2x2x2 means);
  2. the steady state of the wave equation on the n/4 grid (the discrete
     Poisson solution with the multipole boundary, by the library's direct
     sine-transform solve; the network was trained on a 200-substep critically
     damped solve, which reaches it to ~1e-5) gives a coarse potential,
     prolonged to n/2 -- the global cue a local network cannot build by itself;
  3. a 4-layer 3x3x3 convolution network (16 channels, tanh, bf16 weights and
     activations, FP32 accumulation) maps (rho, coarse phi, the coarse phi's
     residual of the discrete Eq. 1) at n/2 to a correction of phi and to
     dphi/dt, in units scaled by max(rho) because phi is linear in rho;
  4. the n/2 prediction is prolonged to n and handed to hgs_set_state.

The zero start stays the fallback: start_solver() sets the predicted start
and keeps it only if its residual R_b is below the zero start's (which is 1),
else it resets the solver to zero.  Steps to a residual tolerance count fine
substeps; the coarse cue is reported in fine-step equivalents: a damped solve
costs (n/4)^3 / n^3 of a fine substep per coarse substep, the direct solve its
6 (n/4)^4 multiply-adds against ~6 n^3 per fine substep, (n/4)^4 / n^3.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import hgs

NC = hgs.NN_CHANNELS
N_LAYERS = 4
IN_CH = 3   # rho, coarse phi, its residual of the discrete Poisson equation
OUT_CH = 2  # phi correction, dphi/dt


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_weights.npz")


def lambda_min(n: int, dx: float) -> float:
    """Slowest Dirichlet mode of the 7-point Laplacian on an n^3 grid."""
    return 3.0 * (4.0 / dx ** 2) * math.sin(math.pi / (2.0 * (n + 1))) ** 2


def eta_critical(n: int, dx: float, c: float = 1.0) -> float:
    return 2.0 * c * math.sqrt(lambda_min(n, dx))


@dataclass
class Net:
    """Parameters: FP32 masters (w: (27,16,16), b: (16,)) per layer, bfloat16
    copies of the weights, Adam moments."""

    device: object
    w: list = field(default_factory=list)
    b: list = field(default_factory=list)
    w16: list = field(default_factory=list)
    mw: list = field(default_factory=list)
    vw: list = field(default_factory=list)
    mb: list = field(default_factory=list)
    vb: list = field(default_factory=list)
    t: int = 0
    out_scale: float = 1.0
    coarse_steps: int = 200  # length of the coarse solve the network was trained with

    @staticmethod
    def create(device, seed: int = 0) -> "Net":
        import torch

        net = Net(device)
        g = torch.Generator().manual_seed(seed)
        for layer in range(N_LAYERS):
            cin = IN_CH if layer == 0 else NC
            cout = OUT_CH if layer == N_LAYERS - 1 else NC
            w = torch.zeros((27, NC, NC), dtype=torch.float32)
            std = math.sqrt(1.0 / (27 * cin))
            w[:, :cout, :cin] = torch.randn((27, cout, cin), generator=g) * std
            if layer == N_LAYERS - 1:
                w *= 0.1
            net.w.append(w.to(device))
            net.b.append(torch.zeros(NC, dtype=torch.float32, device=device))
            net.w16.append(net.w[-1].to(torch.bfloat16))
            for lst in (net.mw, net.vw):
                lst.append(torch.zeros_like(net.w[-1]))
            for lst in (net.mb, net.vb):
                lst.append(torch.zeros_like(net.b[-1]))
        return net

    def state_dict(self) -> dict:
        d = {"out_scale": np.array(self.out_scale), "coarse_steps": np.array(self.coarse_steps)}
        for i in range(N_LAYERS):
            d[f"w{i}"] = self.w[i].cpu().numpy()
            d[f"b{i}"] = self.b[i].cpu().numpy()
        return d

    def load_state_dict(self, d: dict) -> None:
        import torch

        self.out_scale = float(d["out_scale"])
        if "coarse_steps" in d:
            self.coarse_steps = int(d["coarse_steps"])
        for i in range(N_LAYERS):
            self.w[i] = torch.from_numpy(np.asarray(d[f"w{i}"], dtype=np.float32)).to(self.device)
            self.b[i] = torch.from_numpy(np.asarray(d[f"b{i}"], dtype=np.float32)).to(self.device)
            self.w16[i] = self.w[i].to(torch.bfloat16)

    def save(self, path: str) -> None:
        np.savez(path, **self.state_dict())

    @staticmethod
    def load(path: str, device) -> "Net":
        net = Net.create(device)
        with np.load(path, allow_pickle=False) as d:
            net.load_state_dict({k: d[k] for k in d.files})
        return net

    # -- forward / backward on packed inputs x: (B, Z, Y, X, 16) bf16
    def forward(self, x):
        import torch

        acts = [x]
        for i in range(N_LAYERS):
            last = i == N_LAYERS - 1
            out = torch.empty(x.shape, dtype=torch.float32 if last else torch.bfloat16, device=x.device)
            hgs.nn_conv3d(acts[-1], self.w16[i], self.b[i], out, hgs.NN_F32 if last else hgs.NN_TANH_BF16)
            acts.append(out)
        return acts

    def backward(self, acts, g_out, ws=None):
        """g_out: bf16 gradient of the loss w.r.t. the last layer's output.
        Returns [(dw, db)] per layer."""
        import torch

        grads = [None] * N_LAYERS
        g = g_out
        wt = torch.empty_like(self.w16[0])
        for i in range(N_LAYERS - 1, -1, -1):
            dw = torch.empty((27, NC, NC), dtype=torch.float32, device=g.device)
            db = torch.empty(NC, dtype=torch.float32, device=g.device)
            ws = hgs.nn_wgrad(acts[i], g, dw, db, ws)
            grads[i] = (dw, db)
            if i > 0:
                hgs.nn_flip_weights(self.w16[i], wt)
                gn = torch.empty(g.shape, dtype=torch.bfloat16, device=g.device)
                hgs.nn_conv3d(g, wt, None, gn, hgs.NN_DTANH_BF16, aux=acts[i])
                g = gn
        return grads, ws

    def adam_step(self, grads, lr: float):
        self.t += 1
        for i, (dw, db) in enumerate(grads):
            hgs.nn_adam(self.w[i], self.mw[i], self.vw[i], dw, self.w16[i], lr, self.t)
            hgs.nn_adam(self.b[i], self.mb[i], self.vb[i], db, None, lr, self.t)


class Features:
    """Coarse cue and packed network inputs for a set of fine densities."""

    def __init__(self, n: int, device, coarse_steps: int = 200, lmax: int = 4, coarse: str = "direct"):
        if coarse not in ("direct", "relax"):
            raise ValueError(f"unknown coarse solve {coarse!r}")
        self.n, self.device, self.coarse_steps, self.lmax, self.coarse = n, device, coarse_steps, lmax, coarse
        self.nh, self.nq = n // 2, n // 4
        self._batches = {}
        self._direct = None

    def restrict(self, rho):
        """rho: (B, n, n, n) fp32 -> (rho at n/2, rho at n/4)."""
        import torch

        B = rho.shape[0]
        r2 = torch.empty((B, self.nh, self.nh, self.nh), dtype=rho.dtype, device=rho.device)
        hgs.nn_restrict2(rho, r2)
        r4 = torch.empty((B, self.nq, self.nq, self.nq), dtype=rho.dtype, device=rho.device)
        hgs.nn_restrict2(r2, r4)
        return r2, r4

    def bind_stream(self, stream) -> None:
        """Issue the coarse solves on `stream` (the library calls go to a
        solver's own stream; a captured prediction needs the capture stream)."""
        import torch

        m = self.nq
        self._direct = (hgs.Solver(m, storage="f32", lmax=self.lmax, device=self.device, stream=stream),
                        torch.empty(2 * m ** 3, dtype=torch.float64, device=self.device))

    def coarse_phi(self, r4):
        """Coarse potentials on the n/4 grids, prolonged to n/2: the direct
        Poisson solve of each coarse density (coarse = "direct"), or the damped
        solve the network was trained on (coarse = "relax")."""
        import torch

        B, m = r4.shape[0], self.nq
        if self.coarse == "direct":
            if self._direct is None:
                self._direct = (hgs.Solver(m, storage="f32", lmax=self.lmax, device=self.device),
                                torch.empty(2 * m ** 3, dtype=torch.float64, device=r4.device))
            sv, scratch = self._direct
            phi4 = torch.empty((B, m, m, m), dtype=torch.float32, device=r4.device)
            for i in range(B):
                sv.poisson_direct(r4[i], scratch)
                sv.potential(with_phidot=False, out=phi4[i])
            phi2 = torch.empty((B, self.nh, self.nh, self.nh), dtype=torch.float32, device=r4.device)
            hgs.nn_prolong2(phi4, phi2)
            return phi2
        dx = 2.0 / m
        if B not in self._batches:
            # two substeps per fused launch: on 32^3 grids a launch is bound by
            # its pipeline fill, and depth 2 is the fastest (200 substeps, one
            # grid: 0.91 ms against 1.07 ms at depth 4 and 4.8 ms streaming);
            # every depth gives bit-identical states
            self._batches[B] = (hgs.Batch([m] * B, storage="f32", lmax=self.lmax, eta=eta_critical(m, dx),
                                          tblock=2, device=self.device),
                                torch.zeros((m, m, m), dtype=torch.float32, device=r4.device))
        b, zero = self._batches[B]
        for g in b.grids:
            g.set_state(zero, None, 0.4 * dx)
        rhos = [r4[i].contiguous() for i in range(B)]
        b.step(rhos, 1.0, 0.4 * dx, self.coarse_steps)
        phi4 = torch.stack([g.potential(with_phidot=False)[0] for g in b.grids])
        phi2 = torch.empty((B, self.nh, self.nh, self.nh), dtype=torch.float32, device=r4.device)
        hgs.nn_prolong2(phi4, phi2)
        return phi2

    @property
    def coarse_cost_fine_steps(self) -> float:
        if self.coarse == "direct":
            return self.nq ** 4 / self.n ** 3
        return self.coarse_steps * (self.nq / self.n) ** 3

    def inputs(self, rho):
        """Planar network inputs (B, 3, n/2^3) fp32, the coarse phi at n/2 and the
        per-sample scale max|rho| (B,) fp32.  rho: (B, n, n, n) fp32, positive
        somewhere in every sample."""
        import torch

        B = rho.shape[0]
        r2, r4 = self.restrict(rho)
        phi2 = self.coarse_phi(r4)
        scale = torch.empty(B, dtype=torch.float32, device=rho.device)
        if B <= hgs.NN_MAXABS_NOALLOC_MAX_B:
            hgs.nn_maxabs_noalloc(rho, scale)  # no scratch buffer: capturable as it is
        else:
            hgs.nn_maxabs(rho, scale)
        h = 2.0 * (2.0 / self.n)
        planar = torch.empty((B, IN_CH) + tuple(r2.shape[1:]), dtype=torch.float32, device=rho.device)
        hgs.nn_features(r2, phi2, scale, 4.0 * math.pi * h * h, planar)
        return planar, phi2, scale


def pack(planar):
    import torch

    B = planar.shape[0]
    x = torch.empty((B,) + tuple(planar.shape[2:]) + (NC,), dtype=torch.bfloat16, device=planar.device)
    hgs.nn_pack(planar, x)
    return x


def predict_fine(net: Net, planar, phi2, scale, n: int):
    """Fine-grid start (phi, phidot) (B, n, n, n) fp32 from the network."""
    import torch

    B = planar.shape[0]
    x = pack(planar)
    out = net.forward(x)[-1]
    phi2f = torch.empty_like(phi2)
    pd2 = torch.empty_like(phi2)
    hgs.nn_compose(phi2, out, scale, net.out_scale, phi2f, pd2)
    phi2 = phi2f
    phi = torch.empty((B, n, n, n), dtype=torch.float32, device=planar.device)
    pd = torch.empty_like(phi)
    hgs.nn_prolong2(phi2, phi)
    hgs.nn_prolong2(pd2, pd)
    return phi, pd


class Predictor:
    """The whole prediction for B densities of n^3 cells -- restriction, the
    coarse direct solve, features, the network, composition and prolongation
    (about two dozen library launches) -- captured once into a HIP graph and
    replayed, so its cost is the kernels' and not their launches'.  The input
    is copied into a buffer the graph reads; the outputs are buffers the graph
    writes (overwritten by the next call)."""

    def __init__(self, net: Net, n: int, B: int = 1, device="cuda"):
        import torch

        self.net, self.n, self.B = net, n, B
        self.stream = torch.cuda.Stream(device=device)
        self.feats = Features(n, device, coarse_steps=net.coarse_steps)
        self.feats.bind_stream(self.stream)
        self.rho = torch.zeros((B, n, n, n), dtype=torch.float32, device=device)
        self.rho.fill_(1.0)
        with torch.cuda.stream(self.stream):
            # eager pass first: the library and torch allocate what they need
            # outside the capture
            planar, phi2, scale = self.feats.inputs(self.rho)
            predict_fine(net, planar, phi2, scale, n)
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            planar, phi2, scale = self.feats.inputs(self.rho)
            self.phi, self.pd = predict_fine(net, planar, phi2, scale, n)

    def __call__(self, rho):
        """rho: (B, n, n, n) fp32 -> (phi, phidot), (B, n, n, n) fp32 each,
        ordered on the current stream."""
        import torch

        cur = torch.cuda.current_stream(self.rho.device)
        self.rho.copy_(rho)
        self.stream.wait_stream(cur)
        self.graph.replay()
        cur.wait_stream(self.stream)
        return self.phi, self.pd


def start_solver(solver, rho, phi, phidot, dt: float):
    """Hand a predicted start (phi, phidot) to the solver, with the zero start
    as the fallback: the start is kept if its residual R_b (the residual of
    the discrete Eq. 1 relative to the linear system's right-hand side, with
    the multipole boundary of rho) is below the zero start's, which is 1 by
    construction; otherwise the solver is reset to the zero start.  Decided on
    the device in stream order (hgs_keep_start_if_better): returns a device
    int32 tensor holding 1 (kept) or 0 (reset), read without blocking the
    stream's work."""
    import torch

    solver.set_state(phi, phidot, dt)
    kept = torch.empty(1, dtype=torch.int32, device=phi.device)
    solver.keep_start_if_better(rho, kept)
    return kept


def converged_phi(rhos, n: int, device, steps: int = 1500, storage: str = "f64", lmax: int = 4):
    """Potentials of the damped solver run to convergence (the training targets),
    for a list of (n, n, n) densities; one batch of grids."""
    import torch

    dx = 2.0 / n
    dt_ = torch.float64 if storage == "f64" else torch.float32
    b = hgs.Batch([n] * len(rhos), storage=storage, lmax=lmax, eta=eta_critical(n, dx), device=device)
    b.step([r.to(dt_).contiguous() for r in rhos], 1.0, 0.4 * dx, steps)
    out = [g.potential(with_phidot=False)[0] for g in b.grids]
    res = [g.residual(r.to(dt_).contiguous())[0] for g, r in zip(b.grids, rhos)]
    b.close()
    return out, res


def steps_to_tolerance(rho, n: int, tol: float, start=None, max_steps: int = 4000, check: int = 4,
                       storage: str = "f32", lmax: int = 4, device="cuda", metric: str = "R_b", ref=None):
    """Substeps of the damped fine solver until the criterion falls below tol,
    from zero or from start = (phi, phidot).  metric: "R_b" (the residual
    relative to the linear system's right-hand side, boundary terms
    included), "R_f" (relative to the source alone) or "E" (relative
    distance to the converged potential ref).  A start goes through
    start_solver (the zero start is the fallback).  Returns (steps, criterion
    after the first check, criterion at the end, whether the start was
    kept)."""
    import torch

    if metric not in ("R_b", "R_f", "E"):
        raise ValueError(f"unknown criterion {metric!r}")
    if metric == "E" and ref is None:
        raise ValueError("E needs the converged potential ref")

    dx = 2.0 / n
    dt = 0.4 * dx
    s = hgs.Solver(n, storage=storage, lmax=lmax, eta=eta_critical(n, dx), device=device)
    dtype = s.dtype
    r = rho.to(dtype).contiguous()
    # one step of zero length is not allowed; set the ghosts with a first step of
    # `check` substeps from the chosen start and count those substeps
    kept = None
    if start is not None:
        kept = start_solver(s, r, start[0].to(dtype).contiguous(), start[1].to(dtype).contiguous(), dt)
    if metric == "E":
        ref64 = ref.to(torch.float64)
        ref_norm = float(ref64.norm())
    r0 = None
    steps = 0
    while steps < max_steps:
        s.step(r, 1.0, dt, check)
        steps += check
        if metric == "E":
            rb = float((s.potential(with_phidot=False)[0].to(torch.float64) - ref64).norm()) / ref_norm
        else:
            rb = s.residual(r)[0 if metric == "R_b" else 1]
        if r0 is None:
            r0 = rb
        if rb < tol:
            break
    used = bool(kept.item()) if kept is not None else False
    s.close()
    return steps, r0, rb, used
