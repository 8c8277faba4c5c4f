"""FNO warm start for the Stokes ADMM: data generation by the solver itself,
training with the FNO kernels, and warm-started solves.

The network is trained only on solutions produced by acm_stokes_solve_batched
(g = e_x).  A warm-started solve still runs the unmodified ADMM to the same
tolerance, so the answer is the method's own; the network only changes the
starting iterate (u0 = (1-H) u_pred, q0 = p_pred, a0 = lambda0 from the
fixed-point reaction in the solid).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import inputs as I
from .api import acm_stokes_solve, acm_stokes_solve_batched
from .fno import FNO


def _one_cell(args):
    n, seed, radius_vox, por_lo, por_hi = args
    por = por_lo + (por_hi - por_lo) * I.SplitMix64(seed ^ 0x5DEECE66D).uniform()
    return I.overlapping_spheres(n, radius_vox, por, seed=seed)


def make_cells(n: int, count: int, seed0: int, radius_vox: float, por_lo: float, por_hi: float,
               workers: int = 1):
    """Overlapping-sphere cells with porosity drawn uniformly in [por_lo, por_hi]
    (the draw uses the cell's own SplitMix64 stream).  workers > 1 builds them
    in a process pool: call it only before the process has touched the GPU."""
    jobs = [(n, seed0 + i, radius_vox, por_lo, por_hi) for i in range(count)]
    if workers <= 1 or count < 2 * workers:
        return [_one_cell(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_one_cell, jobs, chunksize=max(1, count // (8 * workers)))


def generate_dataset(cells, eps=1e-6, batch=64, max_iter=200000, log=print):
    """Solve every cell (g = e_x) with the batched solver.  Returns device
    tensors H (B, n, n, n) uint8 and Y (B, 4, n, n, n) float32 = (u, q)."""
    n = cells[0].shape[-1]
    B = len(cells)
    H = torch.from_numpy(np.stack(cells)).cuda()
    Y = torch.empty((B, 4, n, n, n), dtype=torch.float32, device="cuda")
    t0 = time.time()
    iters = []
    for s in range(0, B, batch):
        Hs = [H[i] for i in range(s, min(B, s + batch))]
        us = [Y[i, :3] for i in range(s, min(B, s + batch))]
        qs = [Y[i, 3] for i in range(s, min(B, s + batch))]
        r = acm_stokes_solve_batched(Hs, [(1.0, 0.0, 0.0)] * len(Hs), eps=eps, max_iter=max_iter,
                                     us=us, qs=qs)
        iters += [st["iters"] for st in r["stats"]]
        log(f"[warmstart] solved cells {s}..{s + len(Hs) - 1} ({time.time() - t0:.1f} s)")
    return H, Y, dict(seconds=time.time() - t0, iters=iters)


class Normaliser:
    """Per-channel scale so that the targets have unit RMS."""

    def __init__(self, Y: torch.Tensor):
        self.scale = Y.double().pow(2).mean(dim=(0, 2, 3, 4)).sqrt().float().clamp_min(1e-30)

    def encode(self, Y):
        return Y / self.scale.view(1, -1, 1, 1, 1)

    def decode(self, Z):
        return Z * self.scale.view(1, -1, 1, 1, 1)


def train(net: FNO, H: torch.Tensor, Yn: torch.Tensor, epochs=10, batch=8, lr=1e-3,
          lr_final=1e-4, seed=0, log=print):
    """Adam on the mean-squared error of the normalised targets."""
    B = H.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = max(1, B // batch)
    total = epochs * steps_per_epoch
    dout = torch.empty((batch,) + tuple(Yn.shape[1:]), dtype=torch.float32, device=H.device)
    hist = []
    t0 = time.time()
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(B, generator=g)
        losses = []
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch].to(H.device)
            Hb = H.index_select(0, idx).contiguous()
            Yb = Yn.index_select(0, idx).contiguous()
            out = net.forward(Hb, train=True)
            losses.append(net.mse(out, Yb, dout))
            net.backward(Hb, dout)
            frac = k / max(1, total - 1)
            net.adam(lr=lr * (lr_final / lr) ** frac)
            k += 1
        hist.append(float(np.mean(losses)))
        log(f"[warmstart] epoch {ep}: loss {hist[-1]:.4e} ({time.time() - t0:.1f} s)")
    return dict(loss=hist, seconds=time.time() - t0, steps=k)


def predict(net: FNO, norm: Normaliser, H: torch.Tensor):
    """(u_pred (3, n, n, n), p_pred (n, n, n)) for one cell H (n, n, n)."""
    out = net.forward(H.unsqueeze(0).contiguous(), train=False)
    Y = norm.decode(out)[0]
    return Y[:3].contiguous(), Y[3].contiguous()


def relative_error(net: FNO, norm: Normaliser, H: torch.Tensor, Y: torch.Tensor) -> float:
    """Relative L2 error of the predicted velocity over a set of cells."""
    num = den = 0.0
    for i in range(H.shape[0]):
        u, _ = predict(net, norm, H[i])
        num += float((u - Y[i, :3]).double().pow(2).sum())
        den += float(Y[i, :3].double().pow(2).sum())
    return (num / den) ** 0.5


def solve_plain_and_warm(net: FNO, norm: Normaliser, H: torch.Tensor, eps=1e-6, max_iter=400000):
    """Plain (zero start) and FNO-warm-started ADMM solves of one cell, g = e_x."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp = acm_stokes_solve(H, (1.0, 0.0, 0.0), eps=eps, max_iter=max_iter, want_q=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    u0, p0 = predict(net, norm, H)
    rw = acm_stokes_solve(H, (1.0, 0.0, 0.0), eps=eps, max_iter=max_iter, u=u0, q=p0,
                          warm_start=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kp = float(rp["u"][0].double().mean())
    kw = float(rw["u"][0].double().mean())
    return dict(plain_iters=rp["stats"]["iters"], warm_iters=rw["stats"]["iters"],
                plain_s=t1 - t0, warm_s=t2 - t1, k_plain=kp, k_warm=kw,
                k_rel_diff=abs(kw - kp) / max(abs(kp), 1e-300),
                converged=bool(rp["stats"]["converged"] and rw["stats"]["converged"]))
