"""Parameter sweeps of the solvers (the shape of the paper's penalty and
comparison-medium studies, Section 4.1 and Section 4.2), on synthetic cells.

Each sweep runs the HIP solvers only; nothing here computes the method."""
from __future__ import annotations

import torch

from . import abi
from .api import acm_stokes_solve, acm_transport_step


def penalty_sweep(H: torch.Tensor, g=(1.0, 0.0, 0.0), factors=(0.25, 0.5, 1.0, 2.0, 4.0),
                  which: str = "b", eps: float = 1e-5, max_iter: int = 20000) -> dict:
    """ADMM iterations to eps with fixed penalties, one of alpha, beta, b
    scaled by each factor from its default nu/h (the others at nu/h), and
    with the adaptive schedule (Section 4.1, eq. varying algorithm)."""
    n = max(H.shape)
    p0 = float(n)  # nu / h with nu = 1, h = 1/n
    out = {"which": which, "factors": list(factors), "fixed": [], "adaptive": None}
    for f in factors:
        pen = dict(alpha=p0, beta=p0, b=p0, adaptive=0)
        pen[which] = p0 * f
        r = acm_stokes_solve(H, g, penalty=pen, eps=eps, max_iter=max_iter, want_q=False)
        out["fixed"].append(r["stats"]["iters"] if r["stats"]["converged"] else None)
    r = acm_stokes_solve(H, g, penalty=dict(tau=(5.0, 10.0, 5.0)), eps=eps, max_iter=max_iter,
                         want_q=False)
    out["adaptive"] = r["stats"]["iters"]
    return out


def comparison_medium_sweep(H: torch.Tensor, u: torch.Tensor, g_chi=(1.0, 0.0, 0.0),
                            Pe: float = 10.0, A0s=(0.55, 1.1, 2.2, 4.4), B0_scales=(0.0, 1.0),
                            eta: float = 0.01, eps: float = 1e-6, max_iter: int = 5000) -> dict:
    """LS iterations of the steady cell problem for each comparison medium A0
    and B0 = scale * mean_Y(B) (Section 4.2); None where it does not converge."""
    pore = (H == 0)
    d = u.shape[0]
    B0m = [Pe * float((u[c] * pore).sum()) / H.numel() for c in range(d)]
    rows = []
    for s in B0_scales:
        B0 = [s * b for b in B0m]
        its = []
        for A0 in A0s:
            try:
                r = acm_transport_step(H, u, list(g_chi)[:d], Pe, A0=A0, B0=B0, eta=eta, eps=eps,
                                       max_iter=max_iter)
                its.append(r["stats"]["iters"] if r["stats"]["converged"] else None)
            except abi.AcmError:
                its.append(None)  # a residual became non-finite
        rows.append(dict(B0_scale=s, iters=its))
    return {"A0": list(A0s), "rows": rows}
