"""Parameter sweeps of the solvers: the shape of the paper's penalty study
(Section 4.1, Fig. pen_par: iterations against fixed alpha, beta, b and the
adaptive schedule, on the model and a random geometry) and of its
comparison-medium study (Section 4.2, Fig. comp_med: LS iterations against A0
and B0), on synthetic cells.

Each sweep runs the HIP solvers only; nothing here computes the method.
`run_all()` is what the benchmark records; `python -m
paper_2312_15554_amd.sweeps out.json` writes the same dictionary to a file."""
from __future__ import annotations

import json
import sys

import torch

from . import abi
from .api import acm_stokes_solve, acm_transport_step


def penalty_sweep(H: torch.Tensor, g=(1.0, 0.0, 0.0), factors=(0.25, 0.5, 1.0, 2.0, 4.0),
                  which: str = "b", eps: float = 1e-5, max_iter: int = 20000,
                  tau=(5.0, 10.0, 5.0), dtype=torch.float32) -> dict:
    """ADMM iterations to eps with fixed penalties, one of alpha, beta, b
    scaled by each factor from its default nu/h (the others at nu/h), and
    with the adaptive schedule (Section 4.1, eq. varying algorithm).  Also the
    permeability K_11 of every converged solve (the fixed point does not
    depend on the penalties)."""
    d = len(H.shape)
    g = tuple(g)[:d]
    n = max(H.shape)
    p0 = float(n)  # nu / h with nu = 1, h = 1/n
    out = {"which": which, "factors": list(factors), "fixed": [], "k_fixed": [], "adaptive": None}
    for f in factors:
        pen = dict(alpha=p0, beta=p0, b=p0, adaptive=0)
        pen[which] = p0 * f
        r = acm_stokes_solve(H, g, penalty=pen, eps=eps, max_iter=max_iter, want_q=False, dtype=dtype)
        ok = r["stats"]["converged"]
        out["fixed"].append(r["stats"]["iters"] if ok else None)
        out["k_fixed"].append(float(r["u"][0].double().mean()) if ok else None)
    r = acm_stokes_solve(H, g, penalty=dict(tau=tuple(tau)), eps=eps, max_iter=max_iter,
                         want_q=False, history_cap=max_iter, dtype=dtype)
    out["adaptive"] = r["stats"]["iters"]
    out["k_adaptive"] = float(r["u"][0].double().mean())
    hist = r["history"]
    if hist is not None and len(hist):
        # the penalties every iteration used (Fig. pen_par d, e), sampled
        step = max(1, len(hist) // 50)
        out["adaptive_psi_trace"] = [[int(i)] + [float(v) for v in hist[i, 12:15]]
                                     for i in range(0, len(hist), step)]
    return out


def comparison_medium_sweep(H: torch.Tensor, u: torch.Tensor, g_chi=(1.0, 0.0, 0.0),
                            Pe: float = 10.0, A0s=(0.55, 1.1, 2.2, 4.4), B0_scales=(0.0, 1.0),
                            eta: float = 0.01, eps: float = 1e-6, max_iter: int = 5000,
                            form: str = "central") -> dict:
    """LS iterations of the steady cell problem for each comparison medium A0
    and B0 = scale * mean_Y(B) (Section 4.2); None where it does not converge
    (the iteration contracts only for a large enough A0)."""
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
                                       max_iter=max_iter, form=form)
                its.append(r["stats"]["iters"] if r["stats"]["converged"] else None)
            except abi.AcmError:
                its.append(None)  # diverged
        rows.append(dict(B0_scale=s, iters=its))
    return {"A0": list(A0s), "form": form, "rows": rows}


def geometries(model_n: int = 128, random_n: int = 256):
    """The model geometry (a disc of radius 0.2 L, Section 4) and a random 2D
    geometry standing in for the paper's material image (overlapping discs
    of radius random_n/32 voxels at porosity 0.55)."""
    from .inputs import centred_disc, overlapping_spheres
    return {"model": centred_disc(model_n, 0.2),
            "random": overlapping_spheres((random_n, random_n), random_n / 32.0, 0.55, seed=7)}


def run_all(model_n: int = 128, random_n: int = 256, eps: float = 1e-5, log=print) -> dict:
    """Penalty sweeps (alpha, beta, b; tau of the model geometry {20, 10, 30}
    and of the random geometry {5, 10, 5}, Section 4.1) and comparison-medium
    sweeps (A0 with B0 = 0 and B0 = mean(B), eta = 0.01, Section 4.2, on the
    flow of each geometry scaled to unit pore-mean speed, Pe = 10)."""
    out = {}
    taus = {"model": (20.0, 10.0, 30.0), "random": (5.0, 10.0, 5.0)}
    for name, Hn in geometries(model_n, random_n).items():
        H = torch.from_numpy(Hn).cuda()
        res = {"n": int(Hn.shape[0]), "porosity": float(1.0 - Hn.mean()), "eps": eps}
        for which in ("alpha", "beta", "b"):
            res[which] = penalty_sweep(H, (1.0, 0.0), which=which, eps=eps, max_iter=200000,
                                       tau=taus[name])
            log(f"[sweeps] {name} {which}: fixed {res[which]['fixed']}, adaptive {res[which]['adaptive']}")
        r = acm_stokes_solve(H, (1.0, 0.0), eps=1e-7, max_iter=400000, want_q=False)
        u = r["u"]
        pore = (H == 0)
        ubar = torch.stack([(u[c] * pore).sum() / pore.sum() for c in range(2)]).double()
        un = (u / ubar.norm().float()).contiguous()
        res["comparison_medium"] = comparison_medium_sweep(H, un, (1.0, 0.0), 10.0,
                                                           A0s=(0.3, 0.55, 1.1, 2.2, 4.4),
                                                           eps=eps, max_iter=20000)
        res["comparison_medium_flux"] = comparison_medium_sweep(H, un, (1.0, 0.0), 10.0,
                                                                A0s=(0.3, 0.55, 1.1, 2.2, 4.4),
                                                                eps=eps, max_iter=20000, form="flux")
        log(f"[sweeps] {name} comparison medium: {res['comparison_medium']['rows']} "
            f"(flux form {res['comparison_medium_flux']['rows']})")
        out[name] = res
    return out


if __name__ == "__main__":
    res = run_all()
    with open(sys.argv[1] if len(sys.argv) > 1 else "sweeps.json", "w") as f:
        json.dump(res, f, indent=1)
