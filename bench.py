"""Benchmark: unit-cell Stokes permeability on one MI355X.

Workload (one "step"): the 3D Stokes cell problem on a 128^3 periodic cell of
randomly placed overlapping spheres (radius 8 voxels, centres from SplitMix64
seed 1, added until the pore fraction first drops to 0.40), solved by the ADMM
of Section 3.1 for the three unit pressure gradients e_x, e_y, e_z to
eps = 1e-6 (FP32 fields and transforms, FP64 reductions), followed by the full
permeability tensor (eq. K).  Inputs are resident in HBM before timing starts.

Prints ONE JSON line.  Throughput = voxel-iterations per second over the timed
steps.  The roofline object covers the kernel with the largest share of time in
a profiled solve (HIP events on the library stream); cpu_baseline times the
FP64 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="cell side (voxels)")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=12, help="oracle iterations in the CPU sample")
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="profiling aid: run exactly this many iterations per solve (eps = 0)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="profiling aid: only run a plain device copy of this many MiB, 10 times")
    ap.add_argument("--no-transport", action="store_true", help="skip the 500-step transport run")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-cell batch comparison")
    ap.add_argument("--transport-steps", type=int, default=500)
    ap.add_argument("--no-fno", action="store_true",
                    help="skip training the FNO warm start and the warm vs plain comparison")
    ap.add_argument("--fno-train", type=int, default=2000, help="64^3 training solves")
    ap.add_argument("--fno-epochs", type=int, default=4)
    ap.add_argument("--fno-test", type=int, default=10, help="256^3 test cells")
    ap.add_argument("--fno-held", type=int, default=64,
                    help="held-out 64^3 cells of the batched + warm-started comparison")
    ap.add_argument("--no-256", action="store_true", help="skip the 256^3 section")
    ap.add_argument("--no-scaling", action="store_true", help="skip the size-scaling section")
    ap.add_argument("--no-sweeps", action="store_true", help="skip the parameter sweeps")
    ap.add_argument("--batch-cells", type=int, default=64)
    return ap.parse_args()


def transport_section(H, u_flow, log):
    """Advection-diffusion on the same cell (Section 3.2): flow u(g = e_x)
    scaled to unit pore-mean speed, Pe = 10, eta = 0.01, A0 = 0.55,
    B0 = mean_Y(B), backward Euler dt = 2e-3 from chi = 0, per-step eps = 1e-6,
    for g_chi = e_x, e_y, e_z; D* tensor and solute-mass drift."""
    import torch
    from paper_2312_15554_amd.api import acm_effective_props, acm_transport_step
    args = parse()
    pore = (H == 0)
    ubar = torch.stack([(u_flow[c] * pore).sum() / pore.sum() for c in range(3)]).double()
    un = (u_flow / ubar.norm().float()).contiguous()
    Pe = 10.0
    B0 = [Pe * float((un[c] * pore).sum()) / H.numel() for c in range(3)]
    chis, out = [], dict(steps=args.transport_steps, dt=2e-3, Pe=Pe, B0=B0)
    iters, secs = [], []
    # Comparison medium: the smallest A0 of a ladder for which the first time
    # step converges (Section 4.2: the best value is the smallest that converges).
    from paper_2312_15554_amd import abi
    A0 = None
    for cand in [0.55 * 2 ** k for k in range(8)]:
        try:
            r = acm_transport_step(H, un, [1.0, 0.0, 0.0], Pe, eta=0.01, A0=cand, B0=B0, dt=2e-3,
                                   n_steps=1, eps=1e-6, max_iter=2000)
        except abi.AcmError as e:
            log(f"transport A0={cand:g}: {e}")
            continue
        if r["stats"]["converged"]:
            A0 = cand
            break
        log(f"transport A0={cand:g}: not converged in 2000 iterations")
    if A0 is None:
        raise RuntimeError("no comparison medium in the ladder converged")
    out["A0"] = A0
    log(f"transport: comparison medium A0 = {A0:g}")
    for j in range(3):
        g = [0.0, 0.0, 0.0]
        g[j] = 1.0
        chi = torch.zeros(H.shape, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = acm_transport_step(H, un, g, Pe, eta=0.01, A0=A0, B0=B0, dt=2e-3,
                               n_steps=args.transport_steps, eps=1e-6, max_iter=2000, chi=chi)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        iters.append(r["stats"]["iters"])
        chis.append(chi)
        log(f"transport g_chi=e{j}: {r['stats']['iters']} LS iterations, {secs[-1]:.2f} s, "
            f"converged {r['stats']['converged']}")
    # per-kernel event times of one profiled time step (g_chi = e_x, 192 LS
    # iterations with no stop test: a multiple of the 16 between host checks,
    # so that no launch skips after the last iteration) against the byte
    # model of the transport passes
    rp = acm_transport_step(H, un, [1.0, 0.0, 0.0], Pe, eta=0.01, A0=A0, B0=B0, dt=2e-3,
                            n_steps=1, eps=0.0, max_iter=192, check_every=16, profile=True)
    st = rp["stats"]
    nn3 = H.shape[0]
    kern = {}
    for k, kind in (("t_green", "t_green"), ("t_local", "t_slab")):
        if st["kernel_calls"][k]:
            ms = st["kernel_ms"][k] / st["kernel_calls"][k]
            kern[k] = dict(avg_us=round(ms * 1e3, 2), calls=st["kernel_calls"][k],
                           GBps=gbps(kernel_bytes(kind, nn3, 3, 0), ms),
                           algorithmic_bytes=kernel_bytes(kind, nn3, 3, 0),
                           traffic=counter_traffic(k, "transport128") if nn3 == 128 else None)
    out["kernels"] = kern
    # Flux form (face fluxes with harmonic-mean diffusivity): its fixed point
    # carries no A0, so the same problem at two comparison media gives the
    # same D*; the central form's D* moves with A0.  Then the flux form on a
    # flow converged to 1e-8, so that the solute-mass drift reflects the
    # transport rather than the flow's penalty error in the solid.
    def d_column(form, A0v, flow, j=0):
        g = [0.0, 0.0, 0.0]
        g[j] = 1.0
        c = torch.zeros(H.shape, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rr = acm_transport_step(H, flow, g, Pe, eta=0.01, A0=A0v, B0=B0, dt=2e-3,
                                n_steps=args.transport_steps, eps=1e-6, max_iter=4000, chi=c, form=form)
        torch.cuda.synchronize()
        pp = acm_effective_props(H, [], [c], u_transport=flow, Pe=Pe)
        drift = abs(float(pp["mass"][0])) / (float(c.abs().double().sum()) / H.numel())
        return [float(v) for v in pp["D"][:, 0]], rr["stats"]["iters"], time.perf_counter() - ta, drift
    A0b = 2.0 * A0
    flux = {}
    for form in ("flux", "central"):
        D1, it1, s1, dr1 = d_column(form, A0, un)
        D2, it2, s2, dr2 = d_column(form, A0b, un)
        flux[form] = dict(A0=[A0, A0b], D_col_x=[D1, D2], ls_iterations=[it1, it2],
                          seconds=[round(s1, 3), round(s2, 3)],
                          D_xx_rel_change=abs(D1[0] - D2[0]) / abs(D1[0]))
        log(f"transport {form} form, A0 {A0:g} vs {A0b:g}: D*_x. {D1} vs {D2}")
    from paper_2312_15554_amd.api import acm_stokes_solve as _ss
    ut = torch.empty_like(u_flow)
    rt = _ss(H, (1.0, 0.0, 0.0), penalty=dict(tau=(5.0, 10.0, 5.0)), eps=1e-8, max_iter=400000, u=ut,
             want_q=False)
    pore_t = (H == 0)
    ubt = torch.stack([(ut[c] * pore_t).sum() / pore_t.sum() for c in range(3)]).double()
    unt = (ut / ubt.norm().float()).contiguous()
    Dt, itt, st_, drt = d_column("flux", A0, unt)
    flux["flux_on_flow_eps1e-8"] = dict(flow_iterations=rt["stats"]["iters"],
                                        flow_solid_rel_norm=float((unt * (~pore_t)).double().norm() /
                                                                  unt.double().norm()),
                                        D_col_x=Dt, ls_iterations=itt, mass_drift_rel=drt)
    log(f"transport flux form on the 1e-8 flow: D*_x. {Dt}, mass drift {drt:.3e}")
    out["forms"] = flux
    p = acm_effective_props(H, [], chis, u_transport=un, Pe=Pe)
    n = H.numel()
    # What drives the solute-mass drift: with B = Pe (1-H) u the mean of chi
    # changes at the rate mean(chi div_c B), and div_c B is not zero where the
    # flow's penalty error leaves u non-zero in the solid next to the pore.
    nn = H.shape[0]
    Bf = Pe * un * pore
    divB = sum((torch.roll(Bf[c], -1, dims=2 - c) - torch.roll(Bf[c], 1, dims=2 - c)) * (nn / 2.0)
               for c in range(3))
    out["flow_solid_rel_norm"] = float((un * (~pore)).double().norm() / un.double().norm())
    out["divB_rms"] = float(divB.double().pow(2).mean().sqrt())
    out.update(D=[[float(v) for v in row] for row in p["D"]],
               mass=[float(m) for m in p["mass"]],
               mass_drift_rel=[abs(float(p["mass"][j])) / (float(chis[j].abs().double().sum()) / n)
                               for j in range(3)],
               ls_iterations=iters, seconds=[round(x, 3) for x in secs],
               voxel_iters_per_s=sum(iters) * n / sum(secs))
    return out


def fno_section(args, log, cells):
    """FNO warm start: train on method-generated 64^3 solves (r = 4 voxels,
    porosity U[0.35, 0.50], seeds 10000..); then
    (1) the metric's comparison on cells of the training distribution: held-out
        64^3 cells (seeds 30000..) solved one at a time from zero (plain) against
        one batched call warm-started from the network (improved), inference
        included, eps = 1e-6;
    (2) every 256^3 test cell (r = 16, seeds 20000..): plain against warm-started
        single-cell solves to eps = 1e-6;
    (3) a held-out 64^3 cell in FP64 to eps = 1e-10, where the method's band
        around the fixed point is narrow enough for plain and warm-started K to
        be compared (the ACM iteration is the judge of the warm start; FP32
        certifies at most eps ~ b ulp(u), about 5e-9 at 256^3)."""
    import torch
    from paper_2312_15554_amd import warmstart as W
    from paper_2312_15554_amd.api import acm_stokes_solve, acm_stokes_solve_batched
    from paper_2312_15554_amd.fno import FNO
    H, Y, info = W.generate_dataset(cells, eps=1e-6, log=log)
    norm = W.Normaliser(Y)
    net = FNO(channels=32, hidden=128, modes=12, layers=4, seed=0)
    ntr = max(1, int(0.9 * len(cells)))
    tr = W.train(net, H[:ntr], norm.encode(Y[:ntr]), epochs=args.fno_epochs, batch=8, lr=2e-3,
                 lr_final=2e-4, log=log)
    err_hold = W.relative_error(net, norm, H[ntr:], Y[ntr:]) if ntr < len(cells) else None
    del H, Y
    torch.cuda.empty_cache()

    # (1) batched + warm-started against plain single-cell solves, 64^3
    held = [torch.from_numpy(c).cuda() for c in W.make_cells(64, args.fno_held, 30000, 4.0, 0.35, 0.50)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [acm_stokes_solve(h, (1.0, 0.0, 0.0), eps=1e-6, max_iter=400000, want_q=False) for h in held]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    preds = [W.predict(net, norm, h) for h in held]
    rb = acm_stokes_solve_batched(held, [(1.0, 0.0, 0.0)] * len(held), eps=1e-6, max_iter=400000,
                                  us=[p[0] for p in preds], qs=[p[1] for p in preds], warm_start=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    vox = sum(h.numel() for h in held)
    it_p = [r["stats"]["iters"] for r in plain]
    it_w = [st["iters"] for st in rb["stats"]]
    kp = [float(r["u"][0].double().mean()) for r in plain]
    kw = [float(u[0].double().mean()) for u in rb["us"]]
    batched_warm = dict(cells=len(held), n=64, eps=1e-6, plain_seconds=round(t1 - t0, 3),
                        batched_warm_seconds=round(t2 - t1, 3), speedup=round((t1 - t0) / (t2 - t1), 3),
                        plain_iters_mean=sum(it_p) / len(it_p), warm_iters_mean=sum(it_w) / len(it_w),
                        plain_voxel_iters_per_s=sum(i * h.numel() for i, h in zip(it_p, held)) / (t1 - t0),
                        all_converged=all(r["stats"]["converged"] for r in plain) and
                        all(st["converged"] for st in rb["stats"]),
                        k_rel_diff_median=sorted(abs(a - b) / abs(a) for a, b in zip(kp, kw))[len(kp) // 2])
    log(f"fno batched+warm vs plain at 64^3: {batched_warm}")
    del held, plain, preds, rb

    # (2) every 256^3 test cell, plain vs warm at eps = 1e-6
    tests = []
    test_cells = W.make_cells(256, args.fno_test, 20000, 16.0, 0.35, 0.50)
    if test_cells:  # the 256^3 plan is tuned before any timed solve
        acm_stokes_solve(torch.from_numpy(test_cells[0]).cuda(), (1.0, 0.0, 0.0), eps=1e-6, max_iter=400,
                         want_q=False)
    for i, c in enumerate(test_cells):
        r = W.solve_plain_and_warm(net, norm, torch.from_numpy(c).cuda(), eps=1e-6)
        log(f"fno test cell {i}: {r}")
        tests.append(r)
    # (3) the ACM iteration as the judge: a held-out 64^3 cell solved in FP64
    # to eps = 1e-10 from zero and from the network's prediction; at that
    # tolerance the method's band around the fixed point is far below 1e-5
    hc = torch.from_numpy(W.make_cells(64, 1, 30000, 4.0, 0.35, 0.50)[0]).cuda()
    u0, p0 = W.predict(net, norm, hc)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    rp = acm_stokes_solve(hc, (1.0, 0.0, 0.0), dtype=torch.float64, eps=1e-10, max_iter=2000000,
                          want_q=False)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    rw = acm_stokes_solve(hc, (1.0, 0.0, 0.0), dtype=torch.float64, eps=1e-10, max_iter=2000000,
                          u=u0.double().contiguous(), q=p0.double().contiguous(), warm_start=True)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    kp, kw = float(rp["u"][0].mean()), float(rw["u"][0].mean())
    tight = dict(n=64, dtype="f64", eps=1e-10, plain_iters=rp["stats"]["iters"],
                 warm_iters=rw["stats"]["iters"], plain_s=round(tb - ta, 3), warm_s=round(tc - tb, 3),
                 k_plain=kp, k_warm=kw, k_rel_diff=abs(kw - kp) / abs(kp),
                 converged=bool(rp["stats"]["converged"] and rw["stats"]["converged"]))
    log(f"fno held-out 64^3 cell, FP64 to eps 1e-10: {tight}")
    applied = len(test_cells) + args.fno_held
    return dict(train_cells=len(cells), data_seconds=round(info["seconds"], 2),
                train_seconds=round(tr["seconds"], 2), train_steps=tr["steps"],
                training_seconds_per_applied_cell=round((info["seconds"] + tr["seconds"]) / applied, 3),
                final_loss=tr["loss"][-1], holdout_rel_err=err_hold,
                batched_warm_vs_plain_64=batched_warm, tests=tests, judge_fp64_eps1e10=tight,
                iters_saved=[t["plain_iters"] - t["warm_iters"] for t in tests],
                time_ratio_warm_over_plain=[t["warm_s"] / t["plain_s"] for t in tests])


def scaling_section(log):
    """Size scaling on the whole chip, the one-GPU counterpart of the paper's
    scaling study (Section 4): the 2D model cell (disc of radius 0.2 L) at
    128^2 ... 1024^2 and 3D overlapping-sphere cells (porosity 0.40, radius
    N/16) at 32^3 ... 256^3, FP32, a fixed number of ADMM iterations each
    (the captured-graph loop, adaptive penalties).  Reported: time per
    iteration and voxel-iterations/s; at fixed work per CU the paper's weak
    scaling corresponds to constant voxel-iterations/s per CU."""
    import torch
    from paper_2312_15554_amd import inputs as I
    from paper_2312_15554_amd.api import acm_stokes_solve
    rows = []
    for dim, ns, iters in ((2, (128, 256, 512, 1024), 4000), (3, (32, 64, 128, 256), 600)):
        for n in ns:
            if dim == 2:
                Hn = I.centred_disc(n, 0.2)
            else:
                Hn = I.overlapping_spheres(n, n / 16.0, 0.40, seed=1)
            H = torch.from_numpy(Hn).cuda()
            g = (1.0, 0.0, 0.0)[:dim]
            kw = dict(penalty=dict(tau=(5.0, 10.0, 5.0)), eps=0.0, want_q=False)
            acm_stokes_solve(H, g, max_iter=400, **kw)  # tunes the plan
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = acm_stokes_solve(H, g, max_iter=iters, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            vox = Hn.size
            rows.append(dict(dim=dim, n=n, voxels=vox, iterations=r["stats"]["iters"],
                             iter_us=round(dt / iters * 1e6, 2),
                             voxel_iters_per_s=vox * iters / dt,
                             voxels_per_cu=vox / 256.0))
            log(f"scaling: {dim}D {n}: {rows[-1]['iter_us']} us per iteration, "
                f"{rows[-1]['voxel_iters_per_s'] / 1e9:.2f} G voxel-iter/s")
            del H, r
    return rows


def stokes256_section(log):
    """The 256^3 cell of the same construction as the timed workload (radius 16
    voxels, porosity 0.40, seed 1), g = e_x, eps = 1e-6: a converged plain
    solve (single cell, automatic pass structure) and a profiled solve whose
    per-kernel event times give the roofline at this size, where the working
    set is well beyond the 256 MB Infinity Cache."""
    import torch
    from paper_2312_15554_amd import inputs as I
    from paper_2312_15554_amd.api import acm_effective_props, acm_stokes_solve
    n = 256
    Hn = I.overlapping_spheres(n, 16.0, 0.40, seed=1)
    nsolid = int(Hn.sum())
    H = torch.from_numpy(Hn).cuda()
    u = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
    pen = dict(tau=(5.0, 10.0, 5.0))
    acm_stokes_solve(H, (1.0, 0.0, 0.0), penalty=pen, eps=1e-6, max_iter=400, u=u, want_q=False)  # tunes the plan
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = acm_stokes_solve(H, (1.0, 0.0, 0.0), penalty=pen, eps=1e-6, max_iter=400000, u=u, want_q=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    its = r["stats"]["iters"]
    K = acm_effective_props(H, [u], nu=1.0)["K"]
    rp = acm_stokes_solve(H, (1.0, 0.0, 0.0), penalty=pen, eps=1e-6, max_iter=400000, u=u,
                          want_q=False, profile=True)
    km, kc = dict(rp["stats"]["kernel_ms"]), dict(rp["stats"]["kernel_calls"])
    km.pop("other", None), kc.pop("other", None)
    per = {k: dict(avg_us=round(km[k] / kc[k] * 1e3, 2), calls=kc[k],
                   GBps=gbps(kernel_bytes(k, n, 3, nsolid), km[k] / kc[k]))
           for k in km if kc[k] > 0}
    share = {k: km[k] for k in km if kc[k] > 0}
    dom = max(share, key=share.get)
    ach = kernel_bytes(dom, n, 3, nsolid) / (km[dom] / kc[dom] * 1e-3) / 1e9
    out = dict(workload="stokes3d-256^3-overlapping-spheres-r16-porosity0.40-seed1-gx-eps1e-06",
               iterations=its, seconds=round(t1 - t0, 4), converged=bool(r["stats"]["converged"]),
               voxel_iters_per_s=its * float(n ** 3) / (t1 - t0), k_xx=float(K[0][0]),
               iter_us_profiled=round(1e3 * sum(km.values()) / max(1, rp["stats"]["iters"]), 2),
               kernels=per,
               roofline={"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": counter_traffic(dom, "stokes256")})
    log(f"256^3: {its} iterations in {t1 - t0:.2f} s, {out['voxel_iters_per_s'] / 1e9:.1f} G voxel-iter/s, "
        f"kernels {per}")
    return out


def batched_section(ncell, log):
    """64 uneven cells: N from {32, 48, 64, 96, 128}, porosity U[0.3, 0.6]
    (seeds 1000..), radius N/16, Stokes g = e_x, FP32, eps = 1e-6: one call per
    cell (plain) against one batched call."""
    import numpy as np
    import torch
    from paper_2312_15554_amd import inputs as I
    from paper_2312_15554_amd.api import acm_stokes_solve, acm_stokes_solve_batched
    sizes = [32, 48, 64, 96, 128]
    Hs = []
    for k in range(ncell):
        rng = I.SplitMix64(1000 + k)
        nn = sizes[min(4, int(rng.uniform() * 5))]
        por = 0.3 + 0.3 * rng.uniform()
        Hs.append(torch.from_numpy(I.overlapping_spheres(nn, nn / 16.0, por, seed=1000 + k)).cuda())
    vox = [H.numel() for H in Hs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_plain = []
    for H in Hs:
        r = acm_stokes_solve(H, (1.0, 0.0, 0.0), eps=1e-6, max_iter=200000, want_q=False)
        it_plain.append(r["stats"]["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rb = acm_stokes_solve_batched(Hs, [(1.0, 0.0, 0.0)] * ncell, eps=1e-6, max_iter=200000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    it_b = [st["iters"] for st in rb["stats"]]
    vi_p = sum(v * i for v, i in zip(vox, it_plain))
    vi_b = sum(v * i for v, i in zip(vox, it_b))
    log(f"batched: {ncell} cells, {sum(vox) / 1e6:.1f} M voxels: plain {t1 - t0:.2f} s, batched {t2 - t1:.2f} s")
    return dict(cells=ncell, voxels=sum(vox), sizes=[H.shape[0] for H in Hs],
                plain_seconds=round(t1 - t0, 3), batched_seconds=round(t2 - t1, 3),
                plain_voxel_iters_per_s=vi_p / (t1 - t0), batched_voxel_iters_per_s=vi_b / (t2 - t1),
                iterations_equal=it_plain == it_b, speedup=(t1 - t0) / (t2 - t1))


def gbps(nbytes: float, ms: float):
    """GB/s of a kernel moving nbytes in ms, or None without a byte model."""
    return round(nbytes / (ms * 1e-3) / 1e9, 1) if math.isfinite(nbytes) else None


def kernel_bytes(kind: str, n: int, d: int, nsolid: int, real_bytes: int = 4) -> float:
    """Algorithmic HBM bytes one launch of `kind` must move (FP32 fields).
    Half spectra hold nspec = n*n*(n/2+1) complex values per field."""
    ntot = n ** d
    nspec = (n ** (d - 1)) * (n // 2 + 1)
    cb = 2 * real_bytes
    if kind == "green":   # d spectral fields in+out, q-hat and div-hat in+out
        return nspec * cb * (2 * d + 4)
    if kind in ("y_inv", "y_fwd"):
        return nspec * cb * 2 * d
    if kind in ("local", "local+rhs"):
        # spectra in; u in+out; a in+out on solid voxels; H; spectra of r out
        return (2 * d * nspec * cb + 2 * d * ntot * real_bytes + 2 * d * nsolid * real_bytes
                + ntot)
    if kind == "rhs_full":  # the rhs pass when Step 4 changed b: u, a (solid), H in, spectra out
        return d * ntot * real_bytes + d * nsolid * real_bytes + ntot + d * nspec * cb
    if kind == "t_slab":  # transport slab pass (3D): grad chi-hat in, u and H in, 4 spectra out
        return (d + d + 1) * nspec * cb + d * ntot * real_bytes + ntot
    if kind == "t_green":  # transport green pass (3D slab form, time step): 4 spectra,
        # chi-hat and chi-hat of the last step in; chi-hat and grad chi-hat out
        return (4 + 1 + 1 + 1 + d) * nspec * cb
    # "rhs": Step 4 from the FP64 partial sums (a few KB), the full pass only
    # when b changed, so no byte model
    return float("nan")


_PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
# workload -> (counter summary, kernel kind -> symbol prefix of its FP32 instance)
COUNTER_SUMMARIES = {
    "stokes128": (os.path.join(_PROFILES, "stokes3d_128_hbm_counters.md"),
                  {"local": "k_slab_local<float, 128, 128, false>",
                   "local+rhs": "k_slab_local<float, 128, 128, true>",
                   "rhs": "k_slab_rhs<float, 128, 128>"}),
    "stokes256": (os.path.join(_PROFILES, "stokes3d_256_hbm_counters.md"),
                  {"local": "k_rows_step<float, 128>",
                   "y_inv": "k_cols_reg<float, 256, 1>",
                   "y_fwd": "k_cols_reg<float, 256, -1>"}),
    "transport128": (os.path.join(_PROFILES, "transport3d_128_hbm_counters.md"),
                     {"t_local": "k_transport_slab<float, 128>",
                      "t_green": "k_transport_green<float, 128, 3, 0, true, false>"}),
}


def kernel_source_hash() -> str:
    """SHA-256 over the kernel sources (csrc/*.hip, *.hpp in name order)."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2312_15554_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kind: str, workload: str = "stokes128"):
    """HBM bytes per launch of `kind` from the committed rocprofv3 counter
    summary of `workload`: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each
    scaled by the ratio known bytes / counter reading of a plain device copy.
    None when the summary is missing, lacks the kernel, or was taken on other
    kernel sources."""
    path, symbols = COUNTER_SUMMARIES[workload]
    try:
        text = open(path).read()
    except OSError:
        return None
    meta = {}
    rows = {}
    for line in text.splitlines():
        line = line.strip()
        for key in ("source-sha256", "fetch-scale", "write-scale"):
            if line.startswith(key + ":"):
                meta[key] = line.split(":", 1)[1].strip().strip("`")
        if line.startswith("| `acm::"):
            cells = [c.strip().strip("`") for c in line.strip("|").split("|")]
            try:
                rows[cells[0]] = (float(cells[1]), float(cells[2]))
            except (ValueError, IndexError):
                pass
    if meta.get("source-sha256") != kernel_source_hash():
        return None
    sym = symbols.get(kind)
    hits = [v for k, v in rows.items() if sym and k.startswith(f"acm::{sym}")]
    if len(hits) != 1 or "fetch-scale" not in meta or "write-scale" not in meta:
        return None
    fetch_kib, write_kib = hits[0]
    return round(fetch_kib * 1024 * float(meta["fetch-scale"]) +
                 write_kib * 1024 * float(meta["write-scale"]))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent cells or flow directions would shard one per GPU, each GPU "
              "running this single-GPU path on its share).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2312_15554_amd import inputs as I
    from paper_2312_15554_amd.api import acm_effective_props, acm_stokes_solve

    if args.copy_probe_mib:
        # a plain copy of known size: calibrates the HBM byte counters (before
        # anything else, so that no worker pool runs under a profiler)
        import torch
        a = torch.ones(args.copy_probe_mib * (1 << 18), dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 4, "launches": 10}))
        return
    # the FNO training cells are built first, in a forked pool, while the
    # process has not touched the GPU yet
    fno_cells = None
    if not args.no_fno and not args.fixed_iters:
        from paper_2312_15554_amd import warmstart as W
        tc = time.perf_counter()
        fno_cells = W.make_cells(64, args.fno_train, 10000, 4.0, 0.35, 0.50,
                                 workers=max(1, min(os.cpu_count() or 1, 16)))
        print(f"[bench] {len(fno_cells)} FNO training cells built in {time.perf_counter() - tc:.1f} s",
              file=sys.stderr, flush=True)
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    n, d = args.n, 3
    H_np = I.overlapping_spheres(n, 8.0 * n / 128.0, 0.40, seed=1)
    nsolid = int(H_np.sum())
    porosity = 1.0 - nsolid / H_np.size
    H = torch.from_numpy(H_np).cuda()
    dirs = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)]
    us = [torch.empty((d, n, n, n), dtype=torch.float32, device="cuda") for _ in dirs]
    pen = dict(tau=(5.0, 10.0, 5.0))  # random-geometry schedule (Section 4.1 footnote)

    def step():
        its, secs = [], []
        for g, u in zip(dirs, us):
            if args.fixed_iters:
                r = acm_stokes_solve(H, g, penalty=pen, eps=0.0, max_iter=args.fixed_iters, u=u,
                                     want_q=False)
            else:
                r = acm_stokes_solve(H, g, penalty=pen, eps=args.eps, max_iter=200000, u=u,
                                     want_q=False)
            its.append(r["stats"]["iters"])
            secs.append(r["stats"]["seconds"])
            if not args.fixed_iters and not r["stats"]["converged"]:
                raise RuntimeError(f"solve did not converge: {r['stats']}")
        K = acm_effective_props(H, us, nu=1.0)["K"]
        return its, secs, K

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        its_w, secs_w, _ = step()
        log(f"warmup {w}: iterations {its_w}, seconds {[round(x, 3) for x in secs_w]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(step())
        log(f"step {k}: iterations {results[-1][0]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_vi = sum(sum(r[0]) for r in results) * float(n ** d)
    wall = t1 - t0
    its, secs, K = results[-1]

    # ---- roofline: profiled solve (eager launches, HIP events per kernel)
    rp = acm_stokes_solve(H, dirs[0], penalty=pen, eps=0.0 if args.fixed_iters else args.eps,
                          max_iter=args.fixed_iters or 200000, u=us[0], want_q=False, profile=True)
    km, kc = dict(rp["stats"]["kernel_ms"]), dict(rp["stats"]["kernel_calls"])
    if kc["local"] > 0 and kc["rhs"] == 0:  # local and rhs passes in one launch
        km["local+rhs"], kc["local+rhs"] = km.pop("local"), kc.pop("local")
    # Each kernel's events are attached to its own dispatch.  They include a
    # fixed cost of a few microseconds per dispatch, which an empty kernel timed
    # the same way ("other") shows; the graph replays of the solve pay it too
    # (their kernel trace durations equal these event times), so the roofline
    # uses the event times as they are and reports the empty kernel beside.
    ovh_ms = km.pop("other") / kc.pop("other") if kc.get("other") else 0.0
    raw = {k: km[k] / kc[k] for k in km if kc[k] > 0}
    avg_ms = dict(raw)
    share = {k: avg_ms[k] * kc[k] for k in avg_ms}
    dom = max(share, key=share.get)
    avg_s = avg_ms[dom] * 1e-3
    algo = kernel_bytes(dom, n, d, nsolid)
    achieved = algo / avg_s / 1e9
    per_kernel = {k: dict(avg_us=round(avg_ms[k] * 1e3, 2),
                          avg_us_less_empty_kernel=round(max(raw[k] - ovh_ms, 0.0) * 1e3, 2),
                          calls=kc[k],
                          GBps=gbps(kernel_bytes(k, n, d, nsolid), avg_ms[k]))
                  for k in avg_ms}
    iter_us_profiled = 1e3 * sum(km.values()) / max(1, rp["stats"]["iters"])

    log(f"profiled solve: dominant kernel {dom}, {per_kernel}")
    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same cell
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle sample")
        from oracle import acm_oracle as O
        threads = max(1, min(os.cpu_count() or 1, 16))
        O.set_workers(threads)
        tc0 = time.perf_counter()
        O.stokes_admm(H_np, dirs[0], tau=(5.0, 10.0, 5.0), eps=0.0, max_iter=args.cpu_iters)
        tc1 = time.perf_counter()
        cpu = dict(value=args.cpu_iters * float(n ** d) / (tc1 - tc0), unit="voxel-iters/s",
                   cores=threads, kind="oracle",
                   sample=f"{args.cpu_iters} ADMM iterations of the FP64 oracle on the same "
                          f"{n}^3 cell, g = e_x ({tc1 - tc0:.1f} s; scipy.fft workers={threads})")

    # ---- the three directions of the same cell as one batched solve (same H,
    # same tolerance; each direction leaves the batch when it converges)
    dirs_batched = None
    if not args.fixed_iters:
        from paper_2312_15554_amd.api import acm_stokes_solve_batched
        ub = [torch.empty_like(u) for u in us]
        acm_stokes_solve_batched([H] * 3, dirs, penalty=pen, eps=args.eps, max_iter=200000, us=ub)
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        rb = acm_stokes_solve_batched([H] * 3, dirs, penalty=pen, eps=args.eps, max_iter=200000, us=ub)
        torch.cuda.synchronize()
        tb1 = time.perf_counter()
        its_b = [st["iters"] for st in rb["stats"]]
        Kb = acm_effective_props(H, ub, nu=1.0)["K"]
        dirs_batched = dict(seconds=round(tb1 - tb0, 4), iterations=its_b,
                            voxel_iters_per_s=sum(its_b) * float(n ** d) / (tb1 - tb0),
                            speedup_vs_plain=round((wall / args.steps) / (tb1 - tb0), 3),
                            iterations_equal_plain=its_b == list(its),
                            K_max_rel_diff_plain=float(np.max(np.abs(np.array(Kb) - np.array(K))) /
                                                       np.max(np.abs(np.array(K)))))
        log(f"three directions batched: {dirs_batched}")

    s256 = None
    if not args.no_256 and not args.fixed_iters:
        s256 = stokes256_section(log)
    scaling = None
    if not args.no_scaling and not args.fixed_iters:
        scaling = scaling_section(log)
    sweeps = None
    if not args.no_sweeps and not args.fixed_iters:
        from paper_2312_15554_amd import sweeps as SW
        sweeps = SW.run_all(log=log)
    transport = None
    if not args.no_transport and not args.fixed_iters:
        transport = transport_section(H, us[0], log)
    batched = None
    if not args.no_batched and not args.fixed_iters:
        batched = batched_section(args.batch_cells, log)

    fno = fno_section(args, log, fno_cells) if fno_cells is not None else None

    out = {
        "metric": "voxel-iters/s & time-to-1e-6 residual: plain vs batched+FNO warm start",
        "value": total_vi / wall,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"stokes3d-{n}^3-overlapping-spheres-r{8 * n // 128}-porosity0.40-seed1"
                               f"-gx/gy/gz-eps{args.eps:g}-plain-single-cell",
                   "cells": 1, "directions": 3, "eps": args.eps, "porosity": round(porosity, 5)},
        "iterations": its,
        "time_to_tol_s": [round(x, 4) for x in secs],
        "K": [[float(v) for v in row] for row in K],
        "iter_us_profiled": round(iter_us_profiled, 2),
        "kernels": per_kernel,
        "empty_kernel_event_us": round(ovh_ms * 1e3, 2),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(dom)},
        "cpu_baseline": cpu,
        "directions_batched": dirs_batched,
        "stokes_256": s256,
        "size_scaling": scaling,
        "sweeps": sweeps,
        "transport": transport,
        "batched": batched,
        "fno_warm_start": fno,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
