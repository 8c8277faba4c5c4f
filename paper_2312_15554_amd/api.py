"""Python entry points with the C ABI's names.  Arguments are torch tensors on
the GPU (device memory and streams only); every step runs in libacm.so."""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import abi


def _grid(shape) -> abi.acm_grid:
    """acm_grid from a numpy-order cell shape ([z][y][x] or [y][x])."""
    g = abi.acm_grid()
    if len(shape) == 3:
        g.dim = 3
        g.n[0], g.n[1], g.n[2] = shape[2], shape[1], shape[0]
    elif len(shape) == 2:
        g.dim = 2
        g.n[0], g.n[1], g.n[2] = shape[1], shape[0], 1
    else:
        raise ValueError("cell shape must be 2D or 3D")
    return g


def _prec(dtype) -> int:
    if dtype == torch.float64:
        return abi.ACM_FP64
    if dtype == torch.float32:
        return abi.ACM_FP32
    raise ValueError("dtype must be float32 or float64")


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _expect(t: torch.Tensor, shape, dtype, what: str):
    """Buffers the library writes or reads must match exactly: a wrong dtype or
    shape would make the kernels run past the end of the allocation."""
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous device tensor")
    if t.device != torch.device("cuda", torch.cuda.current_device()):
        raise ValueError(f"{what} must live on the current device")


def _check_H(H: torch.Tensor):
    if H.dtype != torch.uint8:
        raise ValueError("H must be uint8")
    _expect(H, H.shape, torch.uint8, "H")


def _dvec(vals, n=3):
    arr = (C.c_double * n)()
    for i, v in enumerate(vals):
        arr[i] = float(v)
    return arr


def default_penalty(**kw) -> abi.acm_penalty:
    p = abi.acm_penalty()
    abi.load().acm_default_penalty(C.byref(p))
    for k, v in kw.items():
        if k in ("phi", "tau", "psi_min"):
            arr = getattr(p, k)
            for i in range(3):
                arr[i] = float(v[i])
        else:
            setattr(p, k, v)
    return p


def _deriv(kind) -> int:
    """acm_opts.derivative of "central" (the paper's symbols) or "spectral"."""
    table = {"central": 0, "spectral": 1}
    if kind not in table:
        raise ValueError(f"derivative must be 'central' or 'spectral', not {kind!r}")
    return table[kind]


def default_opts(**kw) -> abi.acm_opts:
    o = abi.acm_opts()
    abi.load().acm_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def stats_dict(st: abi.acm_stats) -> dict:
    return dict(iters=st.iters, r_p=list(st.r_p), r_d=list(st.r_d), tol_p=list(st.tol_p),
                tol_d=list(st.tol_d), psi=list(st.psi), seconds=st.seconds,
                converged=bool(st.converged), status=st.status,
                kernel_ms={k: st.kernel_ms[i] for i, k in enumerate(abi.KERNEL_KINDS)},
                kernel_calls={k: st.kernel_calls[i] for i, k in enumerate(abi.KERNEL_KINDS)})


def acm_stokes_solve(H: torch.Tensor, g, nu: float = 1.0, *, dtype=torch.float32,
                     penalty: dict | None = None, eps: float = 1e-6, max_iter: int = 1_000_000,
                     check_every: int = 0, use_graph: bool = True, profile: bool = False,
                     history_cap: int = 0, u: torch.Tensor | None = None,
                     q: torch.Tensor | None = None, want_q: bool = True, warm_start: bool = False,
                     pass_mode: int = 0, green_variant: int = 0, derivative: str = "central",
                     step1_form: int = 0, stream=None) -> dict:
    """Stokes cell problem by ADMM (acm_stokes_solve).  H: uint8 device tensor
    in numpy order.  Returns dict(u, q, status, stats, history)."""
    lib = abi.load()
    _check_H(H)
    shape = tuple(H.shape)
    d = len(shape)
    dev = H.device
    if u is None:
        u = torch.empty((d,) + shape, dtype=dtype, device=dev)
    if q is None and want_q:
        q = torch.empty(shape, dtype=dtype, device=dev)
    _expect(u, (d,) + shape, dtype, "u")
    if q is not None:
        _expect(q, shape, dtype, "q")
    pen = default_penalty(**(penalty or {}))
    opts = default_opts(eps=eps, max_iter=max_iter, precision=_prec(dtype), check_every=check_every,
                        use_graph=int(use_graph), profile=int(profile), history_cap=history_cap,
                        warm_start=int(warm_start), pass_mode=int(pass_mode),
                        green_variant=int(green_variant), derivative=_deriv(derivative),
                        step1_form=int(step1_form))
    st = abi.acm_stats()
    hist = (C.c_double * (max(history_cap, 1) * abi.HIST_DOUBLES))() if history_cap > 0 else None
    gr = _grid(shape)
    status = lib.acm_stokes_solve(C.byref(gr), _dev(H, "H"), _dvec(list(g) + [0.0] * (3 - len(g))),
                                  float(nu), C.byref(pen), C.byref(opts), _dev(u, "u"),
                                  _dev(q, "q") if q is not None else None, C.byref(st),
                                  hist, _stream(stream))
    abi.check(status)
    history = None
    if hist is not None:
        n = min(st.iters, history_cap)
        import numpy as np
        history = np.array(hist[: n * abi.HIST_DOUBLES]).reshape(n, abi.HIST_DOUBLES)
    return dict(u=u, q=q, status=status, stats=stats_dict(st), history=history)


def acm_stokes_solve_batched(Hs, gs, nu: float = 1.0, *, dtype=torch.float32,
                             penalty: dict | None = None, eps: float = 1e-6,
                             max_iter: int = 1_000_000, check_every: int = 0,
                             use_graph: bool = True, us=None, qs=None, warm_start: bool = False,
                             pass_mode: int = 0, green_variant: int = 0,
                             derivative: str = "central", step1_form: int = 0,
                             stream=None) -> dict:
    """Many cells in one call (acm_stokes_solve_batched).  Hs: list of uint8
    device tensors (any supported sizes), gs: list of body forces.  Returns
    dict(us, qs, status, stats=[per-cell dicts])."""
    lib = abi.load()
    n = len(Hs)
    if len(gs) != n:
        raise ValueError("one body force per cell")
    grids = (abi.acm_grid * n)()
    gp = (C.c_double * (3 * n))()
    if us is None:
        us = [torch.empty((len(H.shape),) + tuple(H.shape), dtype=dtype, device=H.device) for H in Hs]
    for i, H in enumerate(Hs):
        _check_H(H)
        shape = tuple(H.shape)
        _expect(us[i], (len(shape),) + shape, dtype, f"u[{i}]")
        if qs is not None and qs[i] is not None:
            _expect(qs[i], shape, dtype, f"q[{i}]")
        g1 = _grid(shape)
        grids[i].dim = g1.dim
        for k in range(3):
            grids[i].n[k] = g1.n[k]
            gp[3 * i + k] = float(gs[i][k]) if k < len(gs[i]) else 0.0
    hp = (C.c_void_p * n)(*[H.data_ptr() for H in Hs])
    up = (C.c_void_p * n)(*[u.data_ptr() for u in us])
    qp = None
    if qs is not None:
        qp = (C.c_void_p * n)(*[(q.data_ptr() if q is not None else None) for q in qs])
    pen = default_penalty(**(penalty or {}))
    opts = default_opts(eps=eps, max_iter=max_iter, precision=_prec(dtype), check_every=check_every,
                        use_graph=int(use_graph), warm_start=int(warm_start), pass_mode=int(pass_mode),
                        green_variant=int(green_variant), derivative=_deriv(derivative),
                        step1_form=int(step1_form))
    st = (abi.acm_stats * n)()
    status = lib.acm_stokes_solve_batched(n, grids, hp, gp, float(nu), C.byref(pen), C.byref(opts),
                                          up, qp, st, _stream(stream))
    abi.check(status)
    return dict(us=us, qs=qs, status=status, stats=[stats_dict(st[i]) for i in range(n)])


def acm_fft_r2c(x: torch.Tensor, cell_shape, stream=None) -> torch.Tensor:
    """Forward real FFT of x with shape (nfields, *cell_shape) -> half spectra
    (nfields, *cell_shape[:-1], nx//2+1) complex."""
    lib = abi.load()
    nf = x.shape[0]
    _expect(x, (nf,) + tuple(cell_shape), x.dtype, "x")
    cdt = torch.complex64 if x.dtype == torch.float32 else torch.complex128
    out = torch.empty((nf,) + tuple(cell_shape[:-1]) + (cell_shape[-1] // 2 + 1,), dtype=cdt,
                      device=x.device)
    gr = _grid(cell_shape)
    abi.check(lib.acm_fft_r2c(C.byref(gr), _prec(x.dtype), nf, _dev(x, "x"), _dev(out, "out"),
                              _stream(stream)))
    return out


def acm_fft_c2r(X: torch.Tensor, cell_shape, stream=None) -> torch.Tensor:
    lib = abi.load()
    nf = X.shape[0]
    if X.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("X must be complex64 or complex128")
    _expect(X, (nf,) + tuple(cell_shape[:-1]) + (cell_shape[-1] // 2 + 1,), X.dtype, "X")
    rdt = torch.float32 if X.dtype == torch.complex64 else torch.float64
    out = torch.empty((nf,) + tuple(cell_shape), dtype=rdt, device=X.device)
    gr = _grid(cell_shape)
    abi.check(lib.acm_fft_c2r(C.byref(gr), _prec(rdt), nf, _dev(X, "X"), _dev(out, "out"),
                              _stream(stream)))
    return out


def acm_transport_step(H: torch.Tensor, u: torch.Tensor, g_chi, Pe: float, *,
                       diffusivity: float = 1.0, eta: float = 0.01, A0: float = 0.55,
                       B0=(0.0, 0.0, 0.0), dt: float = math.inf, n_steps: int = 1,
                       eps: float = 1e-6, max_iter: int = 1_000_000, chi: torch.Tensor | None = None,
                       check_every: int = 0, use_graph: bool = True, profile: bool = False,
                       derivative: str = "central", form: str = "central", stream=None) -> dict:
    """Penalised advection-diffusion by the LS iteration (acm_transport_step).
    u: flow field (d, *shape) in the working precision.  chi (optional) holds
    the initial value and receives the result.  form: "central" (the literal
    discretisation) or "flux" (face fluxes with harmonic-mean diffusivity;
    acm_opts.transport_form = 1).  Returns dict(chi, status, stats)."""
    if form not in ("central", "flux"):
        raise ValueError(f"form must be 'central' or 'flux', not {form!r}")
    lib = abi.load()
    _check_H(H)
    shape = tuple(H.shape)
    _prec(u.dtype)
    _expect(u, (len(shape),) + shape, u.dtype, "u")
    if chi is None:
        chi = torch.zeros(shape, dtype=u.dtype, device=u.device)
    _expect(chi, shape, u.dtype, "chi")
    opts = default_opts(eps=eps, max_iter=max_iter, precision=_prec(u.dtype),
                        check_every=check_every, use_graph=int(use_graph), profile=int(profile),
                        derivative=_deriv(derivative), transport_form=1 if form == "flux" else 0)
    st = abi.acm_stats()
    gr = _grid(shape)
    d = len(shape)
    status = lib.acm_transport_step(C.byref(gr), _dev(H, "H"), _dev(u, "u"),
                                    _dvec(list(g_chi) + [0.0] * (3 - len(g_chi))), float(Pe),
                                    float(diffusivity), float(eta), float(A0),
                                    _dvec(list(B0)[:d] + [0.0] * (3 - d)), float(dt), int(n_steps),
                                    C.byref(opts), _dev(chi, "chi"), C.byref(st), _stream(stream))
    abi.check(status)
    return dict(chi=chi, status=status, stats=stats_dict(st))


def acm_effective_props(H: torch.Tensor, us=(), chis=(), u_transport: torch.Tensor | None = None,
                        nu: float = 1.0, Pe: float = 0.0, stream=None) -> dict:
    """Effective permeability rows K[i] (flow i) and diffusivity columns D[:, j]
    (chi j) with solute masses (acm_effective_props)."""
    return _props("acm_effective_props", H, us, chis, u_transport, nu, Pe, stream)


def acm_effective_props_noalloc(H: torch.Tensor, us=(), chis=(), u_transport: torch.Tensor | None = None,
                                nu: float = 1.0, Pe: float = 0.0, stream=None) -> dict:
    """The same as acm_effective_props through the allocation-free entry point
    (acm_effective_props_noalloc): partial sums in the library's fixed device
    array, kernels on the caller's stream."""
    return _props("acm_effective_props_noalloc", H, us, chis, u_transport, nu, Pe, stream)


def _props(entry, H, us, chis, u_transport, nu, Pe, stream) -> dict:
    import numpy as np
    lib = abi.load()
    shape = tuple(H.shape)
    d = len(shape)
    ref = us[0] if len(us) else (chis[0] if len(chis) else None)
    if ref is None:
        raise ValueError("nothing to compute")
    prec = _prec(ref.dtype)
    _check_H(H)
    for x in us:
        _expect(x, (d,) + shape, ref.dtype, "u")
    for x in chis:
        _expect(x, shape, ref.dtype, "chi")
    if u_transport is not None:
        _expect(u_transport, (d,) + shape, ref.dtype, "u_transport")
    nf, nc = len(us), len(chis)
    up = (C.c_void_p * max(nf, 1))(*[_dev(x, "u").value for x in us])
    cp = (C.c_void_p * max(nc, 1))(*[_dev(x, "chi").value for x in chis])
    K = (C.c_double * max(nf * d, 1))()
    D = (C.c_double * max(d * nc, 1))()
    mass = (C.c_double * max(nc, 1))()
    gr = _grid(shape)
    abi.check(getattr(lib, entry)(C.byref(gr), prec, _dev(H, "H"), nf, up, nc, cp,
                                  _dev(u_transport, "u_transport") if u_transport is not None else None,
                                  float(nu), float(Pe), K if nf else None, D if nc else None,
                                  mass if nc else None, _stream(stream)))
    return dict(K=np.array(K[: nf * d]).reshape(nf, d) if nf else None,
                D=np.array(D[: d * nc]).reshape(d, nc) if nc else None,
                mass=np.array(mass[:nc]) if nc else None)
