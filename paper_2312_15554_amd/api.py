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
                     stream=None) -> dict:
    """Stokes cell problem by ADMM (acm_stokes_solve).  H: uint8 device tensor
    in numpy order.  Returns dict(u, q, status, stats, history)."""
    lib = abi.load()
    shape = tuple(H.shape)
    d = len(shape)
    if H.dtype != torch.uint8:
        raise ValueError("H must be uint8")
    dev = H.device
    if u is None:
        u = torch.empty((d,) + shape, dtype=dtype, device=dev)
    if q is None and want_q:
        q = torch.empty(shape, dtype=dtype, device=dev)
    pen = default_penalty(**(penalty or {}))
    opts = default_opts(eps=eps, max_iter=max_iter, precision=_prec(dtype), check_every=check_every,
                        use_graph=int(use_graph), profile=int(profile), history_cap=history_cap,
                        warm_start=int(warm_start))
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


def acm_fft_r2c(x: torch.Tensor, cell_shape, stream=None) -> torch.Tensor:
    """Forward real FFT of x with shape (nfields, *cell_shape) -> half spectra
    (nfields, *cell_shape[:-1], nx//2+1) complex."""
    lib = abi.load()
    nf = x.shape[0]
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
    rdt = torch.float32 if X.dtype == torch.complex64 else torch.float64
    out = torch.empty((nf,) + tuple(cell_shape), dtype=rdt, device=X.device)
    gr = _grid(cell_shape)
    abi.check(lib.acm_fft_c2r(C.byref(gr), _prec(rdt), nf, _dev(X, "X"), _dev(out, "out"),
                              _stream(stream)))
    return out
