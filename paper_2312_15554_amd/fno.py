"""Python side of the FNO warm start: parameter buffers and calls into the C
ABI (acm_fno_*).  Every forward, backward and optimiser step runs in
libacm.so; this module only holds device tensors and marshals arguments."""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import abi
from .api import _dev, _expect, _grid, _stream


class FNO:
    """FNO parameters (FP32 master + BF16 copy + Adam moments) on the GPU."""

    def __init__(self, channels=32, hidden=128, modes=12, layers=4, device="cuda", seed=0):
        self.lib = abi.load()
        self.shape = abi.acm_fno_shape(channels, hidden, modes, layers)
        n = self.lib.acm_fno_param_count(C.byref(self.shape))
        if n < 0:
            raise ValueError("invalid FNO shape")
        self.n = n
        self.params = torch.empty(n, dtype=torch.float32, device=device)
        self.bf16 = torch.empty(n, dtype=torch.int16, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.grad = torch.zeros(n, dtype=torch.float32, device=device)
        self.step = 0
        self._ws = {}
        self.init(seed)

    # ---- layout (mirrors include/acm.h)
    def layout(self):
        Cc, Cp, m, L = (self.shape.channels, self.shape.hidden, self.shape.modes, self.shape.layers)
        nm = (2 * m) * (2 * m) * m
        off, o = {}, 0
        def take(name, size):
            nonlocal o
            off[name] = (o, size)
            o += size
        take("Pw", Cc)
        take("Pb", Cc)
        for l in range(L):
            take(f"R{l}", 2 * nm * Cc * Cc)
            take(f"W{l}", Cc * Cc)
            take(f"b{l}", Cc)
        take("Q1", Cp * Cc)
        take("c1", Cp)
        take("Q2", 4 * Cp)
        take("c2", 4)
        assert o == self.n
        return off

    def init(self, seed=0):
        """Seeded initialisation (scaled uniform / normal), then the BF16 copy."""
        g = torch.Generator(device="cpu").manual_seed(seed)
        Cc, Cp = self.shape.channels, self.shape.hidden
        p = torch.empty(self.n, dtype=torch.float32)
        for name, (o, size) in self.layout().items():
            if name.startswith("R"):
                p[o:o + size] = torch.rand(size, generator=g) / (Cc * Cc)
            elif name.startswith("W"):
                p[o:o + size] = torch.randn(size, generator=g) / math.sqrt(Cc)
            elif name == "Q1":
                p[o:o + size] = torch.randn(size, generator=g) / math.sqrt(Cc)
            elif name == "Q2":
                p[o:o + size] = torch.randn(size, generator=g) / math.sqrt(Cp)
            elif name == "Pw":
                p[o:o + size] = torch.randn(size, generator=g)
            else:
                p[o:o + size] = 0.0
        self.params.copy_(p)
        self.sync_bf16()

    def sync_bf16(self):
        abi.check(self.lib.acm_fno_to_bf16(self.n, _dev(self.params, "params"),
                                           _dev(self.bf16, "bf16"), _stream(None)))

    def bf16_as_float(self) -> torch.Tensor:
        """The BF16 weights the kernels use, widened to FP32 (for checks)."""
        return ((self.bf16.to(torch.int32) & 0xFFFF) << 16).view(torch.float32)

    def workspace(self, n, batch, train):
        key = (n, batch, int(train))
        if key not in self._ws:
            gr = _grid((n, n, n))
            nb = self.lib.acm_fno_workspace_bytes(C.byref(self.shape), C.byref(gr), batch, int(train))
            if nb < 0:
                raise ValueError(abi.load().acm_last_error().decode())
            self._ws = {k: v for k, v in self._ws.items() if k[2] == 0} if train else self._ws
            self._ws[key] = torch.empty(nb, dtype=torch.uint8, device=self.params.device)
        return self._ws[key]

    def forward(self, H: torch.Tensor, train=False, out=None, stream=None):
        """H: uint8 (B, n, n, n) device tensor -> (B, 4, n, n, n) float32."""
        B, n = H.shape[0], H.shape[-1]
        _expect(H, (B, n, n, n), torch.uint8, "H")
        if out is None:
            out = torch.empty((B, 4, n, n, n), dtype=torch.float32, device=H.device)
        _expect(out, (B, 4, n, n, n), torch.float32, "out")
        ws = self.workspace(n, B, train)
        gr = _grid((n, n, n))
        abi.check(self.lib.acm_fno_forward(C.byref(self.shape), C.byref(gr), B, _dev(self.bf16, "bf16"),
                                           _dev(H, "H"), _dev(out, "out"), _dev(ws, "ws"), ws.numel(),
                                           int(train), _stream(stream)))
        return out

    def backward(self, H: torch.Tensor, dout: torch.Tensor, stream=None):
        """Gradient of sum(dout * out) of the last training forward into self.grad."""
        B, n = H.shape[0], H.shape[-1]
        _expect(dout, (B, 4, n, n, n), torch.float32, "dout")
        ws = self.workspace(n, B, True)
        gr = _grid((n, n, n))
        abi.check(self.lib.acm_fno_backward(C.byref(self.shape), C.byref(gr), B, _dev(self.bf16, "bf16"),
                                            _dev(H, "H"), _dev(dout, "dout"), _dev(self.grad, "grad"),
                                            _dev(ws, "ws"), ws.numel(), _stream(stream)))
        return self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        abi.check(self.lib.acm_fno_adam(self.n, _dev(self.params, "p"), _dev(self.bf16, "pb"),
                                        _dev(self.grad, "g"), _dev(self.m, "m"), _dev(self.v, "v"),
                                        self.step, lr, beta1, beta2, eps, _stream(stream)))

    def mse(self, out: torch.Tensor, target: torch.Tensor, dout: torch.Tensor, stream=None) -> float:
        loss = C.c_double()
        abi.check(self.lib.acm_fno_mse(out.numel(), _dev(out, "out"), _dev(target, "target"),
                                       _dev(dout, "dout"), C.byref(loss), _stream(stream)))
        return loss.value
