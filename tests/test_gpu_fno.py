"""FNO forward/backward kernels (through the C ABI) against the FP64 oracle
evaluated on the same BF16-rounded weights."""
import numpy as np
import pytest
import torch

from oracle import fno_oracle as F
from paper_2312_15554_amd import inputs as I
from tests.gpu_common import dev, host, require_gpu


def _oracle_params(net):
    w = host(net.bf16_as_float()).astype(np.float64)
    lay = net.layout()
    C, Cp, m, L = net.shape.channels, net.shape.hidden, net.shape.modes, net.shape.layers
    nm = (2 * m) * (2 * m) * m
    get = lambda k: w[lay[k][0]: lay[k][0] + lay[k][1]]
    p = dict(C=C, Cp=Cp, m=m, L=L, Pw=get("Pw"), Pb=get("Pb"), Q1=get("Q1").reshape(Cp, C),
             c1=get("c1"), Q2=get("Q2").reshape(4, Cp), c2=get("c2"), R=[], W=[], b=[])
    for l in range(L):
        r = get(f"R{l}").reshape(nm, C, C, 2)
        p["R"].append(r[..., 0] + 1j * r[..., 1])
        p["W"].append(get(f"W{l}").reshape(C, C))
        p["b"].append(get(f"b{l}"))
    return p


def _flat_grad(net, g):
    lay = net.layout()
    out = np.zeros(net.n)
    for name, (o, size) in lay.items():
        a = F.grad_of(g, name) if name[0] in "RWb" and name[1:].isdigit() else g[name]
        if np.iscomplexobj(a):
            a = np.stack([a.real, a.imag], axis=-1)
        out[o:o + size] = np.asarray(a).reshape(-1)
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("n,C,m,L,B,shift,hidden", [
    (8, 4, 2, 2, 2, 0, 6), (16, 8, 3, 3, 2, 0, 6), (16, 32, 3, 2, 2, 0, 6), (8, 4, 2, 1, 3, 1, 6),
    (8, 8, 2, 1, 2, 0, 40), (8, 16, 2, 1, 2, 0, 200), (8, 8, 2, 2, 11, 0, 6)])
def test_fno_forward_and_gradients_match_oracle(n, C, m, L, B, shift, hidden):
    """Forward pass and every parameter gradient against the FP64 oracle on
    the same BF16 weights.  32 channels take the matrix-core kernels of the
    pointwise mix (the width the warm start trains), fewer the vector ones.
    The weight-gradient sums run on the matrix cores for 16-byte aligned
    operands; `shift` = 1 hands dout over one float off that alignment, which
    sends the sums over dout to the vector kernel.  The projection widths 40
    and 200 give those sums two 32-row blocks per workgroup (40 rows), and
    more blocks than one workgroup owns (200 rows: two groups of four along
    P for dQ1 and along Q for dQ2), each with a ragged last block.  A batch
    of 11 takes the mode mix, its adjoint and the spectral gradient through a
    full chunk of eight cells and a ragged one of three."""
    require_gpu()
    from paper_2312_15554_amd.fno import FNO
    print(f"fno grad check n={n} C={C} m={m} L={L} B={B} shift={shift} hidden={hidden}", flush=True)
    net = FNO(channels=C, hidden=hidden, modes=m, layers=L, seed=5)
    # larger spectral weights than the training initialisation so that the
    # spectral path carries a visible share of the output
    with torch.no_grad():
        for name, (o, size) in net.layout().items():
            if name.startswith("R"):
                net.params[o:o + size] *= 8.0
    net.sync_bf16()
    Hn = np.stack([I.random_mask((n, n, n), 10 + b, 0.4) for b in range(B)])
    H = dev(Hn)
    out = net.forward(H, train=True)
    p = _oracle_params(net)
    ref, cache = F.forward(p, Hn.astype(float), keep=True)
    scale = np.abs(ref).max()
    assert np.abs(host(out) - ref).max() < 2e-5 * scale
    dout_n = I.random_field((B, 4, n, n, n), 77)
    flat = torch.zeros(dout_n.size + shift, dtype=torch.float32, device="cuda")
    flat[shift:] = dev(dout_n.reshape(-1), torch.float32)
    dout = flat[shift:].view(dout_n.shape)
    assert (dout.data_ptr() % 16 == 0) == (shift == 0)
    g = net.backward(H, dout)
    gref = _flat_grad(net, F.backward(p, cache, dout_n))
    gg = host(g).astype(np.float64)
    for name, (o, size) in net.layout().items():
        a, b = gg[o:o + size], gref[o:o + size]
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
        assert err < 2e-4, (name, err)


@pytest.mark.gpu
def test_fno_rejects_misaligned_weights():
    """The mode weights are read as (re, im) BF16 pairs, so a parameter array
    off 4-byte alignment is refused before any work is queued; the aligned
    array runs."""
    require_gpu()
    import ctypes as C
    from paper_2312_15554_amd.api import _grid
    from paper_2312_15554_amd.fno import FNO
    n, B = 8, 1
    net = FNO(channels=4, hidden=6, modes=2, layers=1, seed=2)
    H = dev(I.random_mask((B, n, n, n), 4, 0.4))
    out = torch.empty((B, 4, n, n, n), dtype=torch.float32, device="cuda")
    ws = net.workspace(n, B, False)
    gr = _grid((n, n, n))
    shifted = torch.zeros(net.bf16.numel() + 1, dtype=net.bf16.dtype, device="cuda")
    shifted[1:] = net.bf16
    args = lambda p: (C.byref(net.shape), C.byref(gr), B, p, H.data_ptr(), out.data_ptr(),
                      ws.data_ptr(), ws.numel(), 0, None)
    assert net.lib.acm_fno_forward(*args(shifted.data_ptr() + 2)) == -1
    assert b"aligned" in net.lib.acm_last_error()
    assert net.lib.acm_fno_forward(*args(net.bf16.data_ptr())) == 0
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()


@pytest.mark.gpu
def test_fno_adam_step_decreases_loss():
    require_gpu()
    from paper_2312_15554_amd.fno import FNO
    n, B = 16, 2
    net = FNO(channels=8, hidden=16, modes=3, layers=2, seed=1)
    H = dev(np.stack([I.random_mask((n, n, n), 20 + b, 0.4) for b in range(B)]))
    target = dev(I.random_field((B, 4, n, n, n), 3) * 0.1, torch.float32)
    dout = torch.empty_like(target)
    losses = []
    for _ in range(30):
        out = net.forward(H, train=True)
        losses.append(net.mse(out, target, dout))
        net.backward(H, dout)
        net.adam(lr=3e-3)
    assert losses[-1] < 0.5 * losses[0], losses


@pytest.mark.gpu
def test_trained_fno_warm_start_saves_iterations():
    """What the learned part gains: an FNO trained only on solves of the
    method itself (64 cells of 32^3 overlapping spheres, g = e_x) starts four
    held-out cells closer to their solutions, so the unmodified ADMM reaches
    the same tolerance in fewer iterations on every one of them, and lands on
    the same permeability within that tolerance's band.  ADMM converges
    linearly, so the saving grows only with the logarithm of the starting
    error (about 8 % here at a held-out velocity error near 0.35)."""
    require_gpu()
    from paper_2312_15554_amd import warmstart as W
    from paper_2312_15554_amd.fno import FNO
    n, ntrain, ntest = 32, 64, 4
    print("fno warm start: data", flush=True)
    cells = W.make_cells(n, ntrain + ntest, 5000, 2.0, 0.35, 0.50)
    H, Y, _ = W.generate_dataset(cells, eps=1e-6, log=lambda m: print(m, flush=True))
    norm = W.Normaliser(Y)
    net = FNO(channels=16, hidden=64, modes=10, layers=4, seed=0)
    W.train(net, H[:ntrain], norm.encode(Y[:ntrain]), epochs=120, batch=8, lr=3e-3, lr_final=1e-4,
            log=lambda m: None)
    err = W.relative_error(net, norm, H[ntrain:], Y[ntrain:])
    print(f"held-out relative velocity error {err:.3f}", flush=True)
    res = [W.solve_plain_and_warm(net, norm, H[i], eps=1e-7, max_iter=200000)
           for i in range(ntrain, ntrain + ntest)]
    for r in res:
        print(r, flush=True)
    assert err < 0.45
    assert all(r["converged"] for r in res)
    assert all(r["warm_iters"] < r["plain_iters"] for r in res)
    plain = sum(r["plain_iters"] for r in res)
    warm = sum(r["warm_iters"] for r in res)
    assert warm <= 0.95 * plain, (warm, plain)
    for r in res:
        assert abs(r["k_warm"] - r["k_plain"]) <= 1e-2 * abs(r["k_plain"])
