"""Closure-network kernels (BF16 MFMA forward/backward, Adam) against the FP64
reference evaluated on the same BF16-rounded weights and inputs."""
import sys

import numpy as np
import pytest
import torch

from oracle import mlp as R

pytestmark = pytest.mark.gpu
TOL = 1e-2  # relative L2 per tensor: BF16 activations between layers


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def setup(B=192, seed=0):
    from paper_1507_06565_amd import mlp
    rng = np.random.default_rng(seed)
    p = R.init_params(seed)
    p += rng.normal(0, 0.02, p.shape)
    p32 = p.astype(np.float32).astype(np.float64)
    net = mlp.ClosureNet(p32)
    # the reference sees exactly the GPU's operands: BF16 matrices, FP32 biases
    pr = p32.copy()
    for n, (o, s) in R.OFFSETS.items():
        if n.startswith("W"):
            k = int(np.prod(s))
            pr[o:o + k] = R.bf16_round(pr[o:o + k])
    X = np.zeros((B, 64))
    X[:, :33] = rng.uniform(0.3, 1.0, (B, 33))
    Xr = R.bf16_round(X)
    xb = torch.tensor(Xr, dtype=torch.float32).to(torch.bfloat16).cuda()
    return net, pr, Xr, xb, rng


@pytest.mark.parametrize("B", [192, 8192])
def test_forward_and_backward_parity(B):
    """B = 8192: 128 workgroups of partial gradients summed by the fixed-order
    reduction kernel, the batch size of a training step."""
    say("test_forward_and_backward_parity", B)
    net, pr, Xr, xb, rng = setup(B=B, seed=B)
    y = net.forward(xb, train=True).cpu().numpy().astype(np.float64)
    Yr, cache = R.forward(pr, Xr)
    e = rel(y, Yr)
    say("forward rel L2", e)
    assert e <= TOL
    dY = rng.normal(0, 1, Yr.shape)
    g, dx = net.backward(xb, torch.tensor(dY, dtype=torch.float32).cuda(), want_dx=True)
    g = g.cpu().numpy().astype(np.float64)
    gr, dXr = R.backward(pr, cache, dY)
    for n, (o, s) in R.OFFSETS.items():
        k = int(np.prod(s))
        e = rel(g[o:o + k], gr[o:o + k])
        say("grad", n, e)
        assert e <= TOL, n
    e = rel(dx.cpu().numpy(), dXr)
    say("dx", e)
    assert e <= TOL


def test_gradients_are_deterministic():
    net, pr, Xr, xb, rng = setup(B=256, seed=3)
    dY = torch.tensor(rng.normal(0, 1, (256, 16)), dtype=torch.float32).cuda()
    net.forward(xb, train=True)
    g1 = net.backward(xb, dY)[0].clone()
    net.forward(xb, train=True)
    g2 = net.backward(xb, dY)[0].clone()
    assert torch.equal(g1, g2)


def test_loss_and_adam():
    net, pr, Xr, xb, rng = setup(B=128, seed=5)
    y = net.forward(xb, train=True)
    T = rng.normal(0, 1, (128, 2))
    M = (rng.uniform(size=(128, 2)) > 0.25).astype(np.float64)
    L, dy = net.loss(y, torch.tensor(T, dtype=torch.float32).cuda(), torch.tensor(M, dtype=torch.float32).cuda(),
                     M.sum())
    Lr, dYr = R.masked_mse(y.cpu().numpy().astype(np.float64), T, M)
    assert abs(L / Lr - 1) < 1e-5
    assert rel(dy.cpu().numpy(), dYr) < 1e-6
    g = rng.normal(0, 1e-2, R.NPARAM).astype(np.float32)
    net.grad.copy_(torch.tensor(g))
    p0 = net.params.cpu().numpy().astype(np.float64)
    net.adam(lr=1e-3)
    net.grad.copy_(torch.tensor(g * 0.5))
    net.adam(lr=1e-3)
    p, m, v = p0, np.zeros(R.NPARAM), np.zeros(R.NPARAM)
    p, m, v = R.adam(p, m, v, g.astype(np.float64), 1)
    p, m, v = R.adam(p, m, v, 0.5 * g.astype(np.float64), 2)
    assert np.max(np.abs(net.params.cpu().numpy() - p)) < 1e-6


def test_windows_and_closure():
    from paper_1507_06565_amd import mlp
    net, pr, Xr, xb, rng = setup(B=64, seed=7)
    eps = rng.uniform(0.3, 1.0, (2, 70))
    x, n = net.windows(eps)
    assert n == 140
    xw = x.float().cpu().numpy()[:n]
    want = np.concatenate([R.windows(e) for e in eps])
    assert np.array_equal(xw, R.bf16_round(want))
    nue, drag = net.closure(eps, 0.1)
    y = net.forward(x).cpu().numpy().astype(np.float64)[:n]
    ne, dr = R.closure(y, eps.ravel(), 0.1)
    assert np.allclose(nue.ravel(), ne, rtol=1e-12) and np.allclose(drag.ravel(), dr, rtol=1e-12, atol=1e-300)


def test_training_reduces_loss():
    """Fit a smooth map of the porosity window on the GPU with the project's
    own forward/backward/Adam kernels."""
    say("test_training_reduces_loss")
    from paper_1507_06565_amd import mlp
    rng = np.random.default_rng(11)
    net = mlp.ClosureNet(R.init_params(2))
    B = 1024
    X = np.zeros((B, 64))
    X[:, :33] = rng.uniform(0.35, 1.0, (B, 33))
    T = np.stack([np.log(1.0 / X[:, 16]), np.log(X[:, :33].mean(1) ** -2)], 1)
    M = np.ones((B, 2))
    xb = torch.tensor(X, dtype=torch.float32).to(torch.bfloat16).cuda()
    t = torch.tensor(T, dtype=torch.float32).cuda()
    mk = torch.tensor(M, dtype=torch.float32).cuda()
    L0 = None
    for it in range(400):
        L = net.train_step(xb, t, mk, M.sum(), lr=2e-3)
        L0 = L if L0 is None else L0
    say("loss", L0, "->", L)
    assert L < 0.05 * L0


def test_profile_loss_parity():
    """Steady-column loss and its adjoint gradient against the FP64
    reference on the same network outputs (both FP64; tolerance set by the
    FP32 outputs and the FP32 gradient store)."""
    from oracle import closure as CL
    from paper_1507_06565_amd import mlp
    net, pr, Xr, xb, rng = setup(B=64, seed=5)
    nprof, nz, nu, G = 3, 48, 1.0 / 6.0, 1e-6
    eps = rng.uniform(0.4, 1.0, (nprof, nz))
    eps[:, 30:] = 1.0
    eps[:, 0] = eps[:, -1] = 0.0
    ut = np.stack([CL.steady_profile(np.where(e > 0, e, 1.0), np.full(nz, nu), np.where(e < 1, 0.02, 0.0), G)
                   for e in eps]) * rng.uniform(0.8, 1.2, (nprof, 1))
    B = 192
    Y = rng.normal(0, 0.5, (B, 16)).astype(np.float32)
    y = torch.tensor(Y).cuda()
    L, dy = net.profile_loss(y, eps.ravel(), ut.ravel(), nprof, nz, nu, G, 0.5)
    Lr, dYr = CL.profile_loss(Y.astype(np.float64), eps.ravel(), ut.ravel(), nprof, nz, nu, G, 0.5)
    say("profile loss", L, Lr)
    assert np.allclose(L, Lr, rtol=1e-10, atol=0)
    g = dy.cpu().numpy()
    assert np.all(g[nprof * nz:] == 0)
    e1 = rel(g[:nprof * nz].astype(np.float64), dYr)
    say("profile loss gradient rel L2", e1)
    assert e1 <= 1e-6
