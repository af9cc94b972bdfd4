"""Plain FP64 reference of the learned closure network (test infrastructure).

The closure maps a window of 33 planar porosities (replicate padding at the
column ends) to two local coefficients of the gray model of Sec. 4 (eps_c is
the porosity of the cell itself; both reduce to the free-fluid values at 1):
    nu_eff / nu = exp((1 - eps_c) o1),    eps nu / K = (1 - eps_c) softplus(o2).
Network: 33 inputs (zero-padded to 64) -> 128 -> 128 -> 128 -> 16 outputs
(2 used), exact-erf GELU between layers, linear output.

Parameter vector layout (FP32 on the device, FP64 here), row-major (K x N):
    W1[64][128] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] W4[128][16] b4[16]
"""
from __future__ import annotations

import math

import numpy as np

IN, IN_PAD, HID, OUT_PAD, OUT = 33, 64, 128, 16, 2
SHAPES = [("W1", (IN_PAD, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (HID, OUT_PAD)), ("b4", (OUT_PAD,))]
OFFSETS = {}
_o = 0
for _n, _s in SHAPES:
    OFFSETS[_n] = (_o, _s)
    _o += int(np.prod(_s))
NPARAM = _o


def unpack(p):
    return {n: p[o:o + int(np.prod(s))].reshape(s) for n, (o, s) in OFFSETS.items()}


def init_params(seed=0):
    """He-style initialisation; rows of W1 beyond the 33 inputs and columns of
    W4 beyond the 2 outputs start at zero."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    P = unpack(p)
    P["W1"][:IN] = rng.normal(0, math.sqrt(2.0 / IN), (IN, HID))
    P["W2"][:] = rng.normal(0, math.sqrt(2.0 / HID), (HID, HID))
    P["W3"][:] = rng.normal(0, math.sqrt(2.0 / HID), (HID, HID))
    P["W4"][:, :OUT] = rng.normal(0, math.sqrt(1.0 / HID), (HID, OUT))
    return p


def gelu(z):
    erf = np.vectorize(math.erf)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    erf = np.vectorize(math.erf)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p, X):
    """X[B, 64] -> Y[B, 16] and the cache of pre-activations."""
    P = unpack(p)
    Z1 = X @ P["W1"] + P["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ P["W2"] + P["b2"]
    H2 = gelu(Z2)
    Z3 = H2 @ P["W3"] + P["b3"]
    H3 = gelu(Z3)
    Y = H3 @ P["W4"] + P["b4"]
    return Y, (X, Z1, H1, Z2, H2, Z3, H3)


def backward(p, cache, dY):
    """Gradient of sum(dY * Y) with respect to the parameters and to X."""
    P = unpack(p)
    X, Z1, H1, Z2, H2, Z3, H3 = cache
    g = np.zeros_like(p)
    G = unpack(g)
    G["W4"][:] = H3.T @ dY
    G["b4"][:] = dY.sum(0)
    dZ3 = (dY @ P["W4"].T) * gelu_prime(Z3)
    G["W3"][:] = H2.T @ dZ3
    G["b3"][:] = dZ3.sum(0)
    dZ2 = (dZ3 @ P["W3"].T) * gelu_prime(Z2)
    G["W2"][:] = H1.T @ dZ2
    G["b2"][:] = dZ2.sum(0)
    dZ1 = (dZ2 @ P["W2"].T) * gelu_prime(Z1)
    G["W1"][:] = X.T @ dZ1
    G["b1"][:] = dZ1.sum(0)
    dX = dZ1 @ P["W1"].T
    return g, dX


def masked_mse(Y, T, M):
    """Loss = sum(M (Y[:, :2] - T)^2) / sum(M) and its gradient dL/dY."""
    n = max(float(M.sum()), 1.0)
    r = (Y[:, :OUT] - T) * M
    dY = np.zeros_like(Y)
    dY[:, :OUT] = 2.0 * r / n
    return float((r * r).sum() / n), dY


def adam(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def windows(eps_profile, half=16):
    """33-cell windows of a porosity profile, replicate padding at the ends;
    returns X[nz, 64] with columns 33.. zero."""
    e = np.asarray(eps_profile, dtype=np.float64)
    nz = len(e)
    X = np.zeros((nz, IN_PAD))
    for z in range(nz):
        for j in range(-half, half + 1):
            X[z, j + half] = e[min(max(z + j, 0), nz - 1)]
    return X


def closure(Y, eps_c, nu):
    """(nu_eff, drag) from the two network outputs and the cells' porosity."""
    o1, o2 = Y[:, 0], Y[:, 1]
    s = 1.0 - np.asarray(eps_c, dtype=np.float64)
    return nu * np.exp(s * o1), s * np.logaddexp(0.0, o2)


def bf16_round(a):
    """Round FP64/FP32 values to bfloat16 (round to nearest even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
