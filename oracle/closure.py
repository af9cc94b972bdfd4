"""Plain FP64 reference of the closure's training signal (test infrastructure).

For shear flow along x, the steady state of the gray model of Sec. 4 (eq.
GeneralizedPor2 with the porous force of eq. PorousForce, Forchheimer term
zero) satisfies in every cell
    d/dz (nu_eff dU/dz) - drag U + eps G = 0,
with U = 0 at the two walls, which lie half a cell outside the first and the
last fluid cell.  Discretisation on the cells 1..nz-2 (the layers 0 and nz-1
are walls): the flux through the face between two cells is the mean of their
viscosities times the difference of their velocities; at a wall the slope is
taken from the parabola through the wall zero and the two nearest cells,
U'(wall) = 3 U_1 - U_2 / 3.

The loss of one profile is sum (U - u_target)^2 / sum u_target^2 over the
fluid cells, scaled by weight / nprof; its gradient with respect to the
closure outputs follows from the adjoint: with A U = b and A^T lam = dL/dU,
dL/dp = -lam^T (dA/dp) U for every coefficient p, and A is linear in the
viscosities and drags, so dA/dp is the matrix assembled from a unit vector.
"""
from __future__ import annotations

import numpy as np


def assemble(nu, drag):
    """Matrix of the steady system on the n interior cells for viscosities
    nu[n] and drags drag[n]."""
    nu = np.asarray(nu, dtype=np.float64)
    drag = np.asarray(drag, dtype=np.float64)
    n = len(nu)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] -= drag[i]
        # lower side
        if i == 0:
            A[i, i] -= 3.0 * nu[i]
            A[i, i + 1] += nu[i] / 3.0
        else:
            f = 0.5 * (nu[i - 1] + nu[i])
            A[i, i] -= f
            A[i, i - 1] += f
        # upper side
        if i == n - 1:
            A[i, i] -= 3.0 * nu[i]
            A[i, i - 1] += nu[i] / 3.0
        else:
            f = 0.5 * (nu[i] + nu[i + 1])
            A[i, i] -= f
            A[i, i + 1] += f
    return A


def steady_profile(eps, nu_eff, drag, G):
    """U[nz] of one column (0 in the wall layers)."""
    eps = np.asarray(eps, dtype=np.float64)
    nz = len(eps)
    A = assemble(nu_eff[1:nz - 1], drag[1:nz - 1])
    U = np.zeros(nz)
    U[1:nz - 1] = np.linalg.solve(A, -eps[1:nz - 1] * G)
    return U


def closure_map(Y, eps, nu):
    s = 1.0 - np.asarray(eps, dtype=np.float64)
    return nu * np.exp(s * Y[:, 0]), s * np.logaddexp(0.0, Y[:, 1])


def profile_loss(Y, eps, u_target, nprof, nz, nu, G, weight):
    """Loss per profile and dL/dY (rows p*nz + z, 16 columns)."""
    Y = np.asarray(Y, dtype=np.float64)
    losses = np.zeros(nprof)
    dY = np.zeros((nprof * nz, Y.shape[1]))
    for p in range(nprof):
        rows = slice(p * nz, (p + 1) * nz)
        e = np.asarray(eps[rows], dtype=np.float64)
        t = np.asarray(u_target[rows], dtype=np.float64)
        nue, drag = closure_map(Y[rows], e, nu)
        inner = slice(1, nz - 1)
        A = assemble(nue[inner], drag[inner])
        U = np.linalg.solve(A, -e[inner] * G)
        w = weight / nprof / max(float((t[inner] ** 2).sum()), 1e-300)
        r = U - t[inner]
        losses[p] = w * float((r * r).sum())
        lam = np.linalg.solve(A.T, 2.0 * w * r)
        n = nz - 2
        gnu = np.zeros(n)
        gdr = np.zeros(n)
        zero = np.zeros(n)
        for i in range(n):
            unit = np.zeros(n)
            unit[i] = 1.0
            gnu[i] = -lam @ assemble(unit, zero) @ U
            gdr[i] = -lam @ assemble(zero, unit) @ U
        s = 1.0 - e[inner]
        sig = 1.0 / (1.0 + np.exp(-Y[rows][inner, 1]))
        dY[p * nz + 1:(p + 1) * nz - 1, 0] = gnu * nue[inner] * s
        dY[p * nz + 1:(p + 1) * nz - 1, 1] = gdr * s * sig
    return losses, dY
