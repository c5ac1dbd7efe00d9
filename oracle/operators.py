"""Matrix-free 2D periodic operators (oracle, test infrastructure).

The paper's test problems are discretised by second-order finite differences
(Section 4.3); here the grids are periodic, point (ix, iy) is stored at index
iy * nx + ix (x fastest), E/W are ix +- 1 and N/S are iy +- 1 (wrapping).

  ADR          (A u) = nu * Lap u - ax * Dx u - ay * Dy u + react * u + d .* u
  Allen-Cahn   (A u) = nu * Lap u + (1 - 3 U^2) .* u         (U = field0)
  Brusselator  Jacobian of  u_t = Du Lap u + a - (b+1) u + u^2 v,
                            v_t = Dv Lap v + b u - u^2 v
               at (U, V) = (field0, field1); vector = [u-plane; v-plane].

Lap is the 5-point Laplacian (u_E + u_W - 2u)/dx^2 + (u_N + u_S - 2u)/dy^2 and
Dx, Dy are centred differences (u_E - u_W)/(2 dx), (u_N - u_S)/(2 dy).
The transposes use Lap^T = Lap and Dx^T = -Dx on a periodic grid.
Pinned by dense-matrix consistency, symmetry of the transpose and the DFT
eigenvalues of the constant-coefficient stencil (tests/test_oracle_operators.py).
"""
from __future__ import annotations

import numpy as np

OP_ADR, OP_ALLEN_CAHN, OP_BRUSSELATOR = 0, 1, 2


def _lap(u2, dx, dy):
    return ((np.roll(u2, -1, axis=1) + np.roll(u2, 1, axis=1) - 2.0 * u2) / dx**2
            + (np.roll(u2, -1, axis=0) + np.roll(u2, 1, axis=0) - 2.0 * u2) / dy**2)


def _dx(u2, dx):
    # (u_E - u_W) / (2 dx);  u_E at ix+1 is np.roll(u, -1, axis=1)
    return (np.roll(u2, -1, axis=1) - np.roll(u2, 1, axis=1)) / (2.0 * dx)


def _dy(u2, dy):
    return (np.roll(u2, -1, axis=0) - np.roll(u2, 1, axis=0)) / (2.0 * dy)


def apply(op, x: np.ndarray) -> np.ndarray:
    """y = A x (or A^T x when op.transpose)."""
    nx, ny = op.nx, op.ny
    npt = nx * ny
    if op.kind == OP_ADR:
        u = x.reshape(ny, nx)
        sgn = 1.0 if op.transpose else -1.0
        y = (op.nu * _lap(u, op.dx, op.dy) + sgn * op.ax * _dx(u, op.dx)
             + sgn * op.ay * _dy(u, op.dy) + op.react * u)
        y = y.reshape(-1)
        if op.field0 is not None:
            y = y + op.field0 * x
        return y
    if op.kind == OP_ALLEN_CAHN:
        u = x.reshape(ny, nx)
        y = op.nu * _lap(u, op.dx, op.dy)
        return y.reshape(-1) + (1.0 - 3.0 * op.field0 ** 2) * x
    if op.kind == OP_BRUSSELATOR:
        U, V = op.field0, op.field1
        a11 = -(op.brus_b + 1.0) + 2.0 * U * V
        a12 = U * U
        a21 = op.brus_b - 2.0 * U * V
        a22 = -U * U
        xu, xv = x[:npt], x[npt:]
        lu = op.nu * _lap(xu.reshape(ny, nx), op.dx, op.dy).reshape(-1)
        lv = op.nu2 * _lap(xv.reshape(ny, nx), op.dx, op.dy).reshape(-1)
        if op.transpose:
            yu = lu + a11 * xu + a21 * xv
            yv = lv + a12 * xu + a22 * xv
        else:
            yu = lu + a11 * xu + a12 * xv
            yv = lv + a21 * xu + a22 * xv
        return np.concatenate([yu, yv])
    raise ValueError(f"unknown operator kind {op.kind}")


def dense(op) -> np.ndarray:
    """Dense matrix of the operator, built column by column (tiny grids only)."""
    n = op.n
    A = np.zeros((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        A[:, i] = apply(op, e)
        e[i] = 0.0
    return A


def diffusion_part(op, x: np.ndarray) -> np.ndarray:
    """d(A x)/d(nu) for the ADR operator: Lap x (used by the adjoint)."""
    u = x.reshape(op.ny, op.nx)
    return _lap(u, op.dx, op.dy).reshape(-1)
