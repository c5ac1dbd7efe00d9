"""Exponential integrators driving the phi combination (oracle, test
infrastructure only).

Section 4.1 of arXiv:2410.14917 uses the phi combination inside exponential
integrators for u' = f(u), with J_n the Jacobian of f at u_n and the
nonlinear remainder R(v) = f(v) - f(u_n) - J_n (v - u_n):

  EPI-q (multistep, eq. epi4): with P previous states u_{n-1}, .., u_{n-P},
      u_{n+1} = u_n + phi_1(h J_n) h f_n + sum_{m=1}^{M} phi_m(h J_n) v_m,
      v_m = sum_{i=1}^{P} alpha_{m,i} h R(u_{n-i}),
    with the coefficient matrices A_q = (alpha_{m,i}) the paper prints for
    q = 4 (M = 3, P = 2) and q = 5 (M = 4, P = 3).  The printed A_6 does not
    satisfy even the third-order conditions (see the order-condition pin), so
    EPI6 is not offered.
  SRERK3 (eq. epirk4, first form):
      z_1 = u_n + phi_1(3/4 h J_n) 3/4 h f(u_n),
      u_{n+1} = u_n + phi_1(h J_n) h f(u_n) + phi_3(h J_n) 32/9 h R(z_1).

Each phi-term sum is one phi combination sum_{k=0}^{p} h^k phi_k(hA) b_k
(Section 2.1) with b_0 = 0, b_1 = f_n and b_m = v_m / h^m, so an EPI step is
one call and an SRERK3 step two (Section 4.1 counts the same).

The paper does not say how a multistep method gets its first P states.  Here
they come from SRERK3, each of the first P steps taken as `start_substeps`
equal SRERK3 steps (this project's choice; the library does the same).

Problems (workloads.Rhs):
  allen_cahn  f(u) = nu Lap u + u - u^3,       J = nu Lap + diag(1 - 3u^2)
  adr         f(u) = nu Lap u - ax Dx u - ay Dy u + gamma u (u - 1/2)(1 - u),
              J = nu Lap - ax Dx - ay Dy + diag(gamma (-3u^2 + 3u - 1/2))
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

from . import krylov, operators

RHS_ALLEN_CAHN, RHS_ADR = 0, 1
EPI4, EPI5, SRERK3 = 0, 1, 2

# the coefficient matrices alpha_{m,i} printed in Section 4.1 (rows m = 1..M,
# columns i = 1..P); the first row is zero in both
EPI_ALPHA = {
    EPI4: [[Fr(0), Fr(0)],
           [Fr(-3, 10), Fr(3, 40)],
           [Fr(32, 5), Fr(-11, 10)]],
    EPI5: [[Fr(0), Fr(0), Fr(0)],
           [Fr(-4, 5), Fr(2, 5), Fr(-4, 45)],
           [Fr(12), Fr(-9, 2), Fr(8, 9)],
           [Fr(3), Fr(0), Fr(-1, 3)]],
}


def history_length(method: int) -> int:
    """P: previous states a step of the method reads (0 for SRERK3)."""
    return len(EPI_ALPHA[method][0]) if method in EPI_ALPHA else 0


def _linear_op(rhs, field=None):
    """workloads.Operator of the linear part of f (ADR kind) with an optional
    diagonal field."""
    from workloads import Operator, OP_ADR
    return Operator(kind=OP_ADR, nx=rhs.nx, ny=rhs.ny, nu=rhs.nu, ax=rhs.ax, ay=rhs.ay,
                    dx=rhs.dx, dy=rhs.dy, field0=field)


def f(rhs, u: np.ndarray) -> np.ndarray:
    """The right-hand side f(u)."""
    lin = operators.apply(_linear_op(rhs), u)
    if rhs.kind == RHS_ALLEN_CAHN:
        return lin + u - u ** 3
    if rhs.kind == RHS_ADR:
        return lin + rhs.gamma * u * (u - 0.5) * (1.0 - u)
    raise ValueError(rhs.kind)


def jacobian(rhs, u: np.ndarray):
    """The Jacobian of f at u as a matrix-free operator (workloads.Operator)."""
    from workloads import Operator, OP_ALLEN_CAHN
    if rhs.kind == RHS_ALLEN_CAHN:
        return Operator(kind=OP_ALLEN_CAHN, nx=rhs.nx, ny=rhs.ny, nu=rhs.nu, dx=rhs.dx,
                        dy=rhs.dy, field0=np.asarray(u, dtype=np.float64))
    if rhs.kind == RHS_ADR:
        return _linear_op(rhs, rhs.gamma * (-3.0 * u * u + 3.0 * u - 0.5))
    raise ValueError(rhs.kind)


def krylov_solver(tol=1e-12, m_max=64, **kw):
    """phi combination solver (op, B columns (N x (p+1)), h, p) -> y by the
    oracle's substepped Krylov method."""
    def solve(op, B, h, p):
        y, info = krylov.phi_combo(op, B, h, p, tol=tol, m_max=m_max, **kw)
        if info.status != krylov.STATUS_OK:
            raise RuntimeError(f"phi combination failed: {info}")
        return y
    return solve


def dense_solver(op, B, h, p):
    """phi combination by the dense augmented-matrix exponential (tiny grids)."""
    from . import phi
    return phi.phi_combo_dense(operators.dense(op), B, h, p)


def remainder(rhs, Jn, un, fn, v, fv):
    """R(v) = f(v) - f(u_n) - J_n (v - u_n)."""
    return fv - fn - operators.apply(Jn, v - un)


def srerk3_step(rhs, u, h, solve):
    """One SRERK3 step (two phi combinations)."""
    n = len(u)
    fn = f(rhs, u)
    Jn = jacobian(rhs, u)
    B1 = np.zeros((n, 2))
    B1[:, 1] = fn
    z1 = u + solve(Jn, B1, 0.75 * h, 1)
    R = remainder(rhs, Jn, u, fn, z1, f(rhs, z1))
    B2 = np.zeros((n, 4))
    B2[:, 1] = fn
    B2[:, 3] = (32.0 / 9.0) * h * R / h ** 3
    return u + solve(Jn, B2, h, 3)


def epi_step(rhs, us, fs, h, method, solve):
    """One EPI step from u_n = us[0] with the previous states us[1..P] and
    their right-hand sides fs (fs[0] = f(u_n)); one phi combination."""
    alpha = EPI_ALPHA[method]
    M, P = len(alpha), len(alpha[0])
    un, fn = us[0], fs[0]
    Jn = jacobian(rhs, un)
    R = [remainder(rhs, Jn, un, fn, us[i], fs[i]) for i in range(1, P + 1)]
    B = np.zeros((len(un), M + 1))
    B[:, 1] = fn
    for m in range(2, M + 1):
        v = h * sum(float(alpha[m - 1][i - 1]) * R[i - 1] for i in range(1, P + 1))
        B[:, m] = v / h ** m
    return un + solve(Jn, B, h, M)


def integrate(rhs, u0, h, nsteps, method, solve, start_substeps=4, start=None):
    """u after nsteps steps of size h from u0.  Multistep methods take their
    first P steps by SRERK3 with start_substeps substeps each, unless
    `start` gives the states u_1..u_P."""
    P = history_length(method)
    u = np.asarray(u0, dtype=np.float64).copy()
    if P == 0:
        for _ in range(nsteps):
            u = srerk3_step(rhs, u, h, solve)
        return u
    hist = [u]                                   # newest first: u_n, u_{n-1}, ...
    for k in range(min(P, nsteps)):
        if start is not None:
            u = np.asarray(start[k], dtype=np.float64).copy()
        else:
            for _ in range(start_substeps):
                u = srerk3_step(rhs, u, h / start_substeps, solve)
        hist.insert(0, u)
    hist = hist[:P + 1]
    fs = [f(rhs, v) for v in hist]
    for _ in range(nsteps - min(P, nsteps)):
        u = epi_step(rhs, hist, fs, h, method, solve)
        hist = [u] + hist[:P]
        fs = [f(rhs, u)] + fs[:P]
    return hist[0]
