"""Derivatives of the phi combination (oracle, test infrastructure).

y(B, A) = sum_{k=0}^p h^k phi_k(hA) b_k = [I 0] exp(h Atilde) z (Section 2.1).

* Directional derivative in the operator, dy = d/de y(B, A + e dA):
  for the block matrix M = [[Atilde, Etilde], [0, Atilde]] with
  Etilde = [[dA, 0], [0, 0]], exp(h M) = [[exp(h Atilde), L], [0, exp(h Atilde)]]
  where L is the Frechet derivative of the exponential at h Atilde in the
  direction h Etilde (Van Loan, IEEE Trans. Automat. Control 23 (1978)), so
  exp(h M) [0; z] = [dy_aug; y_aug].  phi_combo_tangent applies exp(h M) to
  [0; z] with the same substepped Krylov driver as the phi combination
  (oracle.krylov.expmv), on vectors [a; c] of two augmented vectors.
* Gradient with respect to b_k of <g, y>: h^k phi_k(h A^T) g, which is the
  phi combination of the transposed operator with B = [0, ..., 0, g].
"""
from __future__ import annotations

import numpy as np

from . import operators
from .krylov import aug_apply, balance_scale, expmv, start_vector


def tangent_apply(op, dop, B: np.ndarray, p: int, mu: float, x: np.ndarray) -> np.ndarray:
    """M [a; c] = [Atilde a + Etilde c; Atilde c] (a, c augmented, N + p each)."""
    n, n1 = op.n, op.n + p
    a, c = x[:n1], x[n1:]
    ya = aug_apply(op, B, p, mu, a)
    ya[:n] += operators.apply(dop, c[:n])
    yc = aug_apply(op, B, p, mu, c)
    return np.concatenate([ya, yc])


def phi_combo_tangent(op, dop, B: np.ndarray, h: float, p: int, **kw):
    """(y, dy, Info): the phi combination and its derivative along the
    operator direction dop (an operator whose apply is dA)."""
    B = np.asarray(B, dtype=np.float64)
    n, n1 = op.n, op.n + p
    mu = balance_scale(B, p)
    z = start_vector(B, p, mu)
    w0 = np.concatenate([np.zeros(n1), z])
    r, info = expmv(lambda x: tangent_apply(op, dop, B, p, mu, x), w0, h, **kw)
    return r[n1:n1 + n].copy(), r[:n].copy(), info


def grad_B(op, g: np.ndarray, h: float, p: int, phi_combo, **kw) -> np.ndarray:
    """Columns h^k phi_k(h A^T) g, k = 0..p, by the given phi-combination
    routine (Krylov or closed form) applied to the transposed operator."""
    opt = op.with_transpose(not op.transpose)
    n = op.n
    G = np.zeros((n, p + 1))
    for k in range(p + 1):
        Bk = np.zeros((n, k + 1))
        Bk[:, k] = g
        r = phi_combo(opt, Bk, h, k, **kw)
        G[:, k] = r[0] if isinstance(r, tuple) else r
    return G
