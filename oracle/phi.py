"""phi-functions and the dense matrix exponential (oracle, test infrastructure).

phi_0(z) = e^z and phi_k(z) = int_0^1 e^{(1-theta) z} theta^{k-1}/(k-1)! dtheta
(Section 2, eq. phi_int_def).  They satisfy phi_k(0) = 1/k! and the recurrence
phi_k(z) = (phi_{k-1}(z) - 1/(k-1)!) / z, which follows from integrating the
definition by parts.

The dense exponential is a Taylor series with scaling and squaring: the matrix
is scaled by 2^-s until its 1-norm is at most 1/2, the series is summed until
the terms stop contributing, and the result is squared s times.  (The GPU
evaluates a fixed-degree polynomial by a different scheme and scaling; the two
share no code.)

The phi combination sum_k h^k phi_k(hA) b_k is defined here as the top block of
exp(h * Atilde) [b_0; e_p] with Atilde = [[A, B], [0, K]], B = [b_p, ..., b_1],
K the p x p upper shift and e_p the p-th unit vector (Section 2.1, eq.
philincomb, with the step h placed as in the left-hand side of that equation).
Pinned by: quadrature of the integral definition, eigen-decomposition and
nilpotent closed forms, and diagonal / DFT closed forms (tests/test_oracle_phi.py).
"""
from __future__ import annotations

import math

import numpy as np


def phi_scalar(k: int, z):
    """phi_k(z) for scalar or array z (real or complex)."""
    z = np.asarray(z)
    out = np.empty(z.shape, dtype=np.result_type(z.dtype, np.float64))
    small = np.abs(z) <= 1.0
    zs = z[small]
    # series  phi_k(z) = sum_n z^n / (n+k)!   (|z| <= 1: 40 terms are ample)
    acc = np.zeros(zs.shape, dtype=out.dtype)
    term = np.full(zs.shape, 1.0 / math.factorial(k), dtype=out.dtype)
    for n in range(40):
        acc = acc + term
        term = term * zs / (n + k + 1)
    out[small] = acc
    zl = z[~small]
    val = np.exp(zl)
    for j in range(1, k + 1):
        val = (val - 1.0 / math.factorial(j - 1)) / zl
    out[~small] = val
    return out if out.shape else out[()]


def expm_taylor(X: np.ndarray) -> np.ndarray:
    """exp(X) by Taylor series with scaling and squaring (dense, float64)."""
    X = np.asarray(X, dtype=np.result_type(X.dtype, np.float64))
    n = X.shape[0]
    norm1 = np.max(np.sum(np.abs(X), axis=0)) if n else 0.0
    s = 0
    if norm1 > 0.5:
        s = int(math.ceil(math.log2(norm1 / 0.5)))
    Xs = X / (2.0 ** s)
    E = np.eye(n, dtype=X.dtype)
    term = np.eye(n, dtype=X.dtype)
    for k in range(1, 40):
        term = term @ Xs / k
        E = E + term
        if np.max(np.abs(term)) <= 1e-18 * np.max(np.abs(E)):
            break
    for _ in range(s):
        E = E @ E
    return E


def augmented_matrix(A: np.ndarray, B: np.ndarray, p: int) -> np.ndarray:
    """Atilde = [[A, Bhat], [0, K]] with Bhat = [b_p, ..., b_1] and K the p x p
    upper shift (ones on the superdiagonal).  B holds columns b_0..b_p."""
    n = A.shape[0]
    At = np.zeros((n + p, n + p))
    At[:n, :n] = A
    for c in range(p):               # column c of Bhat is b_{p-c}
        At[:n, n + c] = B[:, p - c]
    for c in range(p - 1):
        At[n + c, n + c + 1] = 1.0
    return At


def phi_combo_dense(A: np.ndarray, B: np.ndarray, h: float, p: int) -> np.ndarray:
    """sum_{k=0}^p h^k phi_k(hA) b_k via the augmented exponential (dense)."""
    n = A.shape[0]
    At = augmented_matrix(A, B, p)
    z = np.zeros(n + p)
    z[:n] = B[:, 0]
    if p > 0:
        z[n + p - 1] = 1.0
    return (expm_taylor(h * At) @ z)[:n]


def phi_combo_diag(d: np.ndarray, B: np.ndarray, h: float, p: int) -> np.ndarray:
    """Closed form for diagonal A = diag(d): elementwise sum_k h^k phi_k(h d) b_k."""
    y = np.zeros(len(d), dtype=np.result_type(d.dtype, np.float64))
    for k in range(p + 1):
        y = y + (h ** k) * phi_scalar(k, h * d) * B[:, k]
    return y
