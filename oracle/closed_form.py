"""Closed forms that pin the oracle (test infrastructure).

* Constant-coefficient periodic advection-diffusion-reaction: the discrete
  operator is diagonalised by the 2D DFT.  A Fourier mode e^{i(theta_x ix +
  theta_y iy)} with theta = 2 pi k / n is an eigenvector with eigenvalue
      lambda = nu (2cos theta_x - 2)/dx^2 + nu (2cos theta_y - 2)/dy^2
               - i (ax sin theta_x / dx + ay sin theta_y / dy) + r
  (the transpose flips the sign of the advection term).  Hence
      sum_k h^k phi_k(hA) b_k = sum_k h^k IDFT(phi_k(h lambda) DFT(b_k)).
* Diagonal A: phi_k acts elementwise (oracle.phi.phi_combo_diag).
* Derivative along a coefficient direction (nu, ax, ay, r): d lambda is the
  eigenvalue of the direction's stencil (for nu the Laplacian's), and
  d/dz phi_k(z) = phi_k(z) - k phi_{k+1}(z) (differentiate the integral
  definition: the factor (1 - s) splits into phi_k and k phi_{k+1}), so
  d h^k phi_k(h lambda) = h^{k+1} (phi_k - k phi_{k+1})(h lambda) d lambda.
"""
from __future__ import annotations

import numpy as np

from .phi import phi_scalar


def adr_eigenvalues(op) -> np.ndarray:
    """Eigenvalues on the (ny, nx) DFT grid for the constant-coefficient ADR."""
    if op.field0 is not None:
        raise ValueError("closed form needs constant coefficients")
    tx = 2.0 * np.pi * np.fft.fftfreq(op.nx) * 1.0   # 2 pi kx / nx
    ty = 2.0 * np.pi * np.fft.fftfreq(op.ny)
    TX, TY = np.meshgrid(tx, ty)                    # (ny, nx)
    sgn = 1.0 if op.transpose else -1.0
    lam = (op.nu * (2.0 * np.cos(TX) - 2.0) / op.dx**2
           + op.nu * (2.0 * np.cos(TY) - 2.0) / op.dy**2
           + sgn * 1j * (op.ax * np.sin(TX) / op.dx + op.ay * np.sin(TY) / op.dy)
           + op.react)
    return lam


def adr_phi_combo(op, B: np.ndarray, h: float, p: int) -> np.ndarray:
    lam = adr_eigenvalues(op)
    acc = np.zeros((op.ny, op.nx), dtype=complex)
    for k in range(p + 1):
        bk = B[:, k].reshape(op.ny, op.nx)
        acc += (h ** k) * phi_scalar(k, h * lam) * np.fft.fft2(bk)
    return np.real(np.fft.ifft2(acc)).reshape(-1)


def adr_apply_spectral(op, x: np.ndarray) -> np.ndarray:
    """A x through the DFT (used to pin the stencil's eigenvalues)."""
    lam = adr_eigenvalues(op)
    X = np.fft.fft2(x.reshape(op.ny, op.nx))
    return np.real(np.fft.ifft2(lam * X)).reshape(-1)


def adr_laplacian_eigenvalues(op) -> np.ndarray:
    """Eigenvalues of the 5-point Laplacian on the (ny, nx) DFT grid."""
    tx = 2.0 * np.pi * np.fft.fftfreq(op.nx)
    ty = 2.0 * np.pi * np.fft.fftfreq(op.ny)
    TX, TY = np.meshgrid(tx, ty)
    return (2.0 * np.cos(TX) - 2.0) / op.dx**2 + (2.0 * np.cos(TY) - 2.0) / op.dy**2


def adr_phi_combo_dnu(op, B: np.ndarray, h: float, p: int) -> np.ndarray:
    """d/dnu of sum_k h^k phi_k(h A(nu)) b_k for the constant-coefficient ADR."""
    return _adr_phi_combo_deriv(op, adr_laplacian_eigenvalues(op), B, h, p)


def adr_phi_combo_deriv(op, dop, B: np.ndarray, h: float, p: int) -> np.ndarray:
    """Derivative of sum_k h^k phi_k(h A) b_k along the constant-coefficient
    ADR direction dop (same grid and transpose flag as op): A and dA share
    the DFT eigenvectors, and the eigenvalues of dA are those of an ADR
    operator with dop's coefficients (linear in them)."""
    return _adr_phi_combo_deriv(op, adr_eigenvalues(dop), B, h, p)


def _adr_phi_combo_deriv(op, dlam, B, h, p):
    lam = adr_eigenvalues(op)
    acc = np.zeros((op.ny, op.nx), dtype=complex)
    for k in range(p + 1):
        bk = B[:, k].reshape(op.ny, op.nx)
        dphi = phi_scalar(k, h * lam) - k * phi_scalar(k + 1, h * lam)
        acc += (h ** (k + 1)) * dphi * dlam * np.fft.fft2(bk)
    return np.real(np.fft.ifft2(acc)).reshape(-1)
