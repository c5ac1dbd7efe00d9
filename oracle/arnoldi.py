"""Arnoldi processes (oracle, test infrastructure).

Three processes build a basis V and Hessenberg H of the Krylov space K_m(A, b)
with A V_m = V_m H_m + h_{m+1,m} v_{m+1} e_m^T (Section 2.2, eq.
arnoldidecomp1); the first two keep V orthonormal:

* MGSArnoldi: Arnoldi with modified Gram-Schmidt (Algorithm 1): after each
  matrix-vector product, the new vector is orthogonalised against v_1..v_j one
  inner product at a time, then normalised.  Lucky breakdown when the norm is
  negligible.

* HybridArnoldi: the hybrid low-synchronisation Arnoldi (Algorithm 4).  Every
  step takes one grouped reduction temp = V_{1:j+1}^T [v_j, v_{j+1}] (eq.
  output_wywnrm), normalises the previous vector with its true (lagged) norm,
  forms the correction matrix T ~ (V^T V)^{-1} by one of
      'cwy'   T_j row by the compact-WY recursion (Algorithm 5, eq. recursionForT)
      'ncwy'  T ~ I - L, truncated Neumann series (Algorithm 6)
      'gsmgs' T = M^{-1}[I + N M^{-1}], M = I + L, N = -L^T, two Gauss-Seidel
              sweeps on the normal equations (Algorithm 7)
  projects, and "normalises" the new vector by the Pythagorean norm estimate
  (eq. nrmest).

Readings of the printed Algorithm 4 (garbled in places) used here:
  * The rescale by the previous norm estimate is applied to the vectors AND to
    the reduction results, so the reduction returns the true norm of the
    previous vector as the text of Section 3.2.1 says it must.
  * The true norm is the subdiagonal entry H_{j,j-1}; H_{1,1} = temp_{1,2}
    (T_1 = [1]); the projection uses H_{1:j,j}.
  * The sum ss uses the reduction's second column (eq. nrmest summed over
    i = 1..j).  If temp_{j+1,2} - ss <= delta * temp_{j+1,2} the exact norm
    (one extra reduction) replaces the estimate.  Lucky breakdown when the
    norm is <= eps_bd * ||w||.
  * The last subdiagonal H_{m+1,m} is the norm of the projected (not yet
    estimate-normalised) vector v_{m+1}.

* IOPArnoldi: the incomplete orthogonalisation process (Section 2.3.1) in its
  classical Gram-Schmidt form, ioCGS, the baseline of the paper's runtime
  ratios (Section 4.2): the new vector is orthogonalised against only the
  previous `window` basis vectors (two, as in KIOPS), all of their inner
  products taken from the same vector (one reduction, the classical form),
  then normalised by its norm (a second reduction).  H keeps its Hessenberg
  shape but has at most `window` entries above the subdiagonal per column,
  and V is not orthonormal, so V_m^T A V_m differs from H_m.
"""
from __future__ import annotations

import math

import numpy as np


class MGSArnoldi:
    """Algorithm 1.  State can be extended to a larger m (basis reuse)."""

    def __init__(self, apply, b: np.ndarray, m_cap: int, eps_bd: float = 1e-12):
        self.apply = apply
        self.n = len(b)
        self.V = np.zeros((self.n, m_cap + 1), order="F")
        self.H = np.zeros((m_cap + 1, m_cap))
        self.beta = float(np.linalg.norm(b))
        self.eps_bd = eps_bd
        self.j = 0
        self.breakdown = False
        if self.beta > 0.0:
            self.V[:, 0] = b / self.beta

    def extend(self, m: int) -> int:
        """Run steps until j == m or lucky breakdown; returns j."""
        while self.j < m and not self.breakdown:
            j = self.j                          # 0-based column of v_{j+1}
            w = self.apply(self.V[:, j])
            wnorm = np.linalg.norm(w)
            for i in range(j + 1):
                hij = float(self.V[:, i] @ w)
                self.H[i, j] = hij
                w -= hij * self.V[:, i]
            nrm = float(np.linalg.norm(w))
            self.j += 1
            if nrm <= self.eps_bd * wnorm:
                self.H[j + 1, j] = 0.0
                self.breakdown = True
                break
            self.H[j + 1, j] = nrm
            self.V[:, j + 1] = w / nrm
        return self.j


class IOPArnoldi:
    """Incomplete orthogonalisation with classical Gram-Schmidt (ioCGS),
    Section 2.3.1.  Same interface as MGSArnoldi."""

    def __init__(self, apply, b: np.ndarray, m_cap: int, window: int = 2,
                 eps_bd: float = 1e-12):
        if window < 1:
            raise ValueError(window)
        self.apply = apply
        self.window = window
        self.n = len(b)
        self.V = np.zeros((self.n, m_cap + 1), order="F")
        self.H = np.zeros((m_cap + 1, m_cap))
        self.beta = float(np.linalg.norm(b))
        self.eps_bd = eps_bd
        self.j = 0
        self.breakdown = False
        if self.beta > 0.0:
            self.V[:, 0] = b / self.beta

    def extend(self, m: int) -> int:
        """Run steps until j == m or lucky breakdown; returns j."""
        while self.j < m and not self.breakdown:
            j = self.j                          # 0-based column of v_{j+1}
            w = self.apply(self.V[:, j])
            wnorm = float(np.linalg.norm(w))
            lo = max(0, j - self.window + 1)
            h = self.V[:, lo:j + 1].T @ w       # all window products from w
            self.H[lo:j + 1, j] = h
            w = w - self.V[:, lo:j + 1] @ h
            nrm = float(np.linalg.norm(w))
            self.j += 1
            if nrm <= self.eps_bd * wnorm:
                self.H[j + 1, j] = 0.0
                self.breakdown = True
                break
            self.H[j + 1, j] = nrm
            self.V[:, j + 1] = w / nrm
        return self.j


class HybridArnoldi:
    """Algorithm 4 with the correction matrix of Algorithm 5/6/7."""

    def __init__(self, apply, b: np.ndarray, m_cap: int, tform: str = "gsmgs",
                 delta: float = 1e-10, eps_bd: float = 1e-12):
        if tform not in ("cwy", "ncwy", "gsmgs"):
            raise ValueError(tform)
        self.apply = apply
        self.tform = tform
        self.delta = delta
        self.eps_bd = eps_bd
        self.n = len(b)
        self.V = np.zeros((self.n, m_cap + 2), order="F")
        self.H = np.zeros((m_cap + 1, m_cap))
        self.T = np.eye(m_cap)          # CWY / NCWY correction matrix
        self.M = np.eye(m_cap)          # GSMGS: M = I + L
        self.Minv = np.eye(m_cap)       # GSMGS: M^{-1}
        self.Nm = np.zeros((m_cap, m_cap))  # GSMGS: N = -L^T
        self.V[:, 0] = b                # v_1 = b, normalised lazily at step 1
        self.nrm_est = 1.0
        self.beta = None
        self.j = 0
        self.breakdown = False
        self.n_fallback = 0

    # -- correction matrices (Algorithms 5, 6, 7) -------------------------
    def _form_T(self, temp, j):
        """Returns H_{1:j,j}; j is 1-based.  temp is (j+1) x 2."""
        l_row = temp[:j - 1, 0]          # (V_{1:j-1}^T v_j)^T, row j of L
        b = temp[:j, 1]                  # V_j^T v_{j+1}
        if self.tform == "cwy":
            if j > 1:
                self.T[j - 1, :j - 1] = cwy_row(l_row, self.T[:j - 1, :j - 1])
            return self.T[:j, :j] @ b
        if self.tform == "ncwy":
            if j > 1:
                self.T[j - 1, :j - 1] = ncwy_row(l_row)
            return self.T[:j, :j] @ b
        if j > 1:
            self.M[j - 1, :j - 1] = l_row
            self.Nm[:j - 1, j - 1] = -l_row
            self.Minv[j - 1, :j - 1] = cwy_row(l_row, self.Minv[:j - 1, :j - 1])
        return gsmgs_apply(self.M[:j, :j], self.Minv[:j, :j], self.Nm[:j, :j], b)

    def extend(self, m: int) -> int:
        """Run steps until j == m or lucky breakdown; closes H_{m+1,m}."""
        V = self.V
        while self.j < m and not self.breakdown:
            self.j += 1
            j = self.j                                   # 1-based step index
            V[:, j] = self.apply(V[:, j - 1])            # v_{j+1} = A v_j
            temp = V[:, :j + 1].T @ V[:, j - 1:j + 1]    # the one reduction
            if j > 1:
                g = self.nrm_est                         # rescale vectors and
                V[:, j - 1:j + 1] *= g                   # the reduction results
                temp *= g
                temp[j - 1:j + 1, :] *= g
            true_nrm = math.sqrt(temp[j - 1, 0])
            if j == 1:
                self.beta = true_nrm
                if true_nrm == 0.0:
                    self.breakdown = True
                    self.j = 0
                    return 0
            V[:, j - 1:j + 1] /= true_nrm
            temp[:, 1] /= true_nrm
            temp[j - 1:j + 1, 1] /= true_nrm
            if j > 1:
                temp[:j - 1, 0] /= true_nrm
                self.H[j - 1, j - 2] = true_nrm          # subdiagonal, lagged
            self.H[:j, j - 1] = self._form_T(temp, j)
            V[:, j] -= V[:, :j] @ self.H[:j, j - 1]      # project
            ss = float(np.sum(temp[:j, 1] ** 2))
            wn2 = temp[j, 1]
            if wn2 - ss <= self.delta * wn2:
                self.n_fallback += 1
                nrm = float(np.linalg.norm(V[:, j]))     # extra reduction
            else:
                nrm = math.sqrt(wn2 - ss)
            if nrm <= self.eps_bd * math.sqrt(wn2):
                self.breakdown = True
                self.H[j, j - 1] = 0.0
                break
            V[:, j] /= nrm
            self.nrm_est = nrm
        if not self.breakdown and self.j > 0:
            # final reduction: norm of the last (projected) vector
            j = self.j
            nrm = float(np.linalg.norm(V[:, j]))
            self.H[j, j - 1] = self.nrm_est * nrm
        return self.j

    def basis(self) -> np.ndarray:
        """Orthonormal basis V_{1:j+1}; the last column normalised exactly."""
        j = self.j
        Vb = self.V[:, :j + 1].copy()
        if not self.breakdown and j > 0:
            Vb[:, j] /= np.linalg.norm(Vb[:, j])
        return Vb


def cwy_row(l_row: np.ndarray, T_prev: np.ndarray) -> np.ndarray:
    """New row of T_j = (I + L_j)^{-1} from the compact-WY recursion
    T_j = [[T_{j-1}, 0], [-(V_{j-1}^T v_j)^T T_{j-1}, 1]]  (eq. recursionForT)."""
    return -(l_row @ T_prev)


def ncwy_row(l_row: np.ndarray) -> np.ndarray:
    """New row of T ~ I - L (two terms of the Neumann series, Algorithm 6)."""
    return -l_row


def gsmgs_apply(M: np.ndarray, Minv: np.ndarray, N: np.ndarray, b: np.ndarray):
    """x = M^{-1}[I + N M^{-1}] b: the mat-vec p = b + N (M^{-1} b), then the
    lower-triangular solve M x = p by forward substitution (Algorithm 7)."""
    pvec = b + N @ (Minv @ b)
    j = len(b)
    x = np.zeros(j)
    for i in range(j):
        x[i] = (pvec[i] - M[i, :i] @ x[:i]) / M[i, i]
    return x
