// Small Hessenberg exponential F = exp(tau Hbar) e_1 in one workgroup, float64.
//
// Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]] is (m+1) x (m+1); its last entry of
// F is the error estimate of the Krylov projection (eq. kryexp).  The method is
// the [13/13] Pade approximant with scaling and squaring (Higham, "The scaling
// and squaring method for the matrix exponential revisited", SIAM J. Matrix
// Anal. Appl. 26 (2005)): X = tau Hbar / 2^s with ||X||_1 <= theta_13,
// r(X) = q(X)^{-1} p(X) with p(X) = U + V, q(X) = V - U split into odd and even
// powers, then s squarings.  Only the first column is returned, so the last
// squaring is a matrix-vector product.
//
// Matrices are n x n row-major with stride kNmPad in the global scratch a.ex
// (a few tens of KiB, L2-resident).  Each product stages its two operands in
// LDS and accumulates 4x4 register blocks.  The linear solve is Gaussian
// elimination with partial pivoting in LDS.
#pragma once

#include "kp_internal.h"

namespace kp {

constexpr double kTheta13 = 5.371920351148152;   // Higham (2005), Table 2.3

// Pade [13/13] coefficients b_k of p(x) = sum b_k x^k (b_0 = 1), from
// b_k = b_{k-1} (13 - k + 1) / (k (26 - k + 1)).
__device__ inline void pade13_coeffs(double* b) {
  b[0] = 1.0;
  for (int k = 1; k <= 13; ++k) b[k] = b[k - 1] * (double)(14 - k) / ((double)k * (double)(27 - k));
}

// A linear combination c0*S0 + c1*S1 + c2*S2 + d*I of scratch matrices.
struct Lin {
  int s0, s1, s2;
  double c0, c1, c2, d;
};
__device__ inline Lin lin1(int s) { return Lin{s, -1, -1, 1.0, 0.0, 0.0, 0.0}; }

__device__ inline double* slot(const Args& a, int s) {
  return a.ex + (int64_t)s * kNmPad * kNmPad;
}

__device__ inline double lin_at(const Args& a, const Lin& L, int i, int k) {
  const int64_t o = (int64_t)i * kNmPad + k;
  double v = (i == k) ? L.d : 0.0;
  if (L.s0 >= 0) v += L.c0 * slot(a, L.s0)[o];
  if (L.s1 >= 0) v += L.c1 * slot(a, L.s1)[o];
  if (L.s2 >= 0) v += L.c2 * slot(a, L.s2)[o];
  return v;
}

// LDS tile (kNmPad x kNmPad) <- linear combination, zero outside n x n.
__device__ inline void load_lin(const Args& a, const Lin& L, int n, double* s) {
  for (int idx = kp_tid(); idx < kNmPad * kNmPad; idx += kThreads) {
    const int i = idx / kNmPad, k = idx - i * kNmPad;
    s[idx] = (i < n && k < n) ? lin_at(a, L, i, k) : 0.0;
  }
}

// slot[cs] = A * B + D   (A, B, D linear combinations), n x n.
__device__ inline void matmul(const Args& a, int n, const Lin& A, const Lin& B,
                              const Lin& D, int cs, double* sA, double* sB) {
  __syncthreads();
  load_lin(a, A, n, sA);
  load_lin(a, B, n, sB);
  __syncthreads();
  const int nb = (n + 3) >> 2;
  double* C = slot(a, cs);
  for (int blk = kp_tid(); blk < nb * nb; blk += kThreads) {
    const int bi = blk / nb, bj = blk - bi * nb;
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    for (int k = 0; k < n; ++k) {
      double av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = sA[(4 * bi + r) * kNmPad + k];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = sB[k * kNmPad + 4 * bj + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += av[r] * bv[c];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * bi + r;
      if (i >= n) continue;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = 4 * bj + c;
        if (k < n) C[(int64_t)i * kNmPad + k] = acc[r][c] + lin_at(a, D, i, k);
      }
    }
  }
  __syncthreads();
}

// Solve Q R = P in place (Q in sA, P in sB, both n x n): Gaussian elimination
// with partial pivoting, then back substitution; R is left in sB.
__device__ inline void lu_solve(int n, double* sA, double* sB) {
  __shared__ int s_piv;
  const int tid = kp_tid();
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {                      // pivot search by wave 0
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < n; i += 64) {
        const double v = fabs(sA[i * kNmPad + k]);
        if (v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) s_piv = bi;
    }
    __syncthreads();
    const int piv = s_piv;
    if (piv != k) {
      for (int c = tid; c < 2 * n; c += kThreads) {
        double* M = (c < n) ? sA : sB;
        const int cc = (c < n) ? c : c - n;
        const double t = M[k * kNmPad + cc];
        M[k * kNmPad + cc] = M[piv * kNmPad + cc];
        M[piv * kNmPad + cc] = t;
      }
      __syncthreads();
    }
    const double d = sA[k * kNmPad + k];
    for (int i = k + 1 + tid; i < n; i += kThreads) sA[i * kNmPad + k] /= d;
    __syncthreads();
    const int nr = n - k - 1;
    const int ncol = (n - k - 1) + n;
    for (int idx = tid; idx < nr * ncol; idx += kThreads) {
      const int i = k + 1 + idx / ncol;
      const int c = idx - (idx / ncol) * ncol;
      const double f = sA[i * kNmPad + k];
      if (c < n - k - 1) {
        const int cc = k + 1 + c;
        sA[i * kNmPad + cc] -= f * sA[k * kNmPad + cc];
      } else {
        const int cc = c - (n - k - 1);
        sB[i * kNmPad + cc] -= f * sB[k * kNmPad + cc];
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const double d = sA[k * kNmPad + k];
    for (int c = tid; c < n; c += kThreads) sB[k * kNmPad + c] /= d;
    __syncthreads();
    for (int idx = tid; idx < k * n; idx += kThreads) {
      const int i = idx / n, c = idx - i * n;
      sB[i * kNmPad + c] -= sA[i * kNmPad + k] * sB[k * kNmPad + c];
    }
    __syncthreads();
  }
}

// F[0..m] = exp(tau Hbar) e_1 for the Hessenberg H (column-major, leading
// dimension ldh) of size (m+1) x m; zero_sub drops h_{m+1,m} (lucky
// breakdown).  Whole workgroup; lds holds 2 * kNmPad^2 doubles.
__device__ inline void expm_hbar(const Args& a, const double* H, int ldh, int m,
                                 double tau, bool zero_sub, double* F, double* lds) {
  __shared__ double s_red[kWaves];
  __shared__ int s_s;
  double* sA = lds;
  double* sB = lds + kNmPad * kNmPad;
  const int n = m + 1;
  const int tid = kp_tid();
  double b[14];
  pade13_coeffs(b);
  // X = tau * Hbar into slot 0; column sums for the 1-norm
  double* X = slot(a, 0);
  for (int idx = tid; idx < n * n; idx += kThreads) {
    const int i = idx / n, k = idx - i * n;
    double v = 0.0;
    if (k < m && i <= k + 1) {
      v = H[(int64_t)k * ldh + i];
      if (zero_sub && k == m - 1 && i == m) v = 0.0;
    }
    X[(int64_t)i * kNmPad + k] = tau * v;
  }
  __syncthreads();
  double cmax = 0.0;
  for (int k = tid; k < n; k += kThreads) {
    double cs = 0.0;
    for (int i = 0; i < n; ++i) cs += fabs(X[(int64_t)i * kNmPad + k]);
    cmax = fmax(cmax, cs);
  }
  cmax = block_max(cmax, s_red);
  if (tid == 0) {
    int s = 0;
    if (isfinite(cmax) && cmax > kTheta13) {
      int e;
      const double r = frexp(cmax / kTheta13, &e);   // cmax/theta = r 2^e, r in [0.5,1)
      s = (r == 0.5) ? e - 1 : e;                    // smallest s: ratio <= 2^s
    }
    s_s = s;
  }
  __syncthreads();
  const int s = s_s;
  if (s > 0) {
    const double sc = ldexp(1.0, -s);
    for (int idx = tid; idx < n * n; idx += kThreads) {
      const int i = idx / n, k = idx - i * n;
      X[(int64_t)i * kNmPad + k] *= sc;
    }
  }
  const Lin none{-1, -1, -1, 0.0, 0.0, 0.0, 0.0};
  // slots: 0 = X, 1 = X^2, 2 = X^4, 3 = X^6, 4 = V, 5 = W
  matmul(a, n, lin1(0), lin1(0), none, 1, sA, sB);
  matmul(a, n, lin1(1), lin1(1), none, 2, sA, sB);
  matmul(a, n, lin1(2), lin1(1), none, 3, sA, sB);
  // V = X6 (b12 X6 + b10 X4 + b8 X2) + b6 X6 + b4 X4 + b2 X2 + b0 I
  matmul(a, n, lin1(3), Lin{3, 2, 1, b[12], b[10], b[8], 0.0},
         Lin{3, 2, 1, b[6], b[4], b[2], b[0]}, 4, sA, sB);
  // W = X6 (b13 X6 + b11 X4 + b9 X2) + b7 X6 + b5 X4 + b3 X2 + b1 I
  matmul(a, n, lin1(3), Lin{3, 2, 1, b[13], b[11], b[9], 0.0},
         Lin{3, 2, 1, b[7], b[5], b[3], b[1]}, 5, sA, sB);
  // U = X W  (slot 1; X^2 is no longer needed)
  matmul(a, n, lin1(0), lin1(5), none, 1, sA, sB);
  // (V - U) R = (V + U)
  __syncthreads();
  load_lin(a, Lin{4, 1, -1, 1.0, -1.0, 0.0, 0.0}, n, sA);
  load_lin(a, Lin{4, 1, -1, 1.0, 1.0, 0.0, 0.0}, n, sB);
  __syncthreads();
  lu_solve(n, sA, sB);
  // R -> slot 0, then s-1 squarings (alternating slots 0 and 2)
  double* R = slot(a, 0);
  for (int idx = tid; idx < n * n; idx += kThreads) {
    const int i = idx / n, k = idx - i * n;
    R[(int64_t)i * kNmPad + k] = sB[i * kNmPad + k];
  }
  __syncthreads();
  int cur = 0;
  for (int it = 1; it < s; ++it) {
    const int nxt = (cur == 0) ? 2 : 0;
    matmul(a, n, lin1(cur), lin1(cur), none, nxt, sA, sB);
    cur = nxt;
  }
  // F = R_cur (R_cur e_1) if s >= 1, else R e_1
  const double* Rc = slot(a, cur);
  if (s == 0) {
    for (int i = tid; i < n; i += kThreads) F[i] = Rc[(int64_t)i * kNmPad];
  } else {
    double* col = sA;
    for (int i = tid; i < n; i += kThreads) col[i] = Rc[(int64_t)i * kNmPad];
    __syncthreads();
    for (int i = tid; i < n; i += kThreads) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += Rc[(int64_t)i * kNmPad + k] * col[k];
      F[i] = v;
    }
  }
  __syncthreads();
}

}  // namespace kp
