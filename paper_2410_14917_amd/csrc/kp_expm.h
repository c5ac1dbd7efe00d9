// Small Hessenberg exponential F = exp(tau Hbar) e_1 in one workgroup, float64.
//
// Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]] is n x n with n = m + 1 <= 65; the
// last entry of F is the error estimate of the Krylov projection (eq. kryexp).
// The method is the degree-19 Taylor polynomial with scaling and squaring:
// X = tau Hbar / 2^s with ||X||_1 <= theta_19, T_19(X) evaluated by the
// Paterson-Stockmeyer scheme in powers of X^4 (X^2, X^3, X^4, then four
// Horner steps T <- X^4 T + C_i with C_i = sum_{r<4} X^r / (4i + r)!: seven
// products and no linear solve), then s squarings.  theta_19 = 1.26038 is the
// largest 1-norm for which the backward-error bound of the truncated series
// (Al-Mohy and Higham, SIAM J. Matrix Anal. Appl. 31 (2009), Section 3:
// sum_{k>19} |c_k| theta^{k-1} <= 2^-53 for the coefficients c_k of
// log(e^{-x} T_19(x))) holds; the value was computed with exact rational
// series arithmetic.  Only the first column is returned, so the last squaring
// is a matrix-vector product.
//
// Layout: the operands of every product live in LDS (two 68 x 68 row-major
// tiles, zero outside the n x n matrix).  A product is computed with the
// float64 matrix cores (v_mfma_f64_16x16x4f64): the <= 5 x 5 output tiles of
// 16 x 16 are spread over the 8 waves and kept in registers until a barrier,
// after which every output element is written by the one lane that holds it
// (with the linear combinations the Horner steps need), so a product may
// overwrite its own operands.  X, X^2 and X^3, which the combinations C_i
// read, are kept in a small global scratch (L2-resident).
#pragma once

#include "kp_internal.h"

namespace kp {

constexpr double kTheta19 = 1.2603810606426387;

// Taylor coefficients 1/k!, k <= 19.
struct Taylor19 {
  double c[20];
  constexpr Taylor19() : c() {
    c[0] = 1.0;
    for (int k = 1; k <= 19; ++k) c[k] = c[k - 1] / (double)k;
  }
};
constexpr Taylor19 kTaylor{};

__device__ inline double* slot(const Args& a, int s) {
  return a.ex + (int64_t)s * kNmPad * kNmPad;
}

// The output tiles of C = A B (A, B: LDS tiles, stride kNmPad, n <= 65)
// held by this lane: tile t = wave + 8 s (s < kTilesPerWave) of the
// ceil(n/16)^2 tiles of 16 x 16.  Operands of v_mfma_f64_16x16x4f64: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] of the 16 x 4 and 4 x 16
// slices; element v of its accumulator is C[l / 16 + 4 v][l % 16] (checked on
// the device against a host product).
constexpr int kTilesPerWave = 4;
typedef double kp_d4 __attribute__((ext_vector_type(4)));

struct Tiles {
  int nt;                       // tiles per side
  kp_d4 c[kTilesPerWave];
};

__device__ inline void mm_tiles(int n, const double* A, const double* B, Tiles& T) {
  const int lane = kp_tid() & 63, wv = kp_tid() >> 6;
  T.nt = (n + 15) >> 4;
  const int ntile = T.nt * T.nt;
  const int lr = lane & 15, lk = lane >> 4;
  int arow[kTilesPerWave], bcol[kTilesPerWave];
#pragma unroll
  for (int s = 0; s < kTilesPerWave; ++s) {
    T.c[s] = (kp_d4){0.0, 0.0, 0.0, 0.0};
    // tiles past the last one compute on a valid clamped tile and are never
    // written (tiles_for_each skips them), so the four chains run unbranched
    const int t = min(wv + kWaves * s, ntile - 1);
    const int ti = t / T.nt, tj = t - ti * T.nt;
    arow[s] = min(16 * ti + lr, kNmPad - 1);    // A operand: A[row][k]
    bcol[s] = min(16 * tj + lr, kNmPad - 1);    // B operand: B[k][col]
  }
  // the four accumulation chains are interleaved; the operands of step k0 + 4
  // are loaded while step k0 multiplies; entries past n enter as zeros
  double av[kTilesPerWave], bv[kTilesPerWave];
#pragma unroll
  for (int s = 0; s < kTilesPerWave; ++s) {
    const double ta = A[arow[s] * kNmPad + lk], tb = B[lk * kNmPad + bcol[s]];
    av[s] = (lk < n) ? ta : 0.0;
    bv[s] = (lk < n) ? tb : 0.0;
  }
  for (int k0 = 0; k0 < n; k0 += 4) {
    const int k = k0 + 4 + lk;
    const int kc = min(k, kNmPad - 1);
    double an[kTilesPerWave], bn[kTilesPerWave];
#pragma unroll
    for (int s = 0; s < kTilesPerWave; ++s) {
      an[s] = A[arow[s] * kNmPad + kc];
      bn[s] = B[kc * kNmPad + bcol[s]];
    }
#pragma unroll
    for (int s = 0; s < kTilesPerWave; ++s)
      T.c[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], T.c[s], 0, 0, 0);
#pragma unroll
    for (int s = 0; s < kTilesPerWave; ++s) {
      av[s] = (k < n) ? an[s] : 0.0;
      bv[s] = (k < n) ? bn[s] : 0.0;
    }
  }
}

// Calls f(i, k, value) for every element of C = A B inside the n x n matrix
// that this lane holds.
template <typename F>
__device__ inline void tiles_for_each(int n, const Tiles& T, F f) {
  const int lane = kp_tid() & 63, wv = kp_tid() >> 6;
  const int ntile = T.nt * T.nt;
#pragma unroll
  for (int s = 0; s < kTilesPerWave; ++s) {
    const int t = wv + kWaves * s;
    if (t >= ntile) continue;
    const int ti = t / T.nt, tj = t - ti * T.nt;
    const int k = 16 * tj + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ti + (lane >> 4) + 4 * v;
      if (i < n && k < n) f(i, k, T.c[s][v]);
    }
  }
}

// F[0..m] = exp(tau Hbar) e_1 for the Hessenberg H (column-major, leading
// dimension ldh) of size (m+1) x m; zero_sub drops h_{m+1,m} (lucky
// breakdown).  Whole workgroup; lds holds at least 2 kNmPad^2 doubles.
__device__ inline void expm_hbar(const Args& a, const double* H, int ldh, int m,
                                 double tau, bool zero_sub, double* F, double* lds) {
  __shared__ double s_red[kWaves];
  __shared__ int s_s;
  double* sA = lds;
  double* sB = lds + kNmPad * kNmPad;
  const int n = m + 1;
  const int tid = kp_tid();
  const double* c = kTaylor.c;
  // X = tau * Hbar into sA (zero outside n x n); sB zeroed; 1-norm of X
  for (int idx = tid; idx < kNmPad * kNmPad; idx += kThreads) {
    const int i = idx / kNmPad, k = idx - i * kNmPad;
    double v = 0.0;
    if (k < m && i <= k + 1 && i < n) {
      v = H[(int64_t)k * ldh + i];
      if (zero_sub && k == m - 1 && i == m) v = 0.0;
    }
    sA[idx] = tau * v;
    sB[idx] = 0.0;
  }
  __syncthreads();
  double cmax = 0.0;
  for (int k = tid; k < n; k += kThreads) {
    double cs = 0.0;
    for (int i = 0; i < n; ++i) cs += fabs(sA[i * kNmPad + k]);
    cmax = fmax(cmax, cs);
  }
  cmax = block_max(cmax, s_red);
  if (tid == 0) {
    int s = 0;
    if (isfinite(cmax) && cmax > kTheta19) {
      int e;
      const double r = frexp(cmax / kTheta19, &e);   // cmax/theta = r 2^e, r in [0.5,1)
      s = (r == 0.5) ? e - 1 : e;                    // smallest s: ratio <= 2^s
    }
    s_s = s;
  }
  __syncthreads();
  const int s = s_s;
  const double sc = ldexp(1.0, -s);
  double* gX = slot(a, 0);
  double* gX2 = slot(a, 1);
  double* gX3 = slot(a, 2);
  for (int idx = tid; idx < kNmPad * kNmPad; idx += kThreads) {
    const double v = sA[idx] * sc;
    sA[idx] = v;
    gX[idx] = v;
  }
  __syncthreads();
  Tiles T;
  // X2 = X X -> sB and scratch
  mm_tiles(n, sA, sA, T);
  __syncthreads();
  tiles_for_each(n, T, [&](int i, int k, double v) {
    sB[i * kNmPad + k] = v;
    gX2[i * kNmPad + k] = v;
  });
  __syncthreads();
  // X3 = X2 X -> scratch
  mm_tiles(n, sB, sA, T);
  __syncthreads();
  tiles_for_each(n, T, [&](int i, int k, double v) { gX3[i * kNmPad + k] = v; });
  __syncthreads();
  // X4 = X2 X2 -> sA; sB <- C_4 = I/16! + X/17! + X^2/18! + X^3/19!
  mm_tiles(n, sB, sB, T);
  __syncthreads();
  tiles_for_each(n, T, [&](int i, int k, double v) {
    const int o = i * kNmPad + k;
    sA[o] = v;
    sB[o] = ((i == k) ? c[16] : 0.0) + c[17] * gX[o] + c[18] * gX2[o] + c[19] * gX3[o];
  });
  __syncthreads();
  // Horner in X^4: T <- X^4 T + C_i, i = 3, 2, 1, 0 (T in sB)
  for (int i4 = 12; i4 >= 0; i4 -= 4) {
    mm_tiles(n, sA, sB, T);
    __syncthreads();
    tiles_for_each(n, T, [&](int i, int k, double v) {
      const int o = i * kNmPad + k;
      sB[o] = v + (((i == k) ? c[i4] : 0.0) + c[i4 + 1] * gX[o] + c[i4 + 2] * gX2[o] +
                   c[i4 + 3] * gX3[o]);
    });
    __syncthreads();
  }
  // s - 1 squarings in place in sB
  for (int it = 1; it < s; ++it) {
    mm_tiles(n, sB, sB, T);
    __syncthreads();
    tiles_for_each(n, T, [&](int i, int k, double v) { sB[i * kNmPad + k] = v; });
    __syncthreads();
  }
  // F = R (R e_1) if s >= 1, else R e_1 (R = sB)
  if (s == 0) {
    for (int i = tid; i < n; i += kThreads) F[i] = sB[i * kNmPad];
  } else {
    double* col = sA;
    for (int i = tid; i < n; i += kThreads) col[i] = sB[i * kNmPad];
    __syncthreads();
    for (int i = tid; i < n; i += kThreads) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += sB[i * kNmPad + k] * col[k];
      F[i] = v;
    }
  }
  __syncthreads();
}

}  // namespace kp
