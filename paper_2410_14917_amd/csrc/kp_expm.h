// Small Hessenberg exponential F = exp(tau Hbar) e_1 in one workgroup, float64.
//
// Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]] is n x n with n = m + 1 <= 65; the
// last entry of F is the error estimate of the Krylov projection (eq. kryexp).
// The method is the [13/13] Pade approximant with scaling and squaring
// (Higham, "The scaling and squaring method for the matrix exponential
// revisited", SIAM J. Matrix Anal. Appl. 26 (2005)): X = tau Hbar / 2^s with
// ||X||_1 <= theta_13, r(X) = q(X)^{-1} p(X) with p(X) = U + V and
// q(X) = V - U split into odd and even powers, then s squarings.  Only the
// first column is returned, so the last squaring is a matrix-vector product.
//
// Layout: the operands of every product live in LDS (two 68 x 68 row-major
// tiles, zero outside the n x n matrix).  A product is computed with the
// float64 matrix cores (v_mfma_f64_16x16x4f64): the <= 5 x 5 output tiles of
// 16 x 16 are spread over the 8 waves and kept in registers until a barrier,
// after which every output element is written by the one lane that holds it
// (with the linear combinations the Pade evaluation needs), so a product may
// overwrite its own operands.  Intermediate powers go to a small global
// scratch (L2-resident) only where the two LDS tiles do not suffice.  The
// linear system q(X) R = p(X) is solved by Gauss-Jordan elimination with
// partial pivoting on the n x 2n matrix [q | p]: every thread keeps its
// elements in registers for the whole elimination, and each step exchanges
// only the pivot column and the pivot row through LDS (two barriers per
// step, the pivot search done redundantly by every wave with DPP
// reductions, no row swaps).
#pragma once

#include "kp_internal.h"

namespace kp {

constexpr double kTheta13 = 5.371920351148152;   // Higham (2005), Table 2.3

// Pade [13/13] numerator coefficients normalised to b_0 = 1:
// b_k = b_{k-1} (13 - k + 1) / (k (26 - k + 1)).
struct Pade13 {
  double b[14];
  constexpr Pade13() : b() {
    b[0] = 1.0;
    for (int k = 1; k <= 13; ++k) b[k] = b[k - 1] * (double)(14 - k) / ((double)k * (double)(27 - k));
  }
};
constexpr Pade13 kPade{};

constexpr int kGjLd = 131;   // row stride of the Gauss-Jordan matrix [q | p]

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

// Largest 64-bit unsigned key over the wave (every lane gets it): DPP within
// rows of 16 lanes, then the four row results through readlane.
template <int CTRL>
__device__ inline uint64_t dpp_u64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ inline uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ inline uint64_t wave_max_u64(uint64_t v) {
  v = umax64(v, dpp_u64<0xB1>(v));    // quad_perm [1,0,3,2]
  v = umax64(v, dpp_u64<0x4E>(v));    // quad_perm [2,3,0,1]
  v = umax64(v, dpp_u64<0x141>(v));   // row_half_mirror
  v = umax64(v, dpp_u64<0x140>(v));   // row_mirror
  uint64_t m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, 16 * r);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 16 * r);
    m = umax64(m, ((uint64_t)hi << 32) | lo);
  }
  return m;
}

// Pivot key of row r: |v| with its 7 low mantissa bits replaced by 127 - r
// (ties and near-ties go to the smaller row index; every row still available
// has a key >= 63, rows already used and rows past n have key 0).
__device__ inline uint64_t pivot_key(double v, int n, int r, uint64_t used_lo, bool used64) {
  const bool used = (r < 64) ? (((used_lo >> (r & 63)) & 1u) != 0) : used64;
  const uint64_t bits = (uint64_t)__double_as_longlong(fabs(v));
  const uint64_t key = (bits & ~(uint64_t)127) | (uint64_t)(127 - r);
  return (r < n && !used) ? key : 0;
}

constexpr int kGjRows = (kNmPad + 3) / 4;   // rows of [q | p] per thread

struct GjShared {
  double col[2][kNmPad];     // pivot column of the step (double-buffered)
  double row[2][2 * kNmPad]; // pivot row of the step (double-buffered)
  double pv[kNmPad];         // pivot value of step k
  int stepof[kNmPad];        // step at which row r was the pivot row
};

// Solve q R = p for the n x n matrices held as G = [q | p] (LDS, stride
// kGjLd) by Gauss-Jordan elimination with partial pivoting.  Thread
// (rg, cl) = (tid / 128, tid % 128) holds rows rg + 4 s of columns cl and
// cl + 128 in registers.  R is written to R (LDS, stride kNmPad, zero outside
// n x n); R may alias G.
__device__ inline void gauss_jordan(int n, const double* G, GjShared& sh, double* R) {
  const int t = kp_tid(), lane = t & 63;
  const int rg = t >> 7, cl = t & 127;
  const int cA = cl, cB = cl + 128;
  const bool hasA = cA < 2 * n, hasB = cB < 2 * n;
  double gA[kGjRows], gB[kGjRows];
#pragma unroll
  for (int s = 0; s < kGjRows; ++s) {
    const int r = rg + 4 * s;
    gA[s] = (r < n && hasA) ? G[r * kGjLd + cA] : 0.0;
    gB[s] = (r < n && hasB) ? G[r * kGjLd + cB] : 0.0;
  }
  __syncthreads();
  uint64_t used_lo = 0;
  bool used64 = false;
  for (int k = 0; k < n; ++k) {
    const int par = k & 1;
    if (cA == k) {                                   // the owners of column k publish it
#pragma unroll
      for (int s = 0; s < kGjRows; ++s) sh.col[par][rg + 4 * s] = gA[s];
    }
    __syncthreads();
    const double c0 = sh.col[par][lane];
    const double c1 = sh.col[par][min(lane + 64, kNmPad - 1)];
    const uint64_t key = umax64(pivot_key(c0, n, lane, used_lo, used64),
                                pivot_key(c1, n, lane + 64, used_lo, used64));
    const int P = 127 - (int)(wave_max_u64(key) & 127u);
    if (P < 64) used_lo |= (uint64_t)1 << P; else used64 = true;
    const double pval = sh.col[par][P];
    if (rg == (P & 3)) {                             // the owners of row P publish it
      const int sP = P >> 2;
      double vA = 0.0, vB = 0.0;
#pragma unroll
      for (int s = 0; s < kGjRows; ++s)
        if (s == sP) {
          vA = gA[s];
          vB = gB[s];
        }
      if (hasA) sh.row[par][cA] = vA;
      if (hasB) sh.row[par][cB] = vB;
    }
    if (t == 0) {
      sh.pv[k] = pval;
      sh.stepof[P] = k;
    }
    __syncthreads();
    const double inv = 1.0 / pval;
    const double pA = (hasA && cA > k) ? sh.row[par][cA] : 0.0;
    const double pB = hasB ? sh.row[par][cB] : 0.0;
    double cv[kGjRows];
#pragma unroll
    for (int s = 0; s < kGjRows; ++s) cv[s] = sh.col[par][rg + 4 * s];   // all loads first
#pragma unroll
    for (int s = 0; s < kGjRows; ++s) {
      const int r = rg + 4 * s;
      const double f = (r < n && r != P) ? cv[s] * inv : 0.0;
      gA[s] -= f * pA;
      gB[s] -= f * pB;
    }
  }
  __syncthreads();
  for (int idx = t; idx < kNmPad * kNmPad; idx += kThreads) R[idx] = 0.0;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kGjRows; ++s) {
    const int r = rg + 4 * s;
    if (r >= n) continue;
    const int i = sh.stepof[r];
    const double d = sh.pv[i];
    if (hasA && cA >= n) R[i * kNmPad + cA - n] = gA[s] / d;
    if (hasB && cB >= n) R[i * kNmPad + cB - n] = gB[s] / d;
  }
  __syncthreads();
}

// F[0..m] = exp(tau Hbar) e_1 for the Hessenberg H (column-major, leading
// dimension ldh) of size (m+1) x m; zero_sub drops h_{m+1,m} (lucky
// breakdown).  Whole workgroup; lds holds at least kNmPad * kGjLd doubles.
__device__ inline void expm_hbar(const Args& a, const double* H, int ldh, int m,
                                 double tau, bool zero_sub, double* F, double* lds) {
  __shared__ double s_red[kWaves];
  __shared__ int s_s;
  __shared__ GjShared gj;
  double* sA = lds;
  double* sB = lds + kNmPad * kNmPad;
  double* G = lds;
  const int n = m + 1;
  const int tid = kp_tid();
  const double* b = kPade.b;
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
    if (isfinite(cmax) && cmax > kTheta13) {
      int e;
      const double r = frexp(cmax / kTheta13, &e);   // cmax/theta = r 2^e, r in [0.5,1)
      s = (r == 0.5) ? e - 1 : e;                    // smallest s: ratio <= 2^s
    }
    s_s = s;
  }
  __syncthreads();
  const int s = s_s;
  const double sc = ldexp(1.0, -s);
  double* gX = slot(a, 0);
  for (int idx = tid; idx < kNmPad * kNmPad; idx += kThreads) {
    const double v = sA[idx] * sc;
    sA[idx] = v;
    gX[idx] = v;
  }
  __syncthreads();
  Tiles T;
  // X2 = X X -> sB
  mm_tiles(n, sA, sA, T);
  __syncthreads();
  tiles_for_each(n, T, [&](int i, int k, double v) { sB[i * kNmPad + k] = v; });
  __syncthreads();
  // X4 = X2 X2 -> sA (X stays in slot 0)
  mm_tiles(n, sB, sB, T);
  __syncthreads();
  tiles_for_each(n, T, [&](int i, int k, double v) { sA[i * kNmPad + k] = v; });
  __syncthreads();
  // X6 = X4 X2; then, elementwise: sA <- X6, sB <- L1 = b12 X6 + b10 X4 + b8 X2,
  // slot 1 <- L2 = b13 X6 + b11 X4 + b9 X2, slot 2 <- DV = b6 X6 + b4 X4 + b2 X2 + b0 I,
  // slot 3 <- DW = b7 X6 + b5 X4 + b3 X2 + b1 I
  mm_tiles(n, sA, sB, T);
  __syncthreads();
  {
    double* gL2 = slot(a, 1);
    double* gDV = slot(a, 2);
    double* gDW = slot(a, 3);
    tiles_for_each(n, T, [&](int i, int k, double x6) {
      const int o = i * kNmPad + k;
      const double x4 = sA[o], x2 = sB[o];
      const double eye = (i == k) ? 1.0 : 0.0;
      sA[o] = x6;
      sB[o] = b[12] * x6 + b[10] * x4 + b[8] * x2;
      gL2[o] = b[13] * x6 + b[11] * x4 + b[9] * x2;
      gDV[o] = b[6] * x6 + b[4] * x4 + b[2] * x2 + b[0] * eye;
      gDW[o] = b[7] * x6 + b[5] * x4 + b[3] * x2 + b[1] * eye;
    });
  }
  __syncthreads();
  // V = X6 L1 + DV -> slot 4; sB <- L2
  mm_tiles(n, sA, sB, T);
  __syncthreads();
  {
    const double* gL2 = slot(a, 1);
    const double* gDV = slot(a, 2);
    double* gV = slot(a, 4);
    tiles_for_each(n, T, [&](int i, int k, double v) {
      const int o = i * kNmPad + k;
      gV[o] = v + gDV[o];
      sB[o] = gL2[o];
    });
  }
  __syncthreads();
  // W = X6 L2 + DW -> sB; sA <- X
  mm_tiles(n, sA, sB, T);
  __syncthreads();
  {
    const double* gDW = slot(a, 3);
    tiles_for_each(n, T, [&](int i, int k, double v) {
      const int o = i * kNmPad + k;
      sB[o] = v + gDW[o];
      sA[o] = gX[o];
    });
  }
  __syncthreads();
  // U = X W; G = [V - U | V + U]
  mm_tiles(n, sA, sB, T);
  __syncthreads();
  {
    const double* gV = slot(a, 4);
    tiles_for_each(n, T, [&](int i, int k, double u) {
      const double v = gV[i * kNmPad + k];
      G[i * kGjLd + k] = v - u;
      G[i * kGjLd + n + k] = v + u;
    });
  }
  __syncthreads();
  // R = q^{-1} p -> sA (zero-padded)
  gauss_jordan(n, G, gj, sA);
  // s - 1 squarings in place in sA
  for (int it = 1; it < s; ++it) {
    mm_tiles(n, sA, sA, T);
    __syncthreads();
    tiles_for_each(n, T, [&](int i, int k, double v) { sA[i * kNmPad + k] = v; });
    __syncthreads();
  }
  // F = R (R e_1) if s >= 1, else R e_1
  if (s == 0) {
    for (int i = tid; i < n; i += kThreads) F[i] = sA[i * kNmPad];
  } else {
    double* col = sB;
    for (int i = tid; i < n; i += kThreads) col[i] = sA[i * kNmPad];
    __syncthreads();
    for (int i = tid; i < n; i += kThreads) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += sA[i * kNmPad + k] * col[k];
      F[i] = v;
    }
  }
  __syncthreads();
}

}  // namespace kp
