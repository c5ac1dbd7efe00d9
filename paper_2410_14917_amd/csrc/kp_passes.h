// Streaming passes over the augmented vectors (HBM-bound): stage, matvec fused
// with the grouped inner products, basis update fused with the norm, combine
// and finish.  A workgroup processes the element pairs [blockIdx.x*ppw, ...);
// a pass that ends in a reduction writes one partial vector per workgroup to
// a.part (slots of kKStride doubles).
#pragma once

#include "kp_internal.h"

namespace kp {

// ---- basis element access (double or float storage) -----------------------

template <typename TB> struct Pair;
template <> struct Pair<double> {
  __device__ static double2 load(const double* p) {
    return *reinterpret_cast<const double2*>(p);
  }
  __device__ static void store(double* p, double a, double b) {
    *reinterpret_cast<double2*>(p) = make_double2(a, b);
  }
};
template <> struct Pair<float> {
  __device__ static double2 load(const float* p) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    return make_double2((double)v.x, (double)v.y);
  }
  __device__ static void store(float* p, double a, double b) {
    *reinterpret_cast<float2*>(p) = make_float2((float)a, (float)b);
  }
};

template <typename TB> __device__ inline double rnd(double v) { return (double)(TB)v; }

// Element e of the vector the matvec of step jj multiplies: the float64 state
// u at the first step (rounded through the basis type, which is what basis
// column 0 stores), the stored basis column afterwards.
template <typename TB>
struct Src {
  const TB* col;
  const double* u;
  bool from_u;
  __device__ double operator()(int64_t e) const {
    return from_u ? rnd<TB>(u[e]) : (double)col[e];
  }
};

// (A x)_e for an element e < N of the grid operator (no augmented term).
template <typename TB>
__device__ inline double op_apply(const Args& a, const Src<TB>& x, int64_t e) {
  const int nx = a.nx, ny = a.ny;
  const int64_t npt = a.npt;
  int64_t plane = 0, q = e;
  if (a.kind == KP_OP_BRUSSELATOR && e >= npt) {
    plane = npt;
    q = e - npt;
  }
  const int iy = (int)(q / nx);
  const int ix = (int)(q - (int64_t)iy * nx);
  const int64_t qe = (ix == nx - 1) ? q + 1 - nx : q + 1;
  const int64_t qw = (ix == 0) ? q - 1 + nx : q - 1;
  const int64_t qn = (iy == ny - 1) ? q + nx - npt : q + nx;
  const int64_t qs = (iy == 0) ? q - nx + npt : q - nx;
  const double c = x(plane + q);
  const double xe = x(plane + qe), xw = x(plane + qw);
  const double xn = x(plane + qn), xs = x(plane + qs);
  if (a.kind == KP_OP_ADR) {
    const double lap = a.cx * (xe + xw - 2.0 * c) + a.cy * (xn + xs - 2.0 * c);
    const double adv = a.adx * (xe - xw) + a.ady * (xn - xs);
    double v = lap + (a.transpose ? adv : -adv) + a.react * c;
    if (a.f0) v += a.f0[q] * c;
    return v;
  }
  if (a.kind == KP_OP_ALLEN_CAHN) {
    const double lap = a.cx * (xe + xw - 2.0 * c) + a.cy * (xn + xs - 2.0 * c);
    const double U = a.f0[q];
    return lap + (1.0 - 3.0 * U * U) * c;
  }
  // Brusselator Jacobian: pointwise blocks [[a11, a12], [a21, a22]]
  const double U = a.f0[q], W = a.f1[q];
  const double a11 = 2.0 * U * W - (a.bb + 1.0), a12 = U * U;
  const double a21 = a.bb - 2.0 * U * W, a22 = -U * U;
  const bool vplane = plane != 0;
  const double other = x(vplane ? q : npt + q);
  const double cxx = vplane ? a.cx2 : a.cx, cyy = vplane ? a.cy2 : a.cy;
  const double lap = cxx * (xe + xw - 2.0 * c) + cyy * (xn + xs - 2.0 * c);
  if (!a.transpose)
    return vplane ? lap + a21 * other + a22 * c : lap + a11 * c + a12 * other;
  return vplane ? lap + a12 * other + a22 * c : lap + a11 * c + a21 * other;
}

// (Atilde x)_e for any element of the padded augmented vector:
// top block A x_top + sum_c tc[c] b_{p-c} (tc = x_tail / mu), tail K x_tail
// (upward shift), zero in the padding.
template <typename TB>
__device__ inline double aug_apply(const Args& a, const Src<TB>& x, int64_t e,
                                   const double* tc) {
  if (e < a.N) {
    double v = op_apply<TB>(a, x, e);
    for (int c = 0; c < a.p; ++c) v += tc[c] * a.B[(int64_t)(a.p - c) * a.ldb + e];
    return v;
  }
  const int64_t k = e - a.N;
  if (k + 1 < a.p) return x(e + 1);
  return 0.0;
}

// ---- stage: u = [b_0; 0] (the leader adds mu e_p), max |b_k| for k >= 1 -----
// Partial slots: [0] = max |b_k|, [1] = 1 if a non-finite entry was seen.
__device__ inline void stage_pass(const Args& a, double* red) {
  const int64_t beg = (int64_t)blockIdx.x * a.ppw * 2;
  const int64_t end = min(a.ld, beg + a.ppw * 2);
  double mx = 0.0, bad = 0.0;
  for (int64_t e = beg + threadIdx.x; e < end; e += kThreads) {
    double v = 0.0;
    if (e < a.N) {
      v = a.B[e];
      if (!isfinite(v)) bad = 1.0;
      for (int k = 1; k <= a.p; ++k) {
        const double b = a.B[(int64_t)k * a.ldb + e];
        if (!isfinite(b)) bad = 1.0;
        mx = fmax(mx, fabs(b));
      }
    }
    a.u[e] = v;
  }
  mx = block_max(mx, red);
  bad = block_max(bad, red);
  if (threadIdx.x == 0) {
    a.part[(int64_t)blockIdx.x * kKStride + 0] = mx;
    a.part[(int64_t)blockIdx.x * kKStride + 1] = bad;
  }
}

// ---- matvec + grouped inner products (Algorithm 4: matvec and reduction) ----
// Step jj (0-based; x = basis column jj, or u when jj == 0) writes w = Atilde x
// into column jj+1 (and x into column 0 at the first step) and the partial
// inner products of V_{1:j+1}^T [x_j, w] (eq. output_wywnrm):
//   slot 2i = x_i . x,  slot 2i+1 = x_i . w  (i <= jj),  slot 2jj+2 = w . w.
// One pass reads x (with its stencil neighbours), B, the fields and the
// columns 0..jj-1 once, and writes w once.
constexpr int kR = 2;    // element pairs per thread per sub-tile
constexpr int kCh = 8;   // basis columns per chunk

template <typename TB>
__device__ inline void matvec_dots_pass(const Args& a, int jj, double inv_mu,
                                        double* sacc) {
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < kWaves * kKStride; k += kThreads) sacc[k] = 0.0;
  __syncthreads();
  TB* xcol = V + (int64_t)jj * ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const Src<TB> x{xcol, a.u, jj == 0};
  double tc[kPMax];
#pragma unroll
  for (int c = 0; c < kPMax; ++c) tc[c] = (c < a.p) ? x(a.N + c) * inv_mu : 0.0;

  const int64_t pbeg = (int64_t)blockIdx.x * a.ppw;
  const int64_t pend = min(a.npairs, pbeg + a.ppw);
  double sxx = 0.0, sxw = 0.0, sww = 0.0;
  for (int64_t q0 = pbeg; q0 < pend; q0 += (int64_t)kThreads * kR) {
    double2 xv[kR], wv2[kR];
    bool ok[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int64_t q = q0 + (int64_t)r * kThreads + threadIdx.x;
      ok[r] = q < pend;
      xv[r] = make_double2(0.0, 0.0);
      wv2[r] = make_double2(0.0, 0.0);
      if (ok[r]) {
        const int64_t e = 2 * q;
        xv[r] = make_double2(x(e), x(e + 1));
        const double w0 = rnd<TB>(aug_apply<TB>(a, x, e, tc));
        const double w1 = rnd<TB>(aug_apply<TB>(a, x, e + 1, tc));
        wv2[r] = make_double2(w0, w1);
        Pair<TB>::store(wcol + e, w0, w1);
        if (jj == 0) Pair<TB>::store(xcol + e, xv[r].x, xv[r].y);
      }
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      sxx += xv[r].x * xv[r].x + xv[r].y * xv[r].y;
      sxw += xv[r].x * wv2[r].x + xv[r].y * wv2[r].y;
      sww += wv2[r].x * wv2[r].x + wv2[r].y * wv2[r].y;
    }
    for (int i0 = 0; i0 < jj; i0 += kCh) {
      double ax[kCh], aw[kCh];
#pragma unroll
      for (int c = 0; c < kCh; ++c) {
        ax[c] = 0.0;
        aw[c] = 0.0;
      }
#pragma unroll
      for (int c = 0; c < kCh; ++c) {
        if (i0 + c < jj) {
          const TB* vc = V + (int64_t)(i0 + c) * ld;
#pragma unroll
          for (int r = 0; r < kR; ++r) {
            if (ok[r]) {
              const int64_t e = 2 * (q0 + (int64_t)r * kThreads + threadIdx.x);
              const double2 v = Pair<TB>::load(vc + e);
              ax[c] += v.x * xv[r].x + v.y * xv[r].y;
              aw[c] += v.x * wv2[r].x + v.y * wv2[r].y;
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < kCh; ++c) {
        if (i0 + c < jj) {
          const double sx = wave_sum(ax[c]);
          const double sw = wave_sum(aw[c]);
          if (lane == 0) {
            sacc[wv * kKStride + 2 * (i0 + c)] += sx;
            sacc[wv * kKStride + 2 * (i0 + c) + 1] += sw;
          }
        }
      }
    }
  }
  sxx = wave_sum(sxx);
  sxw = wave_sum(sxw);
  sww = wave_sum(sww);
  if (lane == 0) {
    sacc[wv * kKStride + 2 * jj] += sxx;
    sacc[wv * kKStride + 2 * jj + 1] += sxw;
    sacc[wv * kKStride + 2 * jj + 2] += sww;
  }
  __syncthreads();
  const int nslot = 2 * jj + 3;
  for (int k = threadIdx.x; k < nslot; k += kThreads) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += sacc[w * kKStride + k];
    a.part[(int64_t)blockIdx.x * kKStride + k] = s;
  }
}

// ---- basis update + norm (Algorithm 4: projection and normalisation) --------
// x_{j+1} = coef[jj+1] * w + sum_{i<=jj} coef[i] x_i, in place over column jj+1
// (which holds w); partial slot 0 = ||x_{j+1}||^2.  The columns are visited
// from the newest to the oldest, so the ones the matvec pass read last are the
// first to be re-read.
template <typename TB>
__device__ inline void update_pass(const Args& a, int jj, const double* coef,
                                   double* red) {
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const double cw = coef[jj + 1];
  const int64_t pbeg = (int64_t)blockIdx.x * a.ppw;
  const int64_t pend = min(a.npairs, pbeg + a.ppw);
  double ss = 0.0;
  for (int64_t q0 = pbeg; q0 < pend; q0 += (int64_t)kThreads * kR) {
    double2 acc[kR];
    bool ok[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int64_t q = q0 + (int64_t)r * kThreads + threadIdx.x;
      ok[r] = q < pend;
      acc[r] = make_double2(0.0, 0.0);
      if (ok[r]) {
        const double2 w = Pair<TB>::load(wcol + 2 * q);
        acc[r] = make_double2(cw * w.x, cw * w.y);
      }
    }
    for (int i1 = jj; i1 >= 0; i1 -= kCh) {
#pragma unroll
      for (int c = 0; c < kCh; ++c) {
        const int i = i1 - c;
        if (i >= 0) {
          const TB* vc = V + (int64_t)i * ld;
          const double ci = coef[i];
#pragma unroll
          for (int r = 0; r < kR; ++r) {
            if (ok[r]) {
              const double2 v = Pair<TB>::load(vc + 2 * (q0 + (int64_t)r * kThreads + threadIdx.x));
              acc[r].x += ci * v.x;
              acc[r].y += ci * v.y;
            }
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      if (ok[r]) {
        const int64_t e = 2 * (q0 + (int64_t)r * kThreads + threadIdx.x);
        const double y0 = rnd<TB>(acc[r].x), y1 = rnd<TB>(acc[r].y);
        Pair<TB>::store(wcol + e, y0, y1);
        ss += y0 * y0 + y1 * y1;
      }
    }
  }
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) a.part[(int64_t)blockIdx.x * kKStride] = ss;
}

// ---- combine: u = sum_{i<m} coef[i] x_i  (= beta V_m F, eq. kryexp) ----------
// Also writes out = u_top when this is the last substep.
template <typename TB>
__device__ inline void combine_pass(const Args& a, int m, const double* coef,
                                    bool last) {
  const TB* V = reinterpret_cast<const TB*>(a.V);
  const int64_t ld = a.ld;
  const int64_t pbeg = (int64_t)blockIdx.x * a.ppw;
  const int64_t pend = min(a.npairs, pbeg + a.ppw);
  for (int64_t q0 = pbeg; q0 < pend; q0 += (int64_t)kThreads * kR) {
    double2 acc[kR];
    bool ok[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      ok[r] = (q0 + (int64_t)r * kThreads + threadIdx.x) < pend;
      acc[r] = make_double2(0.0, 0.0);
    }
    for (int i0 = 0; i0 < m; i0 += kCh) {
#pragma unroll
      for (int c = 0; c < kCh; ++c) {
        const int i = i0 + c;
        if (i < m) {
          const TB* vc = V + (int64_t)i * ld;
          const double ci = coef[i];
#pragma unroll
          for (int r = 0; r < kR; ++r) {
            if (ok[r]) {
              const double2 v = Pair<TB>::load(vc + 2 * (q0 + (int64_t)r * kThreads + threadIdx.x));
              acc[r].x += ci * v.x;
              acc[r].y += ci * v.y;
            }
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      if (ok[r]) {
        const int64_t e = 2 * (q0 + (int64_t)r * kThreads + threadIdx.x);
        *reinterpret_cast<double2*>(a.u + e) = acc[r];
        if (last) {
          if (e < a.N) a.out[e] = acc[r].x;
          if (e + 1 < a.N) a.out[e + 1] = acc[r].y;
        }
      }
    }
  }
}

// ---- finish: out = u_top (or NaN when the input was not finite) -------------
__device__ inline void finish_pass(const Args& a, bool nonfinite) {
  const int64_t beg = (int64_t)blockIdx.x * a.ppw * 2;
  const int64_t end = min((int64_t)a.N, beg + a.ppw * 2);
  for (int64_t e = beg + threadIdx.x; e < end; e += kThreads)
    a.out[e] = nonfinite ? __builtin_nan("") : a.u[e];
}

}  // namespace kp
