// Streaming passes over the augmented vectors (HBM-bound): stage, matvec fused
// with the grouped inner products, basis update fused with the norm, combine
// and finish.
//
// Workgroup b owns grid rows [r0, r1) = [b*rows_per_wg, ...) of every species
// plane, i.e. the internal elements [s*npt_pad + r0*nx, s*npt_pad + r1*nx) for
// each plane s ("segments"); workgroup 0 also owns the augmented tail region.
// Elements are processed in pairs (16-byte accesses); segment starts are even
// by construction, and an odd segment end leaves one padding element (kept
// zero) in the last pair.
//
// Every pass walks a segment in sub-tiles of kThreads * kR pairs.  Lanes whose
// pair lies past the segment end load the segment's last pair instead (always
// in bounds) and neither store nor contribute to a sum, so no load sits behind
// a divergent branch and all loads of a column chunk are in flight together.
//
// Producers of a vector that the next matvec multiplies publish the first and
// last row of their range (halo) and the tail with coherent stores.
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

// Vector multiplied by the matvec of step jj: the float64 state u at the first
// step (rounded through the basis type, which is what basis column 0 stores),
// the stored basis column afterwards.  Own elements only (plain loads).
template <typename TB>
struct Src {
  const TB* col;
  const double* u;
  bool from_u;
  __device__ double operator()(int64_t e) const {
    return from_u ? rnd<TB>(u[e]) : (double)col[e];
  }
  __device__ double2 pair(int64_t e) const {
    if (from_u) {
      const double2 v = *reinterpret_cast<const double2*>(u + e);
      return make_double2(rnd<TB>(v.x), rnd<TB>(v.y));
    }
    return Pair<TB>::load(col + e);
  }
};

// ---- ownership --------------------------------------------------------------

struct Rows {
  int r0, r1;
};

__device__ inline Rows own_rows(const Args& a) {
  Rows o;
  o.r0 = (int)blockIdx.x * a.rows_per_wg;
  o.r1 = min(a.ny, o.r0 + a.rows_per_wg);
  return o;
}

// One owned segment: elements [beg, end) of plane `plane`, or the tail.
struct Seg {
  int64_t beg, end;
  int plane;
  bool tail;
};

__device__ inline int num_segs(const Args& a) { return a.nplanes + (blockIdx.x == 0 ? 1 : 0); }

__device__ inline Seg seg_at(const Args& a, const Rows& o, int si) {
  if (si < a.nplanes) {
    const int64_t base = (int64_t)si * a.npt_pad;
    return Seg{base + (int64_t)o.r0 * a.nx, base + (int64_t)o.r1 * a.nx, si, false};
  }
  return Seg{a.tail_off, a.tail_off + kTailPad, 0, true};
}

constexpr int kR = 4;    // element pairs per thread per sub-tile
constexpr int kCh = 4;   // basis columns per chunk of the inner-product loop
constexpr int kCu = 8;   // basis columns per chunk of the linear combinations

// Pair indices of this lane in the sub-tile starting at pair q0; pairs past
// pend are clamped to the last pair (ok = false).
__device__ inline void tile_pairs(int64_t q0, int64_t pend, int64_t* qc, bool* ok) {
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int64_t q = q0 + (int64_t)r * kThreads + threadIdx.x;
    ok[r] = q < pend;
    qc[r] = ok[r] ? q : pend - 1;
  }
}

// acc[r] += sum over the C columns i = i0, i0 + step, ... of coef[i] V_i(pair qc[r]).
// All C * kR loads are issued before the first multiply-add.
template <typename TB, int C>
__device__ inline void axpy_cols(const TB* V, int64_t ld, int i0, int step, const double* coef,
                                 const int64_t* qc, double2* acc) {
  double2 v[C][kR];
  double ci[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const TB* vc = V + (int64_t)(i0 + c * step) * ld;
    ci[c] = coef[i0 + c * step];
#pragma unroll
    for (int r = 0; r < kR; ++r) v[c][r] = Pair<TB>::load(vc + 2 * qc[r]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      acc[r].x += ci[c] * v[c][r].x;
      acc[r].y += ci[c] * v[c][r].y;
    }
}

// Index of the halo slot of (workgroup w, plane s, side: 0 first row, 1 last row).
__device__ inline int64_t halo_at(const Args& a, int w, int s, int side, int ix) {
  return ((int64_t)(w * a.nplanes + s) * 2 + side) * a.nx + ix;
}

// After a pass produced vector x (own elements, plain stores), publish the
// first and last row of the owned range of every plane (stencil halo of the
// neighbouring workgroups) and, for workgroup 0, the augmented tail, with
// coherent stores.  Reads back this workgroup's own fresh data.
template <typename T>
__device__ inline void publish_halo(const Args& a, const Rows& o, const T* x) {
  __syncthreads();
  const int nx = a.nx;
  for (int s = 0; s < a.nplanes; ++s) {
    const int64_t base = (int64_t)s * a.npt_pad;
    for (int ix = threadIdx.x; ix < nx; ix += kThreads) {
      cstore(a.hx + halo_at(a, blockIdx.x, s, 0, ix), (double)x[base + (int64_t)o.r0 * nx + ix]);
      cstore(a.hx + halo_at(a, blockIdx.x, s, 1, ix),
             (double)x[base + (int64_t)(o.r1 - 1) * nx + ix]);
    }
  }
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < kTailPad; k += kThreads) cstore(a.tx + k, (double)x[a.tail_off + k]);
}

// Copy the halo rows this workgroup's stencil needs (the first row of the next
// workgroup, the last row of the previous one, periodic) into LDS:
// hl[s * nx + ix] = row r1 (mod ny), hl[(nplanes + s) * nx + ix] = row r0 - 1.
template <typename TB>
__device__ inline void stage_halo(const Args& a, const Rows& o, double* hl) {
  const int nx = a.nx, b = (int)blockIdx.x;
  const int wn = (o.r1 == a.ny) ? 0 : b + 1;
  const int ws = (o.r0 == 0) ? a.nwg - 1 : b - 1;
  for (int s = 0; s < a.nplanes; ++s)
    for (int ix = threadIdx.x; ix < nx; ix += kThreads) {
      hl[s * nx + ix] = rnd<TB>(cload(a.hx + halo_at(a, wn, s, 0, ix)));
      hl[(a.nplanes + s) * nx + ix] = rnd<TB>(cload(a.hx + halo_at(a, ws, s, 1, ix)));
    }
}

// ---- the operator on one grid element ---------------------------------------
//
// (A x)_e for grid element e (internal index) of plane s, whose in-plane index
// is q (row, ix).  Neighbours inside the owned rows are read from x; the rows
// just outside come from the LDS halo copy (HL) or from the coherent halo
// slots.  All loads are unconditional (dummy indices where unused).
template <typename TB, bool HL>
__device__ inline double op_elem(const Args& a, const Rows& o, const Src<TB>& x, const double* hl,
                                 int s, int64_t e, int q, bool valid) {
  const int nx = a.nx;
  int row = (int)((double)q * a.inv_nx);   // q / nx, corrected by one step
  row -= ((unsigned)row * (unsigned)nx > (unsigned)q) ? 1 : 0;
  row += ((unsigned)(row + 1) * (unsigned)nx <= (unsigned)q) ? 1 : 0;
  const int ix = q - row * nx;
  const bool hn = row + 1 < o.r1, hs = row > o.r0;
  const int64_t ie = (ix == nx - 1) ? e - ix : e + 1;
  const int64_t iw = (ix == 0) ? e + nx - 1 : e - 1;
  const int64_t in = (hn && valid) ? e + nx : e;
  const int64_t is = (hs && valid) ? e - nx : e;
  const int64_t io = (a.nplanes == 2) ? (s ? e - a.npt_pad : e + a.npt_pad) : e;
  const double c = x(e);
  const double xe = x(valid ? ie : e);
  const double xw = x(valid ? iw : e);
  double xn = x(in);
  double xs = x(is);
  const double xo = x(io);
  const int qf = valid ? q : 0;
  const double U = a.f0 ? a.f0[qf] : 0.0;
  const double W = a.f1 ? a.f1[qf] : 0.0;
  if (HL) {
    const double hnv = hl[s * nx + ix];
    const double hsv = hl[(a.nplanes + s) * nx + ix];
    xn = hn ? xn : hnv;
    xs = hs ? xs : hsv;
  } else {
    if (!hn) {
      const int rn = (row + 1 == a.ny) ? 0 : row + 1;
      xn = rnd<TB>(cload(a.hx + halo_at(a, (int)((unsigned)rn / (unsigned)a.rows_per_wg), s, 0, ix)));
    }
    if (!hs) {
      const int rs = (row == 0) ? a.ny - 1 : row - 1;
      xs = rnd<TB>(cload(a.hx + halo_at(a, (int)((unsigned)rs / (unsigned)a.rows_per_wg), s, 1, ix)));
    }
  }
  const double cxx = s ? a.cx2 : a.cx, cyy = s ? a.cy2 : a.cy;
  const double lap = cxx * (xe + xw - 2.0 * c) + cyy * (xn + xs - 2.0 * c);
  if (a.kind == KP_OP_ADR) {
    const double adv = a.adx * (xe - xw) + a.ady * (xn - xs);
    return lap + (a.transpose ? adv : -adv) + (a.react + U) * c;
  }
  if (a.kind == KP_OP_ALLEN_CAHN) return lap + (1.0 - 3.0 * U * U) * c;
  // Brusselator Jacobian: pointwise blocks [[a11, a12], [a21, a22]]; the other
  // species at the same point (xo) is owned by this workgroup too.
  const double a11 = 2.0 * U * W - (a.bb + 1.0), a12 = U * U;
  const double a21 = a.bb - 2.0 * U * W, a22 = -U * U;
  if (!a.transpose) return s ? lap + a21 * xo + a22 * c : lap + a11 * c + a12 * xo;
  return s ? lap + a12 * xo + a22 * c : lap + a11 * c + a21 * xo;
}

// (Atilde x) on the kR pairs of a sub-tile of segment sg.  Grid part:
// A x_top + sum_c tc[c] b_{p-c}; tail part: K x_tail (upward shift); zero in
// the padding.
template <typename TB, bool HL>
__device__ inline void aug_tile(const Args& a, const Rows& o, const Seg& sg, const Src<TB>& x,
                                const double* hl, const int64_t* qc, const double* tc,
                                double2* w) {
  if (sg.tail) {
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int64_t e = 2 * qc[r];
      const int64_t k = e - a.tail_off;
      const double2 nx2 = x.pair(e + 2 < sg.end ? e + 2 : e);
      const double v1 = x(e + 1);
      w[r].x = (k + 1 < a.p) ? v1 : 0.0;
      w[r].y = (k + 2 < a.p) ? nx2.x : 0.0;
    }
    return;
  }
  const int64_t base = (int64_t)sg.plane * a.npt_pad;
  const int64_t xoff = (int64_t)sg.plane * a.npt;   // external plane offset
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int64_t e = 2 * qc[r];
    const bool v1 = e + 1 < sg.end;
    const int q = (int)(e - base);
    w[r].x = op_elem<TB, HL>(a, o, x, hl, sg.plane, e, q, true);
    const double y = op_elem<TB, HL>(a, o, x, hl, sg.plane, v1 ? e + 1 : e, v1 ? q + 1 : q, v1);
    w[r].y = v1 ? y : 0.0;
  }
  for (int c = 0; c < a.p; ++c) {
    const int64_t col = (int64_t)(a.p - c) * a.ldb + xoff - base;
    const double t = tc[c];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int64_t e = 2 * qc[r];
      const bool v1 = e + 1 < sg.end;
      const double b0 = a.B[col + e];
      const double b1 = a.B[col + (v1 ? e + 1 : e)];
      w[r].x += t * b0;
      w[r].y += v1 ? t * b1 : 0.0;
    }
  }
}

// ---- stage: u = [b_0; 0] (the leader adds mu e_p), max |b_k| for k >= 1 -----
// Partial slots: [0] = max |b_k|, [1] = 1 if a non-finite entry was seen.
__device__ inline void stage_pass(const Args& a, double* red) {
  const Rows o = own_rows(a);
  double mx = 0.0, bad = 0.0;
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    for (int64_t e = sg.beg + threadIdx.x; e < ((sg.end + 1) & ~(int64_t)1); e += kThreads) {
      double v = 0.0;
      if (!sg.tail && e < sg.end) {
        const int64_t eext = e - (int64_t)sg.plane * a.npt_pad + (int64_t)sg.plane * a.npt;
        v = a.B[eext];
        if (!isfinite(v)) bad = 1.0;
        for (int k = 1; k <= a.p; ++k) {
          const double b = a.B[(int64_t)k * a.ldb + eext];
          if (!isfinite(b)) bad = 1.0;
          mx = fmax(mx, fabs(b));
        }
      }
      a.u[e] = v;
    }
  }
  publish_halo(a, o, a.u);     // the tail is completed by the leader
  mx = block_max(mx, red);
  bad = block_max(bad, red);
  if (threadIdx.x == 0) {
    cstore(a.part + (int64_t)blockIdx.x * kKStride + 0, mx);
    cstore(a.part + (int64_t)blockIdx.x * kKStride + 1, bad);
  }
}

// ---- matvec + grouped inner products (Algorithm 4: matvec and reduction) ----
// Step jj (0-based; x = basis column jj, or u when jj == 0) writes w = Atilde x
// into column jj+1 (and x into column 0 at the first step) and the partial
// inner products of V_{1:j+1}^T [x_j, w] (eq. output_wywnrm):
//   slot 2i = x_i . x,  slot 2i+1 = x_i . w  (i <= jj),  slot 2jj+2 = w . w.
// sacc: kWaves * kKStride doubles of LDS; hl: the LDS halo copy (HL).
template <typename TB, bool HL>
__device__ inline void matvec_dots_pass(const Args& a, int jj, double inv_mu, double* sacc,
                                        double* hl) {
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const Rows o = own_rows(a);
  for (int k = threadIdx.x; k < kWaves * kKStride; k += kThreads) sacc[k] = 0.0;
  if (HL) stage_halo<TB>(a, o, hl);
  __syncthreads();
  TB* xcol = V + (int64_t)jj * ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const Src<TB> x{xcol, a.u, jj == 0};
  double tc[kPMax];
#pragma unroll
  for (int c = 0; c < kPMax; ++c) tc[c] = (c < a.p) ? rnd<TB>(cload(a.tx + c)) * inv_mu : 0.0;
  double sxx = 0.0, sxw = 0.0, sww = 0.0;
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * kR) {
      int64_t qc[kR];
      bool ok[kR];
      tile_pairs(q0, pend, qc, ok);
      double2 xv[kR], wv2[kR];
#pragma unroll
      for (int r = 0; r < kR; ++r) xv[r] = x.pair(2 * qc[r]);
      aug_tile<TB, HL>(a, o, sg, x, hl, qc, tc, wv2);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        wv2[r].x = rnd<TB>(wv2[r].x);
        wv2[r].y = rnd<TB>(wv2[r].y);
        if (ok[r]) {
          Pair<TB>::store(wcol + 2 * qc[r], wv2[r].x, wv2[r].y);
          if (jj == 0) Pair<TB>::store(xcol + 2 * qc[r], xv[r].x, xv[r].y);
        } else {
          xv[r] = make_double2(0.0, 0.0);
          wv2[r] = make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        sxx += xv[r].x * xv[r].x + xv[r].y * xv[r].y;
        sxw += xv[r].x * wv2[r].x + xv[r].y * wv2[r].y;
        sww += wv2[r].x * wv2[r].x + wv2[r].y * wv2[r].y;
      }
      // x_i . x and x_i . w for the older columns, kCh columns at a time
      int i0 = 0;
      for (; i0 < jj; i0 += kCh) {
        const int nc = min(kCh, jj - i0);
        double2 v[kCh][kR];
#pragma unroll
        for (int c = 0; c < kCh; ++c) {
          const TB* vc = V + (int64_t)(i0 + min(c, nc - 1)) * ld;
#pragma unroll
          for (int r = 0; r < kR; ++r) v[c][r] = Pair<TB>::load(vc + 2 * qc[r]);
        }
#pragma unroll
        for (int c = 0; c < kCh; ++c) {
          double ax = 0.0, aw = 0.0;
#pragma unroll
          for (int r = 0; r < kR; ++r) {
            ax += v[c][r].x * xv[r].x + v[c][r].y * xv[r].y;
            aw += v[c][r].x * wv2[r].x + v[c][r].y * wv2[r].y;
          }
          if (c < nc) {
            ax = wave_sum(ax);
            aw = wave_sum(aw);
            if (lane == 0) {
              sacc[wv * kKStride + 2 * (i0 + c)] += ax;
              sacc[wv * kKStride + 2 * (i0 + c) + 1] += aw;
            }
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
    cstore(a.part + (int64_t)blockIdx.x * kKStride + k, s);
  }
}

// ---- basis update (Algorithm 4: projection and normalisation) --------------
// x_{j+1} = coef[jj+1] * w + sum_{i<=jj} coef[i] x_i, in place over column jj+1
// (which holds w); the halo rows and the tail are published.  With want_norm,
// partial slot 0 = ||x_{j+1}||^2 (the exact norm of the newest vector, needed
// only when the Arnoldi process closes).  Columns are visited from the newest
// to the oldest, so the ones the previous matvec pass read last come first.
template <typename TB>
__device__ inline void update_pass(const Args& a, int jj, const double* coef, double* red,
                                   bool want_norm) {
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const double cw = coef[jj + 1];
  const Rows o = own_rows(a);
  double ss = 0.0;
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * kR) {
      int64_t qc[kR];
      bool ok[kR];
      tile_pairs(q0, pend, qc, ok);
      double2 acc[kR];
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const double2 w = Pair<TB>::load(wcol + 2 * qc[r]);
        acc[r] = make_double2(cw * w.x, cw * w.y);
      }
      int i1 = jj;
      for (; i1 >= kCu - 1; i1 -= kCu) axpy_cols<TB, kCu>(V, ld, i1, -1, coef, qc, acc);
      for (; i1 >= 0; --i1) axpy_cols<TB, 1>(V, ld, i1, -1, coef, qc, acc);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const double y0 = rnd<TB>(acc[r].x), y1 = rnd<TB>(acc[r].y);
        if (ok[r]) {
          Pair<TB>::store(wcol + 2 * qc[r], y0, y1);
          ss += y0 * y0 + y1 * y1;
        }
      }
    }
  }
  publish_halo(a, o, wcol);
  if (want_norm) {
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) cstore(a.part + (int64_t)blockIdx.x * kKStride, ss);
  }
}

// ---- combine: u = sum_{i<m} coef[i] x_i  (= beta V_m F, eq. kryexp) ----------
// Also writes out = u_top when this is the last substep.
template <typename TB>
__device__ inline void combine_pass(const Args& a, int m, const double* coef, bool last) {
  const TB* V = reinterpret_cast<const TB*>(a.V);
  const int64_t ld = a.ld;
  const Rows o = own_rows(a);
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    const int64_t shift = (int64_t)sg.plane * (a.npt - a.npt_pad);
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * kR) {
      int64_t qc[kR];
      bool ok[kR];
      tile_pairs(q0, pend, qc, ok);
      double2 acc[kR];
#pragma unroll
      for (int r = 0; r < kR; ++r) acc[r] = make_double2(0.0, 0.0);
      int i0 = 0;
      for (; i0 + kCu <= m; i0 += kCu) axpy_cols<TB, kCu>(V, ld, i0, 1, coef, qc, acc);
      for (; i0 < m; ++i0) axpy_cols<TB, 1>(V, ld, i0, 1, coef, qc, acc);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        if (ok[r]) {
          const int64_t e = 2 * qc[r];
          *reinterpret_cast<double2*>(a.u + e) = acc[r];
          if (last && !sg.tail) {
            if (e < sg.end) a.out[e + shift] = acc[r].x;
            if (e + 1 < sg.end) a.out[e + 1 + shift] = acc[r].y;
          }
        }
      }
    }
  }
  if (!last) publish_halo(a, o, a.u);
}

// ---- finish: out = u_top (or NaN when the input was not finite) -------------
__device__ inline void finish_pass(const Args& a, bool nonfinite) {
  const Rows o = own_rows(a);
  for (int si = 0; si < a.nplanes; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t shift = (int64_t)sg.plane * (a.npt - a.npt_pad);
    for (int64_t e = sg.beg + threadIdx.x; e < sg.end; e += kThreads)
      a.out[e + shift] = nonfinite ? __builtin_nan("") : a.u[e];
  }
}

}  // namespace kp
