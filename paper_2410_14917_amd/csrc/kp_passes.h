// Streaming passes over the augmented vectors (HBM-bound): stage, matvec fused
// with the grouped inner products, basis update fused with the norm, combine
// and finish.
//
// Workgroup b owns grid rows [r0, r1) = [b*rows_per_wg, ...) of every species
// plane, i.e. the internal elements [s*npt_pad + r0*nx, s*npt_pad + r1*nx) for
// each plane s ("segments").  Workgroup 0 also owns the p entries of the
// augmented tail; they are handled column-parallel (one lane per basis column)
// after its segments, so the tail costs one memory round trip rather than a
// sweep over all columns.
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

// A wave-uniform pointer, kept in scalar registers: column accesses are then a
// scalar base plus a 32-bit per-lane byte offset, and the compiler cannot
// re-associate the base into per-lane 64-bit loop invariants.
template <typename T>
__device__ inline T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

#define KP_GLOBAL __attribute__((address_space(1)))
typedef double kp_d2 __attribute__((ext_vector_type(2)));
typedef float kp_f2 __attribute__((ext_vector_type(2)));

template <typename TB>
__device__ inline double2 load_at(const TB* base, uint32_t byte_off) {
  const KP_GLOBAL char* p = (const KP_GLOBAL char*)base + byte_off;
  if constexpr (sizeof(TB) == 8) {
    const kp_d2 v = *(const KP_GLOBAL kp_d2*)p;
    return make_double2(v.x, v.y);
  } else {
    const kp_f2 v = *(const KP_GLOBAL kp_f2*)p;
    return make_double2((double)v.x, (double)v.y);
  }
}

// Vector multiplied by the matvec of step jj: the float64 state u at the first
// step (rounded through the basis type, which is what basis column 0 stores),
// the stored basis column afterwards.  Own elements only (plain loads).
template <typename TB>
struct Src {
  static constexpr bool kLds = false;
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

// A plain basis column: the matvec passes read x_j through it, having copied
// the state into column 0 before the first step's pass, so that no element
// load chooses between two sources (such a choice put a branch, and a wait for
// memory, after every load of the stencil).
template <typename TB>
struct Col {
  static constexpr bool kLds = false;
  const TB* col;
  __device__ double operator()(int64_t e) const { return (double)col[e]; }
  __device__ double2 pair(int64_t e) const { return Pair<TB>::load(col + e); }
};

// x_j of a workgroup that owns one sub-tile, in LDS as the basis update left
// it: element e of the block at l[e - t0] (t0: the block's first pair).
struct LdsX {
  static constexpr bool kLds = true;
  const double* l;
  int64_t t0;
  __device__ double operator()(int64_t e) const { return l[e - t0]; }
};

// ---- ownership --------------------------------------------------------------

struct Rows {
  int r0, r1;
};

__device__ inline Rows own_rows(const Args& a) {
  Rows o;
  o.r0 = min(a.ny, wg_rank(a) * a.rows_per_wg);
  o.r1 = min(a.ny, o.r0 + a.rows_per_wg);
  return o;
}

// One owned segment: elements [beg, end) of plane `plane`.
struct Seg {
  int64_t beg, end;
  int plane;
};

__device__ inline int num_segs(const Args& a) { return a.nplanes; }

__device__ inline Seg seg_at(const Args& a, const Rows& o, int si) {
  const int64_t base = (int64_t)si * a.npt_pad;
  return Seg{base + (int64_t)o.r0 * a.nx, base + (int64_t)o.r1 * a.nx, si};
}

// Offset of plane s in the caller's arrays (B, fields): the plain layout puts
// plane s at s*npt; in tangent mode both planes belong to one plane of the
// operator.
__device__ inline int64_t ext_off(const Args& a, int s) {
  return a.tangent ? 0 : (int64_t)s * a.npt;
}

// Output array of plane s (indexed by the in-plane index).
__device__ inline double* out_plane(const Args& a, int s) {
  if (a.tangent) return s == 0 ? a.dout : a.out;
  return a.out + (int64_t)s * a.npt;
}

// The tail shift K acts within each block of pb entries (two blocks in
// tangent mode): entry k takes entry k+1 unless k closes its block.
__device__ inline bool tail_shift_in(const Args& a, int k) {
  return k + 1 < a.p && ((k + 1) % a.pb) != 0;
}

// Copies the state u (rounded to the basis type) into column 0 over the
// workgroup's own pairs (with the padding element of an odd segment end),
// before the first step's matvec pass reads it there (the pass's barrier
// orders the stores before the loads).
template <typename TB>
__device__ inline void copy_state(const Args& a, const Rows& o, TB* col0) {
  for (int si = 0; si < num_segs(a); ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t end = 2 * ((sg.end + 1) >> 1);
    for (int64_t e = sg.beg + kp_tid(); e < end; e += kThreads) col0[e] = (TB)a.u[e];
  }
}

constexpr int kR = 4;    // element pairs per thread per sub-tile
constexpr int kCh = 2;   // basis columns per chunk of the inner-product loop
constexpr int kCu = 5;   // basis columns per chunk of the linear combinations
// ... per basis type: a float basis takes two columns per chunk (measured over
// 1, 2, 3, 4 and 6: two fastest), a float64 one kCu
template <typename TB> constexpr int kCuOf = sizeof(TB) == 4 ? 2 : kCu;

// Element offsets of this lane's kR pairs in the sub-tile that starts at
// element 2*q0 (lane offsets stay below 2 * kThreads * kR, so every column
// access is a uniform base plus a 32-bit lane offset); pairs past pend are
// clamped to the last pair (ok = false).
__device__ inline void tile_pairs(int64_t q0, int64_t pend, uint32_t* lo, bool* ok) {
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int64_t q = q0 + (int64_t)r * kThreads + kp_tid();
    ok[r] = q < pend;
    lo[r] = (uint32_t)(2 * ((ok[r] ? q : pend - 1) - q0));
  }
}

// Columns of one chunk are held as loaded (a float basis stays packed until
// it is multiplied), so that a float chunk of 2 * kCh columns takes the
// registers of a double chunk of kCh: the float pass keeps as many bytes in
// flight as the double one.  Each column's sums are formed and recorded on
// their own, so the chunk width does not change any result.
template <typename TB> struct Raw;
template <> struct Raw<double> {
  typedef double2 type;
  static constexpr int kCols = kCh;
  __device__ static double2 load(const double* base, uint32_t byte_off) {
    return load_at(base, byte_off);
  }
};
template <> struct Raw<float> {
  typedef kp_f2 type;
  static constexpr int kCols = 2 * kCh;
  __device__ static kp_f2 load(const float* base, uint32_t byte_off) {
    return *(const KP_GLOBAL kp_f2*)((const KP_GLOBAL char*)base + byte_off);
  }
};

// acc[r] += sum over the nc columns i = i0, i0 + step, ... of coef[i] V_i(pair r),
// the columns in that order; nc <= C is wave-uniform.  The loads are kept as
// stored (float pairs stay packed) and widened at use.  The columns past nc
// add nothing: a double chunk loads them as repeats of the last column with
// coefficient 0, so that all C * kR loads issue before the first multiply-add
// without a branch; a float chunk skips them behind a uniform branch (measured
// faster for each type: 2 % and 1 % of the benchmark calls against
// single-column remainder steps).  The coefficients are read with coherent
// loads (they were published by the leader), issued with the column loads.
template <typename TB, int C>
__device__ inline void axpy_cols(const TB* V, int64_t ld, int64_t t0, int i0, int step, int nc,
                                 const double* coef, const uint32_t* lo, double2* acc) {
  typename Raw<TB>::type v[C][kR];
  double ci[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i = i0 + min(c, nc - 1) * step;
    const TB* vc = uniform_ptr(V + (int64_t)i * ld + t0);
    if constexpr (sizeof(TB) == 8) {
      const double cv = cload(coef + i);
      ci[c] = (c < nc) ? cv : 0.0;
#pragma unroll
      for (int r = 0; r < kR; ++r) v[c][r] = Raw<TB>::load(vc, lo[r] * (uint32_t)sizeof(TB));
    } else if (c < nc) {
      ci[c] = cload(coef + i);
#pragma unroll
      for (int r = 0; r < kR; ++r) v[c][r] = Raw<TB>::load(vc, lo[r] * (uint32_t)sizeof(TB));
    } else {
      ci[c] = 0.0;
#pragma unroll
      for (int r = 0; r < kR; ++r) v[c][r] = typename Raw<TB>::type{};
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < kR; ++r) {   // fused multiply-adds, written out (update_pass
      acc[r].x = __builtin_fma(ci[c], (double)v[c][r].x, acc[r].x);   // repeats them)
      acc[r].y = __builtin_fma(ci[c], (double)v[c][r].y, acc[r].y);
    }
}


// Index of the halo slot of (workgroup w, plane s, side: 0 first row, 1 last row).
__device__ inline int64_t halo_at(const Args& a, int w, int s, int side, int ix) {
  return ((int64_t)(w * a.nplanes + s) * 2 + side) * a.nx + ix;
}

// A producer of a vector that the next matvec multiplies publishes, with
// coherent stores, the elements of the first and last row of each owned plane
// segment (the stencil halo of the neighbouring workgroups).  Called for the
// element pair (e, e+1) of segment sg with the values as stored; lanes outside
// the boundary rows store nothing.  (The tail is published by tail_update /
// tail_combine.)
__device__ inline void publish_elem(const Args& a, const Seg& sg, int64_t e, double v) {
  if (e >= sg.end) return;
  const int64_t off = e - sg.beg, last0 = sg.end - sg.beg - a.nx;
  if (off < a.nx) cstore(a.hx + halo_at(a, wg_rank(a), sg.plane, 0, (int)off), v);
  if (off >= last0) cstore(a.hx + halo_at(a, wg_rank(a), sg.plane, 1, (int)(off - last0)), v);
}

__device__ inline void publish_pair(const Args& a, const Seg& sg, int64_t e, double v0,
                                    double v1) {
  if (e - sg.beg < a.nx || e + 1 >= sg.end - a.nx) {
    publish_elem(a, sg, e, v0);
    publish_elem(a, sg, e + 1, v1);
  }
}

// Copy the halo rows this workgroup's stencil needs (the first row of the next
// workgroup, the last row of the previous one, periodic) into LDS:
// hl[s * nx + ix] = row r1 (mod ny), hl[(nplanes + s) * nx + ix] = row r0 - 1.
template <typename TB>
__device__ inline void stage_halo(const Args& a, const Rows& o, double* hl) {
  const int nx = a.nx, b = wg_rank(a);
  const int wn = (o.r1 == a.ny) ? 0 : b + 1;
  const int ws = (o.r0 == 0) ? a.nwg - 1 : b - 1;
  for (int s = 0; s < a.nplanes; ++s)
    for (int ix = kp_tid(); ix < nx; ix += kThreads) {
      hl[s * nx + ix] = rnd<TB>(cload(a.hx + halo_at(a, wn, s, 0, ix)));
      hl[(a.nplanes + s) * nx + ix] = rnd<TB>(cload(a.hx + halo_at(a, ws, s, 1, ix)));
    }
}

// ---- the operator on one grid element ---------------------------------------
//
// (A x)_e for grid element e (internal index) of plane s, whose in-plane index
// is q (row, ix).  Neighbours inside the owned rows are read from x (the
// basis column, or LDS where the update left x_j); the rows just outside come from the LDS halo copy (HL) or from the coherent halo
// slots.  All loads are unconditional (dummy indices where unused).
template <typename TB, bool HL, typename XS>
__device__ inline double op_elem(const Args& a, const Rows& o, const XS& x, const double* hl,
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
  // (the multiply-adds are written out, so that every instantiation of the
  // stencil, x from the basis or from LDS, rounds alike)
  const double cxx = (s && !a.tangent) ? a.cx2 : a.cx, cyy = (s && !a.tangent) ? a.cy2 : a.cy;
  const double lap = __builtin_fma(cxx, __builtin_fma(-2.0, c, xe + xw),
                                   cyy * __builtin_fma(-2.0, c, xn + xs));
  double tv = 0.0;
  if (!XS::kLds && a.tangent && s == 0) {   // (one plane when x is in LDS)
    // dA applied to the c half (plane 1) at the same point (Van Loan block)
    const int64_t o = a.npt_pad;
    const double c1 = xo;
    const double e1 = x((valid ? ie : e) + o), w1 = x((valid ? iw : e) + o);
    double n1 = x(in + o), s1 = x(is + o);
    if (HL) {
      const double hn1 = hl[1 * nx + ix];
      const double hs1 = hl[(a.nplanes + 1) * nx + ix];
      n1 = hn ? n1 : hn1;
      s1 = hs ? s1 : hs1;
    } else {
      if (!hn) {
        const int rn = (row + 1 == a.ny) ? 0 : row + 1;
        n1 = rnd<TB>(cload(a.hx + halo_at(a, (int)((unsigned)rn / (unsigned)a.rows_per_wg), 1, 0, ix)));
      }
      if (!hs) {
        const int rs = (row == 0) ? a.ny - 1 : row - 1;
        s1 = rnd<TB>(cload(a.hx + halo_at(a, (int)((unsigned)rs / (unsigned)a.rows_per_wg), 1, 1, ix)));
      }
    }
    const double dadv = __builtin_fma(a.dadx, e1 - w1, a.dady * (n1 - s1));
    const double dlap = __builtin_fma(a.dcx, __builtin_fma(-2.0, c1, e1 + w1),
                                      a.dcy * __builtin_fma(-2.0, c1, n1 + s1));
    tv = __builtin_fma(a.dreact, c1, dlap + (a.transpose ? dadv : -dadv));
  }
  if (a.kind == KP_OP_ADR) {
    const double adv = __builtin_fma(a.adx, xe - xw, a.ady * (xn - xs));
    return __builtin_fma(a.react + U, c, lap + (a.transpose ? adv : -adv)) + tv;
  }
  if (a.kind == KP_OP_ALLEN_CAHN) return __builtin_fma(__builtin_fma(-3.0 * U, U, 1.0), c, lap) + tv;
  // Brusselator Jacobian: pointwise blocks [[a11, a12], [a21, a22]]; the other
  // species at the same point (xo) is owned by this workgroup too.
  const double a11 = __builtin_fma(2.0 * U, W, -(a.bb + 1.0)), a12 = U * U;
  const double a21 = __builtin_fma(-2.0 * U, W, a.bb), a22 = -(U * U);
  if (!a.transpose)
    return s ? __builtin_fma(a22, c, __builtin_fma(a21, xo, lap))
             : __builtin_fma(a12, xo, __builtin_fma(a11, c, lap));
  return s ? __builtin_fma(a22, c, __builtin_fma(a12, xo, lap))
           : __builtin_fma(a21, xo, __builtin_fma(a11, c, lap));
}

// (Atilde x) on the kR pairs of a sub-tile of plane segment sg:
// A x_top + sum_c tc[c] b_{p-c} (the tail rows, K x_tail, are done by
// tail_matvec_dots); zero in the padding.
template <typename TB, bool HL, typename XS>
__device__ inline void aug_tile(const Args& a, const Rows& o, const Seg& sg, const XS& x,
                                const double* hl, int64_t t0, const uint32_t* lo,
                                const double* tc, double2* w) {
  const int64_t base = (int64_t)sg.plane * a.npt_pad;
  const int64_t xoff = ext_off(a, sg.plane);         // offset in the caller's arrays
  // B-hat x_tail / mu: the columns b_{p-c}, two at a time with all their
  // loads issued before the first use (the first two go out with the
  // stencil's loads)
  double b0[2][kR][2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (c < a.pb) {
      const int64_t col = (int64_t)(a.pb - c) * a.ldb + xoff - base;
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int64_t e = t0 + lo[r];
        b0[c][r][0] = a.B[col + e];
        b0[c][r][1] = a.B[col + ((e + 1 < sg.end) ? e + 1 : e)];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int64_t e = t0 + lo[r];
    const bool v1 = e + 1 < sg.end;
    const int q = (int)(e - base);
    w[r].x = op_elem<TB, HL>(a, o, x, hl, sg.plane, e, q, true);
    const double y = op_elem<TB, HL>(a, o, x, hl, sg.plane, v1 ? e + 1 : e, v1 ? q + 1 : q, v1);
    w[r].y = v1 ? y : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (c < a.pb) {
      const double t = tc[c];
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const bool v1 = t0 + lo[r] + 1 < sg.end;
        w[r].x = __builtin_fma(t, b0[c][r][0], w[r].x);
        w[r].y = v1 ? __builtin_fma(t, b0[c][r][1], w[r].y) : w[r].y;
      }
    }
  }
  for (int c0 = 2; c0 < a.pb; c0 += 2) {
    double bv[2][kR][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (c0 + c < a.pb) {
        const int64_t col = (int64_t)(a.pb - c0 - c) * a.ldb + xoff - base;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          const int64_t e = t0 + lo[r];
          bv[c][r][0] = a.B[col + e];
          bv[c][r][1] = a.B[col + ((e + 1 < sg.end) ? e + 1 : e)];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (c0 + c < a.pb) {
        const double t = tc[c0 + c];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          const bool v1 = t0 + lo[r] + 1 < sg.end;
          w[r].x = __builtin_fma(t, bv[c][r][0], w[r].x);
          w[r].y = v1 ? __builtin_fma(t, bv[c][r][1], w[r].y) : w[r].y;
        }
      }
    }
  }
}

// ---- both species of the Brusselator at one grid point ------------------------
//
// The two planes of the Brusselator Jacobian couple only pointwise, so one
// pass can take both species of a grid point together: the fields U, W and
// both centres are loaded once for the two results (each species is the
// other's coupling term), and one memory round trip yields two elements.
// Element e is in plane 0 (in-plane index q), e + npt_pad its partner in
// plane 1; y0, y1 round exactly as op_elem's results for the two planes.
template <typename TB, bool HL, typename XS>
__device__ inline void op_br2(const Args& a, const Rows& o, const XS& x, const double* hl,
                              int64_t e, int q, bool valid, double& y0, double& y1) {
  const int nx = a.nx;
  const int64_t P = a.npt_pad;
  int row = (int)((double)q * a.inv_nx);   // q / nx, corrected by one step
  row -= ((unsigned)row * (unsigned)nx > (unsigned)q) ? 1 : 0;
  row += ((unsigned)(row + 1) * (unsigned)nx <= (unsigned)q) ? 1 : 0;
  const int ix = q - row * nx;
  const bool hn = row + 1 < o.r1, hs = row > o.r0;
  const int64_t ie = (valid && ix != nx - 1) ? e + 1 : (valid ? e - ix : e);
  const int64_t iw = (valid && ix != 0) ? e - 1 : (valid ? e + nx - 1 : e);
  const int64_t in = (hn && valid) ? e + nx : e;
  const int64_t is = (hs && valid) ? e - nx : e;
  const double c0 = x(e), c1 = x(e + P);
  const double e0 = x(ie), e1 = x(ie + P);
  const double w0 = x(iw), w1 = x(iw + P);
  double n0 = x(in), n1 = x(in + P);
  double s0 = x(is), s1 = x(is + P);
  const int qf = valid ? q : 0;
  const double U = a.f0[qf], W = a.f1[qf];
  if (HL) {
    n0 = hn ? n0 : hl[0 * nx + ix];
    n1 = hn ? n1 : hl[1 * nx + ix];
    s0 = hs ? s0 : hl[2 * nx + ix];
    s1 = hs ? s1 : hl[3 * nx + ix];
  } else {
    if (!hn) {
      const int rn = (row + 1 == a.ny) ? 0 : row + 1;
      const int wn = (int)((unsigned)rn / (unsigned)a.rows_per_wg);
      n0 = rnd<TB>(cload(a.hx + halo_at(a, wn, 0, 0, ix)));
      n1 = rnd<TB>(cload(a.hx + halo_at(a, wn, 1, 0, ix)));
    }
    if (!hs) {
      const int rs = (row == 0) ? a.ny - 1 : row - 1;
      const int ws = (int)((unsigned)rs / (unsigned)a.rows_per_wg);
      s0 = rnd<TB>(cload(a.hx + halo_at(a, ws, 0, 1, ix)));
      s1 = rnd<TB>(cload(a.hx + halo_at(a, ws, 1, 1, ix)));
    }
  }
  const double lap0 = __builtin_fma(a.cx, __builtin_fma(-2.0, c0, e0 + w0),
                                    a.cy * __builtin_fma(-2.0, c0, n0 + s0));
  const double lap1 = __builtin_fma(a.cx2, __builtin_fma(-2.0, c1, e1 + w1),
                                    a.cy2 * __builtin_fma(-2.0, c1, n1 + s1));
  const double a11 = __builtin_fma(2.0 * U, W, -(a.bb + 1.0)), a12 = U * U;
  const double a21 = __builtin_fma(-2.0 * U, W, a.bb), a22 = -(U * U);
  const double k0 = a.transpose ? a21 : a12, k1 = a.transpose ? a12 : a21;
  y0 = __builtin_fma(k0, c1, __builtin_fma(a11, c0, lap0));
  y1 = __builtin_fma(a22, c1, __builtin_fma(k1, c0, lap1));
}

// Pairs of a joint sub-tile: pairs r < kR/2 at in-plane pair positions
// q0 + r * kThreads + tid of plane 0, pairs r >= kR/2 at the same positions in
// plane 1 (offset npt_pad); clamped and flagged like tile_pairs.
__device__ inline void tile_pairs_joint(int64_t q0, int64_t pend, int64_t P, uint32_t* lo,
                                        bool* ok) {
#pragma unroll
  for (int r = 0; r < kR / 2; ++r) {
    const int64_t q = q0 + (int64_t)r * kThreads + kp_tid();
    ok[r] = ok[r + kR / 2] = q < pend;
    lo[r] = (uint32_t)(2 * ((ok[r] ? q : pend - 1) - q0));
    lo[r + kR / 2] = lo[r] + (uint32_t)P;
  }
}

// (Atilde x) on a joint sub-tile (both species, plane-0 segment sg): the
// stencil by op_br2, then sum_c tc[c] b_{p-c} on each plane's pairs.
template <typename TB, bool HL, typename XS>
__device__ inline void aug_tile_br2(const Args& a, const Rows& o, const Seg& sg, const XS& x,
                                    const double* hl, int64_t t0, const uint32_t* lo,
                                    const double* tc, double2* w) {
  // plane s's pairs sit at s * npt in the caller's B, at s * npt_pad here
  const int64_t boff1 = (int64_t)a.npt - a.npt_pad;
  bool v1[kR];
#pragma unroll
  for (int r = 0; r < kR; ++r) v1[r] = t0 + lo[r % (kR / 2)] + 1 < sg.end;
  // the columns b_{p-c}, two at a time; the first two go out with the
  // stencil's loads
  auto load_b = [&](int c0, double (&bv)[2][kR][2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (c0 + c < a.pb) {
        const int64_t col = (int64_t)(a.pb - c0 - c) * a.ldb;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          const int64_t e = t0 + lo[r];
          const int64_t ce = col + (r < kR / 2 ? 0 : boff1);
          bv[c][r][0] = a.B[ce + e];
          bv[c][r][1] = a.B[ce + (v1[r] ? e + 1 : e)];
        }
      }
    }
  };
  auto add_b = [&](int c0, const double (&bv)[2][kR][2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (c0 + c < a.pb) {
        const double t = tc[c0 + c];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          w[r].x = __builtin_fma(t, bv[c][r][0], w[r].x);
          w[r].y = v1[r] ? __builtin_fma(t, bv[c][r][1], w[r].y) : w[r].y;
        }
      }
    }
  };
  double b0[2][kR][2];
  load_b(0, b0);
#pragma unroll
  for (int r = 0; r < kR / 2; ++r) {
    const int64_t e = t0 + lo[r];
    const int q = (int)e;   // (plane 0: the internal index is the in-plane one)
    double y00, y01, y10, y11;
    op_br2<TB, HL>(a, o, x, hl, e, q, true, y00, y01);
    op_br2<TB, HL>(a, o, x, hl, v1[r] ? e + 1 : e, v1[r] ? q + 1 : q, v1[r], y10, y11);
    w[r] = make_double2(y00, v1[r] ? y10 : 0.0);
    w[r + kR / 2] = make_double2(y01, v1[r] ? y11 : 0.0);
  }
  add_b(0, b0);
  for (int c0 = 2; c0 < a.pb; c0 += 2) {
    double bv[2][kR][2];
    load_b(c0, bv);
    add_b(c0, bv);
  }
}

// ---- the augmented tail (workgroup 0) -----------------------------------------
// The p tail entries of every vector are handled column-parallel: lane i of
// wave 0 takes basis column i (and i + 64), so the work is one memory round
// trip and at most kPMax wave reductions.

// Tail rows of the matvec of step jj (w_tail = K x_tail, the upward shift
// within each block of pb entries; x_tail is also stored at the first step) and their share of the inner
// products: x_i . x and x_i . w (slots 2i, 2i+1 of wave 0's row of sacc) and
// x . x, x . w, w . w (slots 2jj .. 2jj+2).
template <typename TB>
__device__ inline void tail_matvec_dots(const Args& a, int jj, const Src<TB>& x, TB* V,
                                        double* sacc) {
  const int t = kp_tid();
  if (t >= 64) return;
  const int64_t T0 = a.tail_off, ld = a.ld;
  const int p = a.p;
  TB* xcol = V + (int64_t)jj * ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  double xt[kPMax], wt[kPMax];
#pragma unroll
  for (int k = 0; k < kPMax; ++k) xt[k] = (k < p) ? x(T0 + k) : 0.0;
#pragma unroll
  for (int k = 0; k < kPMax; ++k) wt[k] = (k + 1 < kPMax && tail_shift_in(a, k)) ? xt[k + 1] : 0.0;
  if (t < p) {
    wcol[T0 + t] = (TB)(tail_shift_in(a, t) ? x(T0 + t + 1) : 0.0);
    if (jj == 0) xcol[T0 + t] = (TB)x(T0 + t);
  }
  if (t < jj) {
    const TB* vc = V + (int64_t)t * ld + T0;
    double sx = 0.0, sw = 0.0;
#pragma unroll
    for (int k = 0; k < kPMax; ++k) {
      if (k < p) {
        const double v = (double)vc[k];
        sx += v * xt[k];
        sw += v * wt[k];
      }
    }
    sacc[2 * t] += sx;
    sacc[2 * t + 1] += sw;
  }
  if (t == 0) {
    double xx = 0.0, xw = 0.0, ww = 0.0;
#pragma unroll
    for (int k = 0; k < kPMax; ++k) {
      xx += xt[k] * xt[k];
      xw += xt[k] * wt[k];
      ww += wt[k] * wt[k];
    }
    sacc[2 * jj] += xx;
    sacc[2 * jj + 1] += xw;
    sacc[2 * jj + 2] += ww;
  }
}

// Tail of u = sum_{i < nc} c_i V_i, where c_i = coef[i] (coherent loads) and,
// when extra_col >= 0, column extra_col enters with weight cextra.  Result in
// place of out_col's tail (or of a.u when out_col is null), published to the
// tail copy when publish.  Returns sum y_k^2 in lane 0 of wave 0.
template <typename TB, typename TO>
__device__ inline double tail_combine_cols(const Args& a, const TB* V, int nc, const double* coef,
                                           int extra_col, double cextra, TO* out, bool publish) {
  const int t = kp_tid();
  if (t >= 64) return 0.0;
  const int64_t T0 = a.tail_off, ld = a.ld;
  const int p = a.p;
  double part[kPMax];
#pragma unroll
  for (int k = 0; k < kPMax; ++k) part[k] = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = t + 64 * h;
    const bool on = i < nc || i == extra_col;
    const double ci = on ? ((i == extra_col) ? cextra : cload(coef + i)) : 0.0;
    const TB* vc = V + (int64_t)(on ? i : 0) * ld + T0;
#pragma unroll
    for (int k = 0; k < kPMax; ++k)
      if (k < p && on) part[k] += ci * (double)vc[k];
  }
  double ss = 0.0;
#pragma unroll
  for (int k = 0; k < kPMax; ++k) {
    if (k < p) {
      const double y = rnd<TO>(wave_sum(part[k]));
      if (t == 0) {
        out[T0 + k] = (TO)y;
        if (publish) cstore(a.tx + k, y);
        ss += y * y;
      }
    }
  }
  return ss;
}

// ---- stage: u = [b_0; 0] (the leader adds mu e_p), max |b_k| for k >= 1 -----
// (tangent mode: u = [0; b_0], the a half zero.)
// Partial slots: [0] = max |b_k|, [1] = 1 if a non-finite entry was seen.
__device__ __attribute__((always_inline)) inline void stage_pass(const Args& a, double* red) {
  const Rows o = own_rows(a);
  double mx = 0.0, bad = 0.0;
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const bool zero = a.tangent && sg.plane == 0;
    const int64_t xoff = ext_off(a, sg.plane) - (int64_t)sg.plane * a.npt_pad;
    for (int64_t e = sg.beg + kp_tid(); e < ((sg.end + 1) & ~(int64_t)1); e += kThreads) {
      double v = 0.0;
      if (e < sg.end && !zero) {
        const int64_t eext = e + xoff;
        v = a.B[eext];
        if (!isfinite(v)) bad = 1.0;
        for (int k = 1; k <= a.pb; ++k) {
          const double b = a.B[(int64_t)k * a.ldb + eext];
          if (!isfinite(b)) bad = 1.0;
          mx = fmax(mx, fabs(b));
        }
      }
      a.u[e] = v;
      publish_elem(a, sg, e, v);   // the tail is staged by the leader
    }
  }
  mx = block_max(mx, red);
  bad = block_max(bad, red);
  if (kp_tid() == 0) {
    cstore(a.part + (int64_t)wg_rank(a) * kKStride + 0, mx);
    cstore(a.part + (int64_t)wg_rank(a) * kKStride + 1, bad);
  }
}

// ---- matvec + grouped inner products (Algorithm 4: matvec and reduction) ----
// Step jj (0-based; x = basis column jj, or u when jj == 0) writes w = Atilde x
// into column jj+1 (and x into column 0 at the first step) and the partial
// inner products of V_{1:j+1}^T [x_j, w] (eq. output_wywnrm):
//   slot 2i = x_i . x,  slot 2i+1 = x_i . w  (i <= jj),  slot 2jj+2 = w . w.
// sacc: kWaves * kKStride doubles of LDS; hl: the LDS halo copy (HL); prow:
// this workgroup's row of the step buffer of the phase's barrier; own: the
// leader's LDS copy of its sums (nullptr in the other workgroups).
//
// The older columns are visited a chunk at a time (kCh columns of a double
// basis, 2 * kCh of a float one), software-pipelined: the loads of the next
// chunk are in flight while the wave reduces the current one.


// Per-wave sums of x_i . x and x_i . w for the C columns of one chunk
// (columns past nc repeat the last one and are not recorded).
template <int C, typename R>
__device__ inline void dots_chunk(const R (&v)[C][kR], const double2* xv,
                                  const double2* wv2, int i0, int nc, double* sacc) {
  const int lane = kp_tid() & 63, wv = kp_tid() >> 6;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    double ax = 0.0, aw = 0.0;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const double vx = (double)v[c][r].x, vy = (double)v[c][r].y;
      ax = __builtin_fma(vy, xv[r].y, __builtin_fma(vx, xv[r].x, ax));
      aw = __builtin_fma(vy, wv2[r].y, __builtin_fma(vx, wv2[r].x, aw));
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

template <typename TB, int C>
__device__ inline void load_chunk(const TB* V, int64_t ld, int64_t t0, int i0, int nc,
                                  const uint32_t* lo, typename Raw<TB>::type (&v)[C][kR]) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const TB* vc = uniform_ptr(V + (int64_t)(i0 + min(c, nc - 1)) * ld + t0);
#pragma unroll
    for (int r = 0; r < kR; ++r) v[c][r] = Raw<TB>::load(vc, lo[r] * (uint32_t)sizeof(TB));
  }
}

// KEEP (keep_xw: one plane, one sub-tile per workgroup): the region hl of LDS
// holds x_j as pairs (slot r * kThreads + tid, i.e. element e of the block at
// hl[e - t0]) and w (slot (kR + r) * kThreads + tid), both as double2; the
// halo copy moves to the w half.  After the final barrier, when no stencil
// reads either any more, each thread leaves its pairs of x_j and w there for
// the next phase's update, which then needs neither from the basis: w is not
// stored.  XL (with KEEP): the update of this phase has left x_j in the x
// half, so the stencil and the inner products read it from LDS.
template <typename TB, bool HL, bool KEEP, bool XL, bool JT = false>
__device__ __attribute__((always_inline)) inline void matvec_dots_pass(const Args& a, int jj, double* sacc, double* hl,
                                                        double* prow, double* own) {
  static_assert(KEEP || !XL, "x_j is in LDS only where the pass keeps x_j and w");
  static_assert(!(JT && KEEP), "the joint two-species tiles keep nothing on chip");
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  const int lane = kp_tid() & 63, wv = kp_tid() >> 6;
  const Rows o = own_rows(a);
  double* hh = KEEP ? hl + 2 * kR * kThreads : hl;   // the halo copy
  for (int k = kp_tid(); k < kWaves * kKStride; k += kThreads) sacc[k] = 0.0;
  if (HL) stage_halo<TB>(a, o, hh);
  const double inv_mu = cload(&a.pub->inv_mu);
  TB* xcol = V + (int64_t)jj * ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const Src<TB> x{xcol, a.u, jj == 0};   // (the tail entries)
  const Col<TB> xc{xcol};
  if (jj == 0) copy_state<TB>(a, o, xcol);
  __syncthreads();
  double sxx = 0.0, sxw = 0.0, sww = 0.0;
  double2 kx[KEEP && !XL ? kR : 1], kw[KEEP ? kR : 1];   // (with XL, x_j stays where it is)
  // (JT: the Brusselator's two planes in joint sub-tiles over plane 0's rows)
  const int ns = JT ? 1 : num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    // tail entries divided by mu that multiply b_{pb-c} in this plane (the c
    // half of the tail in the tangent mode's plane 1)
    const int toff = (a.tangent && sg.plane == 1) ? a.pb : 0;
    double tc[kPMax];
#pragma unroll
    for (int c = 0; c < kPMax; ++c)
      tc[c] = (c < a.pb) ? rnd<TB>(cload(a.tx + toff + c)) * inv_mu : 0.0;
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * (JT ? kR / 2 : kR)) {
      const int64_t t0 = 2 * q0;
      uint32_t lo[kR];
      bool ok[kR];
      if constexpr (JT)
        tile_pairs_joint(q0, pend, a.npt_pad, lo, ok);
      else
        tile_pairs(q0, pend, lo, ok);
      double2 xv[kR], wv2[kR];
      constexpr int CC = Raw<TB>::kCols;
      typename Raw<TB>::type va[CC][kR], vb[CC][kR];
      // (the first chunk of older columns goes out with the stencil's loads)
      if (jj > 0) load_chunk<TB, CC>(V, ld, t0, 0, min(CC, jj), lo, va);
      if constexpr (XL) {
        const LdsX lx{hl, t0};   // (one sub-tile: t0 is the block's first pair)
#pragma unroll
        for (int r = 0; r < kR; ++r) xv[r] = *reinterpret_cast<const double2*>(hl + lo[r]);
        aug_tile<TB, HL>(a, o, sg, lx, hh, t0, lo, tc, wv2);
      } else {
#pragma unroll
        for (int r = 0; r < kR; ++r) xv[r] = xc.pair(t0 + lo[r]);
        if constexpr (JT)
          aug_tile_br2<TB, HL>(a, o, sg, xc, hh, t0, lo, tc, wv2);
        else
          aug_tile<TB, HL>(a, o, sg, xc, hh, t0, lo, tc, wv2);
      }
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        wv2[r].x = rnd<TB>(wv2[r].x);
        wv2[r].y = rnd<TB>(wv2[r].y);
        if (ok[r]) {
          if (!KEEP) Pair<TB>::store(wcol + t0 + lo[r], wv2[r].x, wv2[r].y);
          if (jj == 0) Pair<TB>::store(xcol + t0 + lo[r], xv[r].x, xv[r].y);
        } else {
          xv[r] = make_double2(0.0, 0.0);
          wv2[r] = make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        sxx = __builtin_fma(xv[r].y, xv[r].y, __builtin_fma(xv[r].x, xv[r].x, sxx));
        sxw = __builtin_fma(xv[r].y, wv2[r].y, __builtin_fma(xv[r].x, wv2[r].x, sxw));
        sww = __builtin_fma(wv2[r].y, wv2[r].y, __builtin_fma(wv2[r].x, wv2[r].x, sww));
      }
      // x_i . x and x_i . w for the older columns, two chunks in flight
      for (int i0 = 0; i0 < jj; i0 += 2 * CC) {
        const int i1 = i0 + CC;
        if (i1 < jj) load_chunk<TB, CC>(V, ld, t0, i1, min(CC, jj - i1), lo, vb);
        dots_chunk<CC>(va, xv, wv2, i0, min(CC, jj - i0), sacc);
        if (i1 >= jj) break;
        const int i2 = i1 + CC;
        if (i2 < jj) load_chunk<TB, CC>(V, ld, t0, i2, min(CC, jj - i2), lo, va);
        dots_chunk<CC>(vb, xv, wv2, i1, min(CC, jj - i1), sacc);
      }
      if constexpr (KEEP) {
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          if constexpr (!XL) kx[r] = xv[r];
          kw[r] = wv2[r];
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
  if (wg_rank(a) == 0) tail_matvec_dots<TB>(a, jj, x, V, sacc);
  __syncthreads();
  // slot k is written by thread k, the thread that reset it (step_part); the
  // leader keeps its own sums in LDS (own), where its reduction reads them,
  // so that no store of its own is outstanding when it starts polling
  const int nslot = 2 * jj + 3;
  for (int k = kp_tid(); k < nslot; k += kThreads) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += sacc[w * kKStride + k];
    if (own)
      own[k] = s;
    else
      cstore(prow + k, s);
  }
  if constexpr (KEEP) {
    double2* kp = reinterpret_cast<double2*>(hl);
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      if constexpr (!XL) kp[r * kThreads + kp_tid()] = kx[r];
      kp[(kR + r) * kThreads + kp_tid()] = kw[r];
    }
  }
}

// ---- basis update (Algorithm 4: projection and normalisation) --------------
// coef: the published coefficients (coherent global memory).
// x_{j+1} = coef[jj+1] * w + sum_{i<=jj} coef[i] x_i, in place over column jj+1
// (which holds w); the halo rows and the tail are published.  With want_norm,
// partial slot 0 = ||x_{j+1}||^2 (the exact norm of the newest vector, needed
// only when the Arnoldi process closes).  Columns are visited from the newest
// to the oldest, so the ones the previous matvec pass read last come first.
template <typename TB>
// kxw: the pairs of x_jj and w the matvec pass of the previous phase left in
// LDS (matvec_dots_pass with KEEP), or null: they are then read from the
// basis.  Either way the columns enter in the same order (w, x_jj, ..., x_0).
// With kxw each thread also leaves its pairs of the new vector in the slots of
// x_jj (its own slots, so no barrier is needed), where the next matvec pass
// reads them.
__device__ __attribute__((always_inline)) inline void update_pass(const Args& a, int jj, const double* coef, double* red,
                                   bool want_norm, double* kxw) {
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const double cw = cload(coef + jj + 1);
  const Rows o = own_rows(a);
  double ss = 0.0;
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * kR) {
      const int64_t t0 = 2 * q0;
      uint32_t lo[kR];
      bool ok[kR];
      tile_pairs(q0, pend, lo, ok);
      double2 acc[kR];
      int i1 = jj;
      if (kxw) {
        const double2* kp = reinterpret_cast<const double2*>(kxw);
        const double cx = cload(coef + jj);
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          const double2 w = kp[(kR + r) * kThreads + kp_tid()];
          const double2 x = kp[r * kThreads + kp_tid()];
          acc[r] = make_double2(__builtin_fma(cx, x.x, cw * w.x), __builtin_fma(cx, x.y, cw * w.y));
        }
        i1 = jj - 1;
      } else {
#pragma unroll
        for (int r = 0; r < kR; ++r) {
          const double2 w = Pair<TB>::load(wcol + t0 + lo[r]);
          acc[r] = make_double2(cw * w.x, cw * w.y);
        }
      }
      for (; i1 >= 0; i1 -= kCuOf<TB>)
        axpy_cols<TB, kCuOf<TB>>(V, ld, t0, i1, -1, min(kCuOf<TB>, i1 + 1), coef, lo, acc);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const double y0 = rnd<TB>(acc[r].x), y1 = rnd<TB>(acc[r].y);
        if (ok[r]) {
          if (kxw) reinterpret_cast<double2*>(kxw)[r * kThreads + kp_tid()] = make_double2(y0, y1);
          Pair<TB>::store(wcol + t0 + lo[r], y0, y1);
          ss += y0 * y0 + y1 * y1;
          publish_pair(a, sg, t0 + lo[r], y0, y1);
        }
      }
    }
  }
  if (wg_rank(a) == 0)
    ss += tail_combine_cols<TB, TB>(a, V, jj + 1, coef, jj + 1, cw, wcol, true);
  if (want_norm) {
    ss = block_sum(ss, red);
    if (kp_tid() == 0) cstore(a.part + (int64_t)wg_rank(a) * kKStride, ss);
  }
}

// ---- combine: u = sum_{i<m} coef[i] x_i  (= beta V_m F, eq. kryexp) ----------
// coef: the published coefficients (coherent global memory).  Also writes
// out = u_top when this is the last substep.
template <typename TB>
__device__ __attribute__((always_inline)) inline void combine_pass(const Args& a, int m, const double* coef, bool last) {
  const TB* V = reinterpret_cast<const TB*>(a.V);
  const int64_t ld = a.ld;
  const Rows o = own_rows(a);
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    double* const outp = out_plane(a, sg.plane) - (int64_t)sg.plane * a.npt_pad;
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * kR) {
      const int64_t t0 = 2 * q0;
      uint32_t lo[kR];
      bool ok[kR];
      tile_pairs(q0, pend, lo, ok);
      double2 acc[kR];
#pragma unroll
      for (int r = 0; r < kR; ++r) acc[r] = make_double2(0.0, 0.0);
      for (int i0 = 0; i0 < m; i0 += kCuOf<TB>)
        axpy_cols<TB, kCuOf<TB>>(V, ld, t0, i0, 1, min(kCuOf<TB>, m - i0), coef, lo, acc);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        if (ok[r]) {
          const int64_t e = t0 + lo[r];
          *reinterpret_cast<double2*>(a.u + e) = acc[r];
          if (!last) publish_pair(a, sg, e, acc[r].x, acc[r].y);
          if (last) {
            if (e < sg.end) outp[e] = acc[r].x;
            if (e + 1 < sg.end) outp[e + 1] = acc[r].y;
          }
        }
      }
    }
  }
  if (wg_rank(a) == 0) tail_combine_cols<TB, double>(a, V, m, coef, -1, 0.0, a.u, !last);
}

// ---- processes with one reduction per inner product (Algorithm 1) or per
// window (ioCGS, Section 2.3.1) ----------------------------------------------
//
// Step jj is a matvec phase (PH_MVEC) followed by projection phases (PH_PROJ),
// each ending in a grid-wide reduction of a few partial sums (the counted
// buffer).  Stored columns carry unit scales as in the hybrid path (x_i =
// column i, v_i = sigma_i x_i).  The matvec multiplies the unit vector
// v_jj = sigma_jj x_jj (sigma_jj published as Pub::xscale; at jj = 0 the
// state vector u itself, whose norm is not known yet), so every stored column
// has the size of A v and none grows with the step; the new column jj+1 is
// projected in place and the leader folds the scales into the coefficients.
constexpr int kMvSlots = 4;   // x.x, x.w, w.w, x_a.w

// Tail rows of the matvec of step jj (lane 0 of workgroup 0: at most kPMax
// entries): w_tail = K (xs x_tail), stored (x_tail too at the first step), and
// their share of the four products.
template <typename TB>
__device__ inline void tail_mvec(const Args& a, int jj, const Src<TB>& x, TB* V, int acol,
                                 double xs, double* sacc) {
  if (kp_tid() != 0) return;
  const int64_t T0 = a.tail_off, ld = a.ld;
  TB* xcol = V + (int64_t)jj * ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  double xx = 0.0, xw = 0.0, ww = 0.0, aw = 0.0;
  for (int k = 0; k < a.p; ++k) {
    const double xk = x(T0 + k);
    const double wk = rnd<TB>(tail_shift_in(a, k) ? xs * x(T0 + k + 1) : 0.0);
    wcol[T0 + k] = (TB)wk;
    if (jj == 0) xcol[T0 + k] = (TB)xk;
    xx += xk * xk;
    xw += xk * wk;
    ww += wk * wk;
    if (acol >= 0) aw += (double)V[(int64_t)acol * ld + T0 + k] * wk;
  }
  sacc[0] += xx;
  sacc[1] += xw;
  sacc[2] += ww;
  sacc[3] += aw;
}

// Matvec of step jj: w = Atilde (s x_jj) into column jj+1, s = Pub::xscale
// (1 at jj = 0, where x_0 = u is stored into column 0), and the partial sums
// x.x, x.w, w.w and, when acol >= 0, x_acol . w, written to this workgroup's
// row of the counted buffer.  sacc: kWaves * kMvSlots doubles of LDS; hl: the
// LDS halo copy.
template <typename TB, bool HL>
__device__ __attribute__((always_inline)) inline void mvec_pass(const Args& a, int jj, int acol,
                                                                double* sacc, double* hl) {
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  const int lane = kp_tid() & 63, wv = kp_tid() >> 6;
  const Rows o = own_rows(a);
  for (int k = kp_tid(); k < kWaves * kMvSlots; k += kThreads) sacc[k] = 0.0;
  if (HL) stage_halo<TB>(a, o, hl);
  const double inv_mu = cload(&a.pub->inv_mu);
  const double xs = jj == 0 ? 1.0 : cload(&a.pub->xscale);
  TB* xcol = V + (int64_t)jj * ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const TB* acp = V + (int64_t)(acol >= 0 ? acol : 0) * ld;
  const Src<TB> x{xcol, a.u, jj == 0};   // (the tail entries)
  const Col<TB> xc{xcol};
  if (jj == 0) copy_state<TB>(a, o, xcol);
  __syncthreads();
  double sxx = 0.0, sxw = 0.0, sww = 0.0, saw = 0.0;
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    const int toff = (a.tangent && sg.plane == 1) ? a.pb : 0;
    double tc[kPMax];
#pragma unroll
    for (int c = 0; c < kPMax; ++c)
      tc[c] = (c < a.pb) ? rnd<TB>(cload(a.tx + toff + c)) * inv_mu : 0.0;
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * kR) {
      const int64_t t0 = 2 * q0;
      uint32_t lo[kR];
      bool ok[kR];
      tile_pairs(q0, pend, lo, ok);
      double2 xv[kR], wv2[kR], av[kR];
      const TB* ac = uniform_ptr(acp + t0);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        xv[r] = xc.pair(t0 + lo[r]);
        av[r] = (acol >= 0) ? load_at(ac, lo[r] * (uint32_t)sizeof(TB)) : make_double2(0.0, 0.0);
      }
      aug_tile<TB, HL>(a, o, sg, xc, hl, t0, lo, tc, wv2);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        wv2[r].x = rnd<TB>(xs * wv2[r].x);
        wv2[r].y = rnd<TB>(xs * wv2[r].y);
        if (ok[r]) {
          Pair<TB>::store(wcol + t0 + lo[r], wv2[r].x, wv2[r].y);
          if (jj == 0) Pair<TB>::store(xcol + t0 + lo[r], xv[r].x, xv[r].y);
        } else {
          xv[r] = make_double2(0.0, 0.0);
          wv2[r] = make_double2(0.0, 0.0);
        }
        sxx = __builtin_fma(xv[r].y, xv[r].y, __builtin_fma(xv[r].x, xv[r].x, sxx));
        sxw = __builtin_fma(xv[r].y, wv2[r].y, __builtin_fma(xv[r].x, wv2[r].x, sxw));
        sww = __builtin_fma(wv2[r].y, wv2[r].y, __builtin_fma(wv2[r].x, wv2[r].x, sww));
        saw += av[r].x * wv2[r].x + av[r].y * wv2[r].y;
      }
    }
  }
  sxx = wave_sum(sxx);
  sxw = wave_sum(sxw);
  sww = wave_sum(sww);
  saw = wave_sum(saw);
  if (lane == 0) {
    sacc[wv * kMvSlots + 0] = sxx;
    sacc[wv * kMvSlots + 1] = sxw;
    sacc[wv * kMvSlots + 2] = sww;
    sacc[wv * kMvSlots + 3] = saw;
  }
  if (wg_rank(a) == 0) tail_mvec<TB>(a, jj, x, V, acol, xs, sacc);
  __syncthreads();
  if (kp_tid() < kMvSlots) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += sacc[w * kMvSlots + kp_tid()];
    cstore(a.part + (int64_t)wg_rank(a) * kKStride + kp_tid(), s);
  }
}

// Projection phase of step jj: column jj+1 (w) += sum_{c = ca..cb} coef[c]
// x_c in place, then the partial sum x_dcol . w (dcol >= 0) or, with
// want_norm, ||w||^2, in slot 0 of this workgroup's row of the counted
// buffer.  With want_norm the result is the next vector the matvec
// multiplies: its halo rows and tail are published.
template <typename TB>
__device__ __attribute__((always_inline)) inline void proj_pass(const Args& a, int jj, int ca, int cb,
                                                                const double* coef, int dcol,
                                                                bool want_norm, double* red) {
  TB* V = reinterpret_cast<TB*>(a.V);
  const int64_t ld = a.ld;
  TB* wcol = V + (int64_t)(jj + 1) * ld;
  const TB* dcp = V + (int64_t)(dcol >= 0 ? dcol : 0) * ld;
  const Rows o = own_rows(a);
  double ss = 0.0;
  const int ns = num_segs(a);
  for (int si = 0; si < ns; ++si) {
    const Seg sg = seg_at(a, o, si);
    const int64_t pend = (sg.end + 1) >> 1;
    for (int64_t q0 = sg.beg >> 1; q0 < pend; q0 += (int64_t)kThreads * kR) {
      const int64_t t0 = 2 * q0;
      uint32_t lo[kR];
      bool ok[kR];
      tile_pairs(q0, pend, lo, ok);
      double2 acc[kR], dv[kR];
      const TB* dc = uniform_ptr(dcp + t0);
      const TB* wc = uniform_ptr(wcol + t0);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        acc[r] = load_at(wc, lo[r] * (uint32_t)sizeof(TB));
        dv[r] = (dcol >= 0) ? load_at(dc, lo[r] * (uint32_t)sizeof(TB)) : make_double2(0.0, 0.0);
      }
      for (int c = ca; c <= cb; ++c) axpy_cols<TB, 1>(V, ld, t0, c, 1, 1, coef, lo, acc);
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const double y0 = rnd<TB>(acc[r].x), y1 = rnd<TB>(acc[r].y);
        if (ok[r]) {
          Pair<TB>::store(wcol + t0 + lo[r], y0, y1);
          if (want_norm) {
            ss += y0 * y0 + y1 * y1;
            publish_pair(a, sg, t0 + lo[r], y0, y1);
          } else {
            ss += dv[r].x * y0 + dv[r].y * y1;
          }
        }
      }
    }
  }
  if (wg_rank(a) == 0 && kp_tid() == 0) {
    // the tail (at most kPMax entries), in the order of the rows above
    const int64_t T0 = a.tail_off;
    for (int k = 0; k < a.p; ++k) {
      double y = (double)wcol[T0 + k];
      for (int c = ca; c <= cb; ++c) y += cload(coef + c) * (double)V[(int64_t)c * ld + T0 + k];
      y = rnd<TB>(y);
      wcol[T0 + k] = (TB)y;
      if (want_norm) {
        cstore(a.tx + k, y);
        ss += y * y;
      } else {
        ss += (double)dcp[T0 + k] * y;
      }
    }
  }
  ss = block_sum(ss, red);
  if (kp_tid() == 0) cstore(a.part + (int64_t)wg_rank(a) * kKStride, ss);
}

// ---- finish: out = u_top (or NaN when the input was not finite) -------------
__device__ __attribute__((always_inline)) inline void finish_pass(const Args& a, bool nonfinite) {
  const Rows o = own_rows(a);
  for (int si = 0; si < a.nplanes; ++si) {
    const Seg sg = seg_at(a, o, si);
    double* const outp = out_plane(a, sg.plane) - (int64_t)sg.plane * a.npt_pad;
    for (int64_t e = sg.beg + kp_tid(); e < sg.end; e += kThreads)
      outp[e] = nonfinite ? __builtin_nan("") : a.u[e];
  }
}

}  // namespace kp
