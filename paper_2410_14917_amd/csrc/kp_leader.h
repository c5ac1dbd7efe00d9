// Serial work at the grid-wide synchronisation points, done by workgroup 0
// (the leader) on O(m^2) data: reduction of the per-workgroup partials, the
// scalar step of the hybrid Arnoldi process, the norm epilogue of the update,
// the small exponential with the substep controller, and the bookkeeping of
// the combine.  The leader owns the State (plain accesses) and publishes what
// the other workgroups need in the Pub block (coherent stores).
#pragma once

#include "kp_expm.h"
#include "kp_internal.h"

namespace kp {

// dst[k] = sum over workgroups of part[w][k], k < nslot; fixed order.
// Thread (g, l) of kRg groups sums the slot pair (kb + 2l, kb + 2l + 1) over
// the workgroups w = g (mod kRg) with 16-byte coherent loads (buffer loads
// with the agent-scope coherence bit, as the 8-byte coherent loads carry;
// rows past nwg lie beyond the descriptor's range and read as zero), all
// issued before they are consumed: about one memory latency per round of
// 128 slots.  grp: LDS scratch of kRg * kKStride doubles.
constexpr int kRg = 8;
constexpr int kBufWord3 = 0x00020000;   // raw buffer descriptor, gfx9 family
constexpr int kCoherentAux = 16;        // sc1: agent-scope coherent load

__device__ inline double lo_double(unsigned x, unsigned y) {
  return __builtin_bit_cast(double, (unsigned long long)x | ((unsigned long long)y << 32));
}

__device__ __attribute__((always_inline)) inline void reduce_partials(const Args& a, int nslot, double* dst, double* grp) {
  constexpr int kP = kThreads / kRg;   // slot pairs per round
  constexpr int kQ = 32;               // workgroups per thread per pass
  const int g = kp_tid() / kP, l = kp_tid() % kP;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      a.part, (short)0, a.nwg * kKStride * (int)sizeof(double), kBufWord3);
  for (int kb = 0; kb < nslot; kb += 2 * kP) {
    const int k = kb + 2 * l;
    if (k < nslot) {
      double sx = 0.0, sy = 0.0;
      for (int w0 = 0; w0 < a.nwg; w0 += kQ * kRg) {
        decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0)) v[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const int w = w0 + g + kRg * q;
          v[q] = __builtin_amdgcn_raw_buffer_load_b128(
              rs, (w * kKStride + k) * (int)sizeof(double), 0, kCoherentAux);
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          sx += lo_double(v[q][0], v[q][1]);
          sy += lo_double(v[q][2], v[q][3]);
        }
      }
      grp[g * kKStride + k] = sx;
      grp[g * kKStride + k + 1] = sy;
    }
  }
  __syncthreads();
  for (int k = kp_tid(); k < nslot; k += kThreads) {
    double s = 0.0;
#pragma unroll
    for (int gg = 0; gg < kRg; ++gg) s += grp[gg * kKStride + k];
    dst[k] = s;
  }
  __syncthreads();
}

// The same reduction for an Arnoldi step, read from the step buffer buf
// without a preceding count of arrivals: each thread reloads its kQ slot
// pairs until none holds kPartEmpty (the second half of a pair past nslot is
// never written and not checked), so the data are taken in the load that
// first sees them.  Row 0 (the leader's own sums) comes from the LDS copy
// own instead of the buffer.  The sums are formed in reduce_partials' order,
// so the result is the same to the bit.  *ok (LDS, 1 on entry) is cleared
// when the wait gives up (the abort flag is then raised).
__device__ __attribute__((always_inline)) inline void gather_step_partials(const Args& a, const double* buf, int nslot,
                                                            const double* own, double* dst, double* grp,
                                                            int* ok) {
  constexpr int kP = kThreads / kRg;
  constexpr int kQ = 32;
  constexpr unsigned kEmptyLo = (unsigned)kPartEmpty, kEmptyHi = (unsigned)(kPartEmpty >> 32);
  const int g = kp_tid() / kP, l = kp_tid() % kP;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(buf), (short)0, a.nwg * kKStride * (int)sizeof(double), kBufWord3);
  __syncthreads();   // grp reuses the LDS of the streaming pass's per-wave sums
  for (int kb = 0; kb < nslot; kb += 2 * kP) {
    const int k = kb + 2 * l;
    if (k < nslot) {
      const bool second = k + 1 < nslot;
      double sx = 0.0, sy = 0.0;
      for (int w0 = 0; w0 < a.nwg; w0 += kQ * kRg) {
        decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0)) v[kQ];
        int64_t t0 = 0;
        for (unsigned it = 0;; ++it) {
#pragma unroll
          for (int q = 0; q < kQ; ++q) {
            const int w = w0 + g + kRg * q;
            v[q] = __builtin_amdgcn_raw_buffer_load_b128(
                rs, (w * kKStride + k) * (int)sizeof(double), 0, kCoherentAux);
          }
          if (w0 == 0 && g == 0) {     // row 0: the leader's own sums
            const double o0 = own[k], o1 = second ? own[k + 1] : 0.0;
            v[0][0] = (unsigned)__double_as_longlong(o0);
            v[0][1] = (unsigned)((unsigned long long)__double_as_longlong(o0) >> 32);
            v[0][2] = (unsigned)__double_as_longlong(o1);
            v[0][3] = (unsigned)((unsigned long long)__double_as_longlong(o1) >> 32);
          }
          bool empty = false;
#pragma unroll
          for (int q = 0; q < kQ; ++q)
            empty |= (v[q][0] == kEmptyLo && v[q][1] == kEmptyHi) ||
                     (second && v[q][2] == kEmptyLo && v[q][3] == kEmptyHi);
          if (!empty) break;
          if (it == 0) t0 = wall_clock64();
          __builtin_amdgcn_s_sleep(1);
          if ((it & 15u) == 15u && (aborted(a) || wait_expired(a, t0))) {
            *ok = 0;
            break;
          }
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          sx += lo_double(v[q][0], v[q][1]);
          sy += lo_double(v[q][2], v[q][3]);
        }
      }
      grp[g * kKStride + k] = sx;
      grp[g * kKStride + k + 1] = sy;
    }
  }
  __syncthreads();
  for (int k = kp_tid(); k < nslot; k += kThreads) {
    double s = 0.0;
#pragma unroll
    for (int gg = 0; gg < kRg; ++gg) s += grp[gg * kKStride + k];
    dst[k] = s;
  }
  __syncthreads();
}

// First phase of an Arnoldi step for the configured process.
__device__ inline int step_phase(const Args& a) {
  return orth_multi_sync(a.orth) ? (int)PH_MVEC : (int)PH_STEP;
}

// ---- stage leader: balance mu, augmented tail, first phase -----------------
__device__ __attribute__((always_inline)) inline void leader_stage(const Args& a, double* red, Ctl& nx) {
  double m0 = 0.0, m1 = 0.0;
  for (int w = kp_tid(); w < a.nwg; w += kThreads) {
    m0 = fmax(m0, cload(a.part + (int64_t)w * kKStride + 0));
    m1 = fmax(m1, cload(a.part + (int64_t)w * kKStride + 1));
  }
  const double mx = block_max(m0, red);
  const double bad = block_max(m1, red);
  double mu = 1.0;
  if (a.pb > 0 && mx > 0.0 && isfinite(mx)) {
    int e;
    frexp(mx, &e);
    mu = ldexp(1.0, e - 1);            // largest power of two <= max |b_k|
  }
  for (int k = kp_tid(); k < kTailPad; k += kThreads) {
    const double v = (a.pb > 0 && k == a.p - 1) ? mu : 0.0;   // e_p of the (c) tail
    a.u[a.tail_off + k] = v;
    cstore(a.tx + k, v);
  }
  if (kp_tid() == 0) {
    State* st = a.st;
    Pub* pb = a.pub;
    st->mu = mu;
    cstore(&pb->inv_mu, 1.0 / mu);
    if (bad != 0.0) {
      nx.status = (int)KP_STATUS_NONFINITE;
      nx.phase = (int)PH_FINISH;
    } else if (a.h == 0.0) {
      nx.phase = (int)PH_FINISH;
    } else {
      nx.j = 0;
      nx.upd = 0;
      nx.phase = step_phase(a);
    }
  }
}

// ---- scalar step of Algorithm 4 --------------------------------------------
// The leader keeps what its serial work reads in LDS for the whole launch
// (loaded once by load_tables, updated as it changes, and mirrored in the
// State for the host and for later launches): the correction matrices, with
// element (row r, column k) of M^{-1} = (I + L)^{-1} / of L at
// Mi[k * kTabLd + r] / Li[k * kTabLd + r], the unit scales sigma, the divisors
// gamma, the squared norms ||A u_j||^2, and three controller flags.
constexpr int kTabLd = kMMax + 1;

struct LeadLds {
  double Mi[kMMax * kTabLd];
  double Li[kMMax * kTabLd];
  double sigma[kMMax + 8];
  double gamma[kMMax + 8];
  double wn2[kMMax + 8];
  int fallback_cur, m_target, breakdown, n_fallback, arnoldi_steps, onchip;
};

__device__ inline void load_tables(const Args& a, LeadLds& L) {
  const State* st = a.st;
  for (int idx = kp_tid(); idx < kMMax * kMMax; idx += kThreads) {
    const int k = idx / kMMax, r = idx - k * kMMax;
    L.Mi[k * kTabLd + r] = st->Minv[(int64_t)k * kLdt + r];
    L.Li[k * kTabLd + r] = st->Lm[(int64_t)k * kLdt + r];
  }
  for (int i = kp_tid(); i < kMMax + 2; i += kThreads) {
    L.sigma[i] = st->sigma[i];
    L.gamma[i] = st->gamma[i];
    L.wn2[i] = st->wn2[i];
  }
  if (kp_tid() == 0) {
    L.fallback_cur = st->fallback_cur;
    L.m_target = st->m_target;
    L.breakdown = st->breakdown;
    L.n_fallback = st->n_fallback;
    L.arnoldi_steps = st->arnoldi_steps;
    L.onchip = st->onchip;
  }
  __syncthreads();
}

// Work arrays of the scalar step in LDS (doubles): L row, b, y, p, H column.
constexpr int kWkL = 0, kWkB = 72, kWkY = 144, kWkP = 216, kWkH = 288;
constexpr int kWkDoubles = kWkH + 72;

// Row r = 8 * wave + lane / 8 of a product of a correction-matrix table with
// v (LDS): sum over k in K(r) of T(r, k) * v[k].  The 8 lanes of the row take
// k = lane mod 8, 8, 16, ... up to hi (loads in flight together, in bounds
// for every r, k < kMMax) and their sums meet by DPP inside the 8-lane group,
// so a product needs no workgroup barrier of its own; every lane of the group
// gets the row's value.  T(r, k) = tab[k * kTabLd + r] (TR = false) or
// tab[r * kTabLd + k] (TR = true, the transposed table).  MODE selects K(r),
// always within k <= hi (the rows used are r <= hi): 0 -> k <= r, 1 -> k < r,
// 2 -> r < k.
template <int MODE, bool TR>
__device__ inline double row_mv(int hi, const double* tab, const double* v, int r) {
  const int s = kp_tid() & 7;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < kMMax / 8; ++t) {
    if (8 * t > hi) break;                     // uniform: no row needs these k
    const int k = s + 8 * t;
    const double x = (TR ? tab[r * kTabLd + k] : tab[k * kTabLd + r]) * v[k];
    const bool in = (k <= hi) && ((MODE == 0) ? (k <= r) : (MODE == 1 ? (k < r) : (k > r)));
    if (in) acc += x;
  }
  acc += dpp_mov<0xB1>(acc);    // quad_perm [1,0,3,2]
  acc += dpp_mov<0x4E>(acc);    // quad_perm [2,3,0,1]
  acc += dpp_mov<0x141>(acc);   // row_half_mirror: the 8-lane sum
  return acc;
}

// tv: reduced inner products of step jj (slot layout of matvec_dots_pass).
// Stored columns x_i carry unit scales sigma_i (u_i = sigma_i x_i); x_j is the
// vector the matvec multiplied, so alpha = ||x_j|| is the lagged true norm and
// H_{j,j-1} = gamma_{j-1} alpha (gamma = divisor applied to x_j when written).
// Every thread of the workgroup calls this; wave 0 holds row i = lane.
__device__ __attribute__((always_inline)) inline void scalar_step(const Args& a, int jj, const double* tv, LeadLds& L,
                                   double* wk, Ctl& nx) {
  State* st = a.st;
  Pub* pb = a.pub;
  double* Mi = L.Mi;
  double* Li = L.Li;
  double* sg = L.sigma;
  double* sl = wk + kWkL;
  double* sb = wk + kWkB;
  double* sy = wk + kWkY;
  double* sp = wk + kWkP;
  double* sh = wk + kWkH;
  const int i = kp_tid();               // row index in wave 0
  const bool w0 = kp_tid() < 64;
  const double gj = tv[2 * jj], cj = tv[2 * jj + 1], cww = tv[2 * jj + 2];
  const double alpha = sqrt(gj);
  if (!(alpha > 0.0) || !isfinite(alpha) || !isfinite(cww)) {
    if (i == 0) {
      if (jj == 0 && alpha == 0.0) {        // zero start vector: result is zero
        st->zero = 1;
        st->beta = 0.0;
        nx.phase = (int)PH_FINISH;
      } else if (alpha == 0.0) {            // exact invariance already reached
        st->breakdown = 1;
        L.breakdown = 1;
        nx.m_eff = jj;
        nx.upd = 0;
        st->H[(int64_t)(jj - 1) * kLdh + jj] = 0.0;
        nx.phase = (int)PH_EXPM;
      } else {
        nx.status = (int)KP_STATUS_NONFINITE;
        nx.phase = (int)PH_FINISH;
      }
    }
    return;
  }
  if (jj > 0 && L.fallback_cur && alpha <= a.eps_bd * sqrt(L.wn2[jj - 1])) {
    // the exact norm of the vector produced with the fallback is negligible:
    // lucky breakdown at the previous step (this step's products are unused)
    if (i == 0) {
      st->breakdown = 1;
      L.breakdown = 1;
      st->H[(int64_t)(jj - 1) * kLdh + jj] = 0.0;
      nx.j = jj;
      nx.m_eff = jj;
      nx.upd = 0;
      nx.phase = (int)PH_EXPM;
    }
    return;
  }
  const double sj = 1.0 / alpha;
  const bool act = w0 && i < jj;
  const double sig = act ? sg[i] : (i == jj ? sj : 0.0);
  const double l = act ? sig * tv[2 * i] * sj : 0.0;                 // L_{j,i}
  const double b = act ? sig * tv[2 * i + 1] * sj : (i == jj ? cj * sj * sj : 0.0);
  const double wn2 = cww * sj * sj;
  if (w0) {
    sl[i] = l;
    sb[i] = b;
  }
  __syncthreads();
  // rows of the triangular products: 8 per wave, 8 lanes per row
  const int r = (kp_tid() >> 6) * 8 + ((kp_tid() & 63) >> 3);
  const bool row_lead = (kp_tid() & 7) == 0;
  // new row of M^{-1} = (I + L)^{-1} by the compact-WY recursion:
  // (M^{-1})_{j,r} = -sum_{r <= k < j} L_{j,k} (M^{-1})_{k,r}; the row is
  // appended to the LDS tables together with the new row of L (row_mv<2>
  // excludes k == r: the unit-diagonal term L_{j,r} * 1 is added here)
  const double mr = -row_mv<2, true>(jj - 1, Mi, sl, r);
  if (row_lead) {
    if (r < jj) {
      Mi[r * kTabLd + jj] = mr - sl[r];
      Li[r * kTabLd + jj] = sl[r];
    } else if (r == jj) {
      Mi[jj * kTabLd + jj] = 1.0;
      Li[jj * kTabLd + jj] = 0.0;
    }
  }
  __syncthreads();
  double Hr;
  if (a.orth == KP_ORTH_H_NCWY) {
    // T = I - L:  H = b - L b
    Hr = sb[r] - row_mv<1, false>(jj, Li, sb, r);
  } else {
    // y = M^{-1} b  (CWY: H = y)
    const double y = row_mv<0, false>(jj, Mi, sb, r);
    if (a.orth == KP_ORTH_H_CWY) {
      Hr = y;
    } else {
      // GSMGS: p = b + N y = b - L^T y, then x = M^{-1} p with the explicit
      // inverse kept above (the same x as the forward substitution M x = p)
      if (row_lead) sy[r] = y;
      __syncthreads();
      const double pv = sb[r] - row_mv<2, true>(jj, Li, sy, r);
      if (row_lead) sp[r] = pv;
      __syncthreads();
      Hr = row_mv<0, false>(jj, Mi, sp, r);
    }
  }
  if (row_lead) sh[r] = Hr;
  __syncthreads();
  double Hi = sh[i & 63];
  if (!w0) return;
  if (i > jj) Hi = 0.0;
  const double ss = wave_sum((i <= jj) ? b * b : 0.0);
  const double est2 = wn2 - ss;
  const int fallback = (est2 <= a.delta * wn2) ? 1 : 0;
  const double gam = fallback ? 1.0 : sqrt(est2);
  const int bd = (!fallback && gam <= a.eps_bd * sqrt(wn2)) ? 1 : 0;
  const bool bad = !isfinite(wave_sum(Hi));
  // write back: correction-matrix rows, H column, update coefficients
  if (act) {
    st->Lm[(int64_t)i * kLdt + jj] = l;
    st->Minv[(int64_t)i * kLdt + jj] = Mi[i * kTabLd + jj];
  }
  if (i <= jj) {
    st->H[(int64_t)jj * kLdh + i] = Hi;
    cstore(&pb->coef[i], -Hi * sig / gam);
  }
  if (i == 0) {
    sg[jj] = sj;
    st->Minv[(int64_t)jj * kLdt + jj] = 1.0;
    cstore(&pb->coef[jj + 1], sj / gam);
    st->sigma[jj] = sj;
    st->gamma[jj] = gam;
    st->wn2[jj] = wn2;
    L.gamma[jj] = gam;
    L.wn2[jj] = wn2;
    if (jj > 0) st->H[(int64_t)(jj - 1) * kLdh + jj] = L.gamma[jj - 1] * alpha;
    if (jj == 0) st->beta = alpha;
    st->fallback_cur = fallback;
    L.fallback_cur = fallback;
    L.n_fallback += fallback;
    st->n_fallback = L.n_fallback;
    if (bad) {
      nx.status = (int)KP_STATUS_NONFINITE;
      nx.phase = (int)PH_FINISH;
    } else if (bd) {
      st->H[(int64_t)jj * kLdh + jj + 1] = 0.0;
      st->breakdown = 1;
      L.breakdown = 1;
      st->arnoldi_steps = ++L.arnoldi_steps;
      nx.j = jj + 1;
      nx.m_eff = jj + 1;
      nx.upd = 0;
      nx.phase = (int)PH_EXPM;
    } else {
      const int j = jj + 1;
      st->arnoldi_steps = ++L.arnoldi_steps;
      nx.j = j;
      nx.m_eff = j;
      nx.upd = 1;
      nx.phase = (int)((j >= L.m_target || j >= a.stop_j) ? PH_CLOSE : PH_STEP);
    }
  }
}

// ---- close of the Arnoldi process: exact norm of the newest vector ---------
// After the pending update produced x_j (j = completed steps), its exact norm
// gives the last subdiagonal H_{j+1,j} = gamma_{j-1} ||x_j|| (the final
// reduction of Algorithm 4).
__device__ __attribute__((always_inline)) inline void leader_close(const Args& a, double nrm2, LeadLds& L,
                                                                  Ctl& nx) {
  if (kp_tid() != 0) return;
  State* st = a.st;
  const int j = nx.j;
  const double nrm = sqrt(nrm2);
  st->H[(int64_t)(j - 1) * kLdh + j] = L.gamma[j - 1] * nrm;
  st->last_nrm2 = nrm2;
  nx.upd = 0;
  if (!isfinite(nrm2)) {
    nx.status = (int)KP_STATUS_NONFINITE;
    nx.phase = (int)PH_FINISH;
    return;
  }
  if (L.fallback_cur && nrm <= a.eps_bd * sqrt(L.wn2[j - 1])) {
    st->H[(int64_t)(j - 1) * kLdh + j] = 0.0;
    st->breakdown = 1;
    L.breakdown = 1;
  }
  nx.phase = (int)((L.breakdown || j >= L.m_target) ? PH_EXPM : PH_STEP);
}

// ---- the leader of the processes with one reduction per inner product -----
// (Algorithm 1, MGS) or per window (ioCGS, Section 2.3.1).  Column i stores
// x_i with v_i = sigma_i x_i.  During step jj column jj+1 holds w / r with
// r = sigma_0 at jj = 0 (the matvec multiplied u = x_0 itself) and r = 1
// after (it multiplied v_jj), so an inner product v_i . w is
// sigma_i r (x_i . column), the projection w -= h v_i adds -h sigma_i / r x_i
// to the column, and ||w|| = r ||column||.

// After the matvec of step jj: tv = [x.x, x.w, w.w, x_acol.w].
__device__ inline void leader_mvec(const Args& a, int jj, const double* tv, LeadLds& L, Ctl& nx) {
  if (kp_tid() != 0) return;
  State* st = a.st;
  Pub* pb = a.pub;
  const double xx = tv[0], xw = tv[1], ww = tv[2], aw = tv[3];
  if (!isfinite(xx) || !isfinite(xw) || !isfinite(ww) || !isfinite(aw)) {
    nx.status = (int)KP_STATUS_NONFINITE;
    nx.phase = (int)PH_FINISH;
    return;
  }
  if (jj == 0) {
    const double beta = sqrt(xx);
    if (beta == 0.0) {                       // zero start vector: the result is zero
      st->zero = 1;
      st->beta = 0.0;
      nx.phase = (int)PH_FINISH;
      return;
    }
    st->beta = beta;
    L.sigma[0] = 1.0 / beta;
    st->sigma[0] = 1.0 / beta;
  }
  const double sj = L.sigma[jj];
  const double r = jj == 0 ? sj : 1.0;
  L.wn2[jj] = r * r * ww;                    // ||A v_jj||^2 (breakdown test)
  st->wn2[jj] = L.wn2[jj];
  double* Hc = st->H + (int64_t)jj * kLdh;
  if (a.orth == KP_ORTH_MGS) {
    // first inner product of Algorithm 1: h_{1,j} = v_1 . w
    const double s0 = L.sigma[0];
    const double h = s0 * r * (jj == 0 ? xw : aw);
    Hc[0] = h;
    cstore(&pb->coef[0], -h * s0 / r);
    nx.i = 1;                                // jj == 0: 1 = jj + 1, the norm
  } else {
    // ioCGS: both products of the window from the same w
    const double h = sj * r * xw;
    Hc[jj] = h;
    cstore(&pb->coef[jj], -h * sj / r);
    if (jj >= 1) {
      const double sa = L.sigma[jj - 1];
      const double ha = sa * r * aw;
      Hc[jj - 1] = ha;
      cstore(&pb->coef[jj - 1], -ha * sa / r);
    }
    nx.i = jj + 1;
  }
  nx.phase = (int)PH_PROJ;
}

// After projection phase i of step jj (s: the reduced slot 0).  i <= jj: the
// MGS inner product with v_i; i = jj + 1: the norm of the projected vector,
// which gives H_{j+1,j} and the unit scale of column jj+1.
__device__ inline void leader_proj(const Args& a, int jj, int i, double s, LeadLds& L, Ctl& nx) {
  if (kp_tid() != 0) return;
  State* st = a.st;
  Pub* pb = a.pub;
  if (!isfinite(s)) {
    nx.status = (int)KP_STATUS_NONFINITE;
    nx.phase = (int)PH_FINISH;
    return;
  }
  const double r = jj == 0 ? L.sigma[0] : 1.0;
  double* Hc = st->H + (int64_t)jj * kLdh;
  if (i <= jj) {
    const double si = L.sigma[i];
    const double h = si * r * s;
    Hc[i] = h;
    cstore(&pb->coef[i], -h * si / r);
    nx.i = i + 1;
    nx.phase = (int)PH_PROJ;
    return;
  }
  const double nw = sqrt(s);                 // || column jj+1 ||
  const double nrm = r * nw;                 // || projected w ||
  const int j = jj + 1;
  st->arnoldi_steps = ++L.arnoldi_steps;
  st->last_nrm2 = s;
  nx.j = j;
  nx.m_eff = j;
  nx.i = 0;
  nx.upd = 0;
  if (!(nrm > a.eps_bd * sqrt(L.wn2[jj]))) {  // lucky breakdown (also w = 0)
    Hc[j] = 0.0;
    st->breakdown = 1;
    L.breakdown = 1;
    nx.phase = (int)PH_EXPM;
    return;
  }
  Hc[j] = nrm;
  L.sigma[j] = 1.0 / nw;
  st->sigma[j] = 1.0 / nw;
  cstore(&pb->xscale, 1.0 / nw);             // the next matvec multiplies v_j
  nx.phase = (int)(j >= L.m_target ? PH_EXPM : PH_MVEC);
}

// ---- small exponential + substep controller (workgroup 0) -------------------
// The controller is this library's own (the paper defers it to KIOPS without
// printing the formulas): omega = err h / (tol beta tau), accept iff
// omega <= 1; on rejection double m (continuing the same Arnoldi process) while
// m < m_max, else shrink tau with the same basis; tau update factor
// clamp(0.9 omega^{-1/(q+1)}, 0.2, 4), q = ceil(m/4).
enum Decision : int { D_ACCEPT = 0, D_GROW = 1, D_SHRINK = 2, D_FAIL_NC = 3, D_FAIL_NF = 4 };

__device__ inline double tau_factor(double omega, int m) {
  if (omega == 0.0) return 4.0;
  const int q = (m + 3) / 4;
  return fmin(4.0, fmax(0.2, 0.9 * pow(omega, -1.0 / (double)(q + 1))));
}

// The proportional-integral law (KP_CTRL_PI) after an accepted substep whose
// predecessor was accepted with error omega_prev > 0: the integral gain 0.7
// and the proportional gain 0.4 (per q + 1) of Gustafsson's PI controller.
__device__ inline double tau_factor_pi(double omega, double omega_prev, int m) {
  if (omega == 0.0) return 4.0;
  const int q = (m + 3) / 4;
  const double f = 0.9 * pow(omega, -0.7 / (double)(q + 1)) * pow(omega_prev, 0.4 / (double)(q + 1));
  return fmin(4.0, fmax(0.2, f));
}

__device__ __attribute__((always_inline)) inline void expm_phase(const Args& a, double* lds, LeadLds& L,
                                                                Ctl& nx) {
  __shared__ int s_dec;
  __shared__ double s_tau;
  State* st = a.st;
  Pub* pb = a.pub;
  const bool fixed = a.fixed_m > 0;
  const int m = nx.m_eff;
  const bool happy = L.breakdown != 0;
  const double t = st->t, beta = st->beta;
  double tau = st->tau;
  if (happy && !fixed) tau = a.h - t;
  int dec = D_ACCEPT;
  while (true) {
    expm_hbar(a, st->H, kLdh, m, tau, happy, st->F, lds);
    if (kp_tid() == 0) {
      st->expm_evals += 1;
      const double err = happy ? 0.0 : beta * fabs(st->F[m]);
      double omega = 0.0;
      int d = D_ACCEPT;
      if (!fixed && !happy) {
        omega = err * a.h / (a.tol * beta * tau);
        if (!isfinite(omega)) {
          d = D_FAIL_NF;
        } else if (omega > 1.0) {
          st->rejected += 1;
          if (m < a.m_max) {
            d = D_GROW;
          } else {
            tau = tau * tau_factor(omega, m);
            d = (tau <= 1e-14 * a.h) ? D_FAIL_NC : D_SHRINK;
          }
        }
      }
      if (!isfinite(err)) d = D_FAIL_NF;
      st->err = err;
      st->omega = omega;
      s_dec = d;
      s_tau = tau;
    }
    __syncthreads();
    dec = s_dec;
    tau = s_tau;
    if (dec != D_SHRINK) break;
  }
  if (dec == D_ACCEPT) {
    for (int i = kp_tid(); i < m; i += kThreads)
      cstore(&pb->coef[i], beta * st->F[i] * st->sigma[i]);
    if (kp_tid() == 0) {
      st->tau = tau;
      const int last = fixed ? (st->substeps + 1 >= a.fixed_substeps) : (tau >= a.h - t);
      nx.last = last;
      nx.phase = (int)PH_COMBINE;
    }
  } else if (dec == D_GROW) {
    if (kp_tid() == 0) {
      st->m_cur = min(2 * st->m_cur, a.m_max);
      st->m_target = st->m_cur;
      L.m_target = st->m_cur;
      st->tau = tau;
      nx.upd = 0;
      nx.phase = step_phase(a);
    }
  } else {
    if (kp_tid() == 0) {
      nx.status = (int)((dec == D_FAIL_NF) ? KP_STATUS_NONFINITE : KP_STATUS_NOT_CONVERGED);
      nx.phase = (int)PH_FINISH;
    }
  }
  __syncthreads();
}

// ---- after the combine: advance time, next substep -------------------------
__device__ __attribute__((always_inline)) inline void leader_combine(const Args& a, LeadLds& L, Ctl& nx) {
  if (kp_tid() != 0) return;
  State* st = a.st;
  const bool fixed = a.fixed_m > 0;
  const int m = nx.m_eff;
  const double tau = st->tau;
  if (st->nlog < kLogMax) {
    st->log_tau[st->nlog] = tau;
    st->log_m[st->nlog] = m;
  }
  st->nlog += 1;
  st->err_max = fmax(st->err_max, st->err);
  st->substeps += 1;
  st->m_last = m;
  const bool last = nx.last != 0;
  st->t = last ? a.h : st->t + tau;
  if (L.breakdown) st->breakdowns += 1;
  if (last) {
    nx.phase = (int)PH_DONE;
    return;
  }
  double tn = tau;
  if (!fixed) {
    tn = tau * ((a.controller == KP_CTRL_PI && st->omega_prev > 0.0)
                    ? tau_factor_pi(st->omega, st->omega_prev, m)
                    : tau_factor(st->omega, m));
    st->omega_prev = st->omega;
    if (st->substeps >= a.max_substeps) {
      nx.status = (int)KP_STATUS_NOT_CONVERGED;
      nx.phase = (int)PH_FINISH;
      return;
    }
    tn = fmin(tn, a.h - st->t);
  }
  st->tau = tn;
  st->breakdown = 0;
  st->m_target = fixed ? a.fixed_m : st->m_cur;
  L.breakdown = 0;
  L.m_target = st->m_target;
  nx.j = 0;
  nx.upd = 0;
  nx.phase = step_phase(a);
}

}  // namespace kp
