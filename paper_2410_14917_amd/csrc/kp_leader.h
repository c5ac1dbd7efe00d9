// Serial work of the grid-wide synchronisation points, done by one workgroup
// (the leader) on O(m^2) data: reduction of the per-workgroup partials, the
// scalar step of the hybrid Arnoldi process, the norm epilogue of the update,
// the small exponential with the substep controller, and the bookkeeping of
// the combine.
#pragma once

#include "kp_expm.h"
#include "kp_internal.h"

namespace kp {

// dst[k] = sum over workgroups of a.part[w][k], k < nslot; fixed order.
// grp: LDS scratch of 8 * kKStride doubles.
__device__ inline void reduce_partials(const Args& a, int nslot, double* dst,
                                       double* grp) {
  const int g = threadIdx.x >> 7, l = threadIdx.x & 127;   // 8 groups x 128
  for (int kb = 0; kb < nslot; kb += 128) {
    const int k = kb + l;
    if (k < nslot) {
      double s = 0.0;
      for (int w = g; w < a.nwg; w += 8) s += a.part[(int64_t)w * kKStride + k];
      grp[g * kKStride + k] = s;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nslot; k += kThreads) {
    double s = 0.0;
    for (int gg = 0; gg < 8; ++gg) s += grp[gg * kKStride + k];
    dst[k] = s;
  }
  __syncthreads();
}

__device__ inline void reduce_max2(const Args& a, double* mx, double* bad) {
  __shared__ double s_red[kWaves];
  double m0 = 0.0, m1 = 0.0;
  for (int w = threadIdx.x; w < a.nwg; w += kThreads) {
    m0 = fmax(m0, a.part[(int64_t)w * kKStride + 0]);
    m1 = fmax(m1, a.part[(int64_t)w * kKStride + 1]);
  }
  *mx = block_max(m0, s_red);
  *bad = block_max(m1, s_red);
}

// ---- stage leader: balance mu, augmented tail, first phase -----------------
__device__ inline void leader_stage(const Args& a) {
  double mx, bad;
  reduce_max2(a, &mx, &bad);
  if (threadIdx.x == 0) {
    State* st = a.st;
    double mu = 1.0;
    if (a.p > 0 && mx > 0.0 && isfinite(mx)) {
      int e;
      frexp(mx, &e);
      mu = ldexp(1.0, e - 1);          // largest power of two <= max |b_k|
    }
    st->mu = mu;
    st->inv_mu = 1.0 / mu;
    if (a.p > 0) a.u[a.N + a.p - 1] = mu;
    if (bad != 0.0) {
      st->status = KP_STATUS_NONFINITE;
      st->phase = PH_FINISH;
    } else if (a.h == 0.0) {
      st->phase = PH_FINISH;
    } else {
      st->phase = PH_STEP;
      st->sub = 0;
      st->j = 0;
    }
  }
}

// ---- scalar step of Algorithm 4 (one wave) ---------------------------------
// tv: reduced inner products of step jj (slot layout of matvec_dots_pass).
// Stored columns x_i carry unit scales sigma_i (u_i = sigma_i x_i); x_j is the
// vector the matvec multiplied, so alpha = ||x_j|| is the lagged true norm and
// H_{j,j-1} = gamma_{j-1} alpha (gamma = divisor applied to x_j when written).
__device__ inline void scalar_step(const Args& a, int jj, const double* tv) {
  if (threadIdx.x >= 64) return;
  State* st = a.st;
  const int i = threadIdx.x;               // lane = row index
  const double gj = tv[2 * jj], cj = tv[2 * jj + 1], cww = tv[2 * jj + 2];
  const double alpha = sqrt(gj);
  if (!(alpha > 0.0) || !isfinite(alpha) || !isfinite(cww)) {
    if (i == 0) {
      if (jj == 0 && alpha == 0.0) {        // zero start vector: result is zero
        st->zero = 1;
        st->beta = 0.0;
        st->phase = PH_FINISH;
      } else if (alpha == 0.0) {            // exact invariance already reached
        st->breakdown = 1;
        st->m_eff = jj;
        st->H[(int64_t)(jj - 1) * kLdh + jj] = 0.0;
        st->phase = PH_EXPM;
      } else {
        st->status = KP_STATUS_NONFINITE;
        st->phase = PH_FINISH;
      }
    }
    return;
  }
  const double sj = 1.0 / alpha;
  const bool act = i < jj;
  const double sig = act ? st->sigma[i] : (i == jj ? sj : 0.0);
  const double l = act ? sig * tv[2 * i] * sj : 0.0;                 // L_{j,i}
  const double b = act ? sig * tv[2 * i + 1] * sj : (i == jj ? cj * sj * sj : 0.0);
  const double wn2 = cww * sj * sj;
  // new row of M^{-1} = (I + L)^{-1} by the compact-WY recursion
  double mr = (i == jj) ? 1.0 : 0.0;
  for (int k = 0; k < jj; ++k) {
    const double lk = __shfl(l, k, 64);
    if (act && i <= k) mr -= lk * st->Minv[(int64_t)i * kLdt + k];
  }
  double Hi = 0.0;
  if (a.orth == KP_ORTH_H_NCWY) {
    // T = I - L:  H = b - L b
    double s = 0.0;
    for (int k = 0; k < jj; ++k) {
      const double bk = __shfl(b, k, 64);
      if (act && k < i) s += st->Lm[(int64_t)k * kLdt + i] * bk;
    }
    const double hj = b - wave_sum((i < jj) ? l * b : 0.0);
    Hi = act ? b - s : (i == jj ? hj : 0.0);
  } else {
    // y = M^{-1} b  (CWY: H = y)
    double y = 0.0;
    for (int k = 0; k < jj; ++k) {
      const double bk = __shfl(b, k, 64);
      if (act && k <= i) y += st->Minv[(int64_t)k * kLdt + i] * bk;
    }
    const double yj = wave_sum((i <= jj) ? mr * b : 0.0);
    if (i == jj) y = yj;
    if (a.orth == KP_ORTH_H_CWY) {
      Hi = (i <= jj) ? y : 0.0;
    } else {
      // GSMGS: p = b + N y = b - L^T y, then forward substitution (I + L) x = p
      double pv = b;
      for (int k = 0; k <= jj; ++k) {
        const double yk = __shfl(y, k, 64);
        if (i < k) {
          const double Lki = (k < jj) ? st->Lm[(int64_t)i * kLdt + k] : l;
          pv -= Lki * yk;
        }
      }
      double x = pv;
      for (int k = 0; k < jj; ++k) {
        const double xk = __shfl(x, k, 64);
        const double lk = __shfl(l, k, 64);
        if (i > k && i <= jj) {
          const double Lik = (i < jj) ? st->Lm[(int64_t)k * kLdt + i] : lk;
          x -= Lik * xk;
        }
      }
      Hi = (i <= jj) ? x : 0.0;
    }
  }
  const double ss = wave_sum((i <= jj) ? b * b : 0.0);
  const double est2 = wn2 - ss;
  const int fallback = (est2 <= a.delta * wn2) ? 1 : 0;
  const double gam = fallback ? 1.0 : sqrt(est2);
  const int bd = (!fallback && gam <= a.eps_bd * sqrt(wn2)) ? 1 : 0;
  const bool bad = !isfinite(wave_sum((i <= jj) ? Hi : 0.0));
  // write back: correction-matrix rows, H column, coefficients
  if (act) {
    st->Lm[(int64_t)i * kLdt + jj] = l;
    st->Minv[(int64_t)i * kLdt + jj] = mr;
  }
  if (i <= jj) {
    st->H[(int64_t)jj * kLdh + i] = Hi;
    st->coef[i] = -Hi * sig / gam;
  }
  if (i == 0) {
    st->Minv[(int64_t)jj * kLdt + jj] = 1.0;
    st->coef[jj + 1] = sj / gam;
    st->sigma[jj] = sj;
    st->gamma[jj] = gam;
    st->wn2[jj] = wn2;
    if (jj > 0) st->H[(int64_t)(jj - 1) * kLdh + jj] = st->gamma[jj - 1] * alpha;
    if (jj == 0) st->beta = alpha;
    st->fallback_cur = fallback;
    st->n_fallback += fallback;
    if (bad) {
      st->status = KP_STATUS_NONFINITE;
      st->phase = PH_FINISH;
    } else if (bd) {
      st->H[(int64_t)jj * kLdh + jj + 1] = 0.0;
      st->breakdown = 1;
      st->j = jj + 1;
      st->m_eff = jj + 1;
      st->arnoldi_steps += 1;
      st->phase = PH_EXPM;
    } else {
      st->sub = 1;
    }
  }
}

// ---- after the update pass: exact norm of x_{j+1} --------------------------
__device__ inline void leader_norm(const Args& a, int jj, double nrm2) {
  if (threadIdx.x != 0) return;
  State* st = a.st;
  const double nrm = sqrt(nrm2);
  st->H[(int64_t)jj * kLdh + jj + 1] = st->gamma[jj] * nrm;
  st->arnoldi_steps += 1;
  st->j = jj + 1;
  st->m_eff = jj + 1;
  st->sub = 0;
  st->last_nrm2 = nrm2;
  if (!isfinite(nrm2)) {
    st->status = KP_STATUS_NONFINITE;
    st->phase = PH_FINISH;
    return;
  }
  if (st->fallback_cur && nrm <= a.eps_bd * sqrt(st->wn2[jj])) {
    st->H[(int64_t)jj * kLdh + jj + 1] = 0.0;
    st->breakdown = 1;
    st->phase = PH_EXPM;
    return;
  }
  if (st->j >= st->m_target) st->phase = PH_EXPM;
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

__device__ inline void expm_phase(const Args& a, double* lds) {
  __shared__ int s_dec;
  __shared__ double s_tau;
  State* st = a.st;
  const bool fixed = a.fixed_m > 0;
  const int m = st->m_eff;
  const bool happy = st->breakdown != 0;
  const double t = st->t, beta = st->beta;
  double tau = st->tau;
  if (happy && !fixed) tau = a.h - t;
  int dec = D_ACCEPT;
  while (true) {
    expm_hbar(a, st->H, kLdh, m, tau, happy, st->F, lds);
    if (threadIdx.x == 0) {
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
    for (int i = threadIdx.x; i < m; i += kThreads) st->coef[i] = beta * st->F[i] * st->sigma[i];
    if (threadIdx.x == 0) {
      st->tau = tau;
      st->last_substep = fixed ? (st->substeps + 1 >= a.fixed_substeps) : (tau >= a.h - t);
      st->phase = PH_COMBINE;
    }
  } else if (dec == D_GROW) {
    if (threadIdx.x == 0) {
      st->m_cur = min(2 * st->m_cur, a.m_max);
      st->m_target = st->m_cur;
      st->tau = tau;
      st->sub = 0;
      st->phase = PH_STEP;
    }
  } else {
    if (threadIdx.x == 0) {
      st->status = (dec == D_FAIL_NF) ? KP_STATUS_NONFINITE : KP_STATUS_NOT_CONVERGED;
      st->phase = PH_FINISH;
    }
  }
  __syncthreads();
}

// ---- after the combine: advance time, next substep -------------------------
__device__ inline void leader_combine(const Args& a) {
  if (threadIdx.x != 0) return;
  State* st = a.st;
  const bool fixed = a.fixed_m > 0;
  const int m = st->m_eff;
  const double tau = st->tau;
  if (st->nlog < kLogMax) {
    st->log_tau[st->nlog] = tau;
    st->log_m[st->nlog] = m;
  }
  st->nlog += 1;
  st->err_max = fmax(st->err_max, st->err);
  st->substeps += 1;
  st->m_last = m;
  const bool last = st->last_substep != 0;
  st->t = last ? a.h : st->t + tau;
  if (st->breakdown) st->breakdowns += 1;
  if (last) {
    st->phase = PH_DONE;
    return;
  }
  double tn = tau;
  if (!fixed) {
    tn = tau * tau_factor(st->omega, m);
    if (st->substeps >= a.max_substeps) {
      st->status = KP_STATUS_NOT_CONVERGED;
      st->phase = PH_FINISH;
      return;
    }
    tn = fmin(tn, a.h - st->t);
  }
  st->tau = tn;
  st->j = 0;
  st->sub = 0;
  st->breakdown = 0;
  st->m_target = fixed ? a.fixed_m : st->m_cur;
  st->phase = PH_STEP;
}

}  // namespace kp
