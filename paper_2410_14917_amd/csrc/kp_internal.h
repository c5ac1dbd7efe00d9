// Internal definitions of libkrylov_phi: device state, kernel arguments,
// reductions and the grid-wide barrier.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krylov_phi.h"

namespace kp {

constexpr int kThreads = 1024;            // threads per workgroup, every kernel
constexpr int kWaves = kThreads / 64;
constexpr int kMMax = KP_MMAX;
constexpr int kPMax = KP_PMAX;
constexpr int kKStride = 2 * kMMax + 8;   // partial-sum slots per workgroup
constexpr int kLdh = kMMax + 1;           // leading dimension of H in the state
constexpr int kLdt = kMMax;               // leading dimension of L, M^{-1}
constexpr int kLogMax = 8192;             // logged substeps
constexpr int kNm = kMMax + 1;            // largest small-exponential size
constexpr int kNmPad = 68;                // padded to a multiple of 4
constexpr int kExSlots = 6;               // scratch matrices of the small exp

// Phases of one phi_combo call (uniform across the grid).
enum Phase : int {
  PH_STAGE = 0,
  PH_STEP = 1,
  PH_EXPM = 2,
  PH_COMBINE = 3,
  PH_FINISH = 4,
  PH_DONE = 5,
};

// State of the call in device memory.  Written only by the leader workgroup
// of a phase (the last workgroup to arrive at a reduction, or workgroup 0 for
// the small exponential); read by every workgroup after a grid-wide sync.
struct State {
  int phase;
  int sub;            // within PH_STEP: 0 = matvec+dots due, 1 = update due
  int status;
  int j;              // completed Arnoldi steps of the current substep
  int m_target;       // steps to reach before the small exponential
  int m_cur;          // current Krylov dimension choice of the controller
  int m_eff;          // Krylov dimension available (j, or breakdown size)
  int breakdown;      // lucky breakdown in this substep
  int fallback_cur;   // the exact norm replaces the estimate at step j
  int last_substep;   // the accepted substep ends at h
  int substeps, rejected, arnoldi_steps, expm_evals, n_fallback, breakdowns;
  int nlog;
  int zero;           // the start vector is zero
  int aborted;
  int m_last;
  int pad_[2];
  double t, tau, beta, mu, inv_mu, err_max, omega, err, last_nrm2;
  double sigma[kMMax + 2];   // unit scale of stored basis column i
  double gamma[kMMax + 2];   // divisor applied to column i+1 when it was written
  double wn2[kMMax + 2];     // ||A u_j||^2 of step j
  double coef[kMMax + 2];    // coefficients of the update / combination pass
  double F[kNmPad];          // exp(tau Hbar) e_1
  double tv[kKStride];       // reduced inner products of the current step
  double H[kLdh * kMMax];    // Hessenberg, column-major
  double Lm[kLdt * kMMax];   // L (strictly lower), column-major
  double Minv[kLdt * kMMax]; // (I + L)^{-1}, column-major
  double log_tau[kLogMax];
  int log_m[kLogMax];
};

// Arguments of every kernel (passed by value).
struct Args {
  void* V;            // basis, ld x (m_max + 2), element type per basis_f32
  double* u;          // substep state vector (length ld), float64
  const double* B;    // N x (p+1), column-major
  int64_t ldb;
  const double* f0;
  const double* f1;
  double* out;
  double* part;       // [nwg][kKStride] partial sums
  unsigned* sync;     // [0] arrivals, [1] generation, [2] abort
  State* st;
  double* ex;         // small-exponential scratch, kExSlots * kNmPad^2
  int64_t ld;         // leading dimension of V and u
  int N, L, p, npt, nx, ny;
  int nwg;
  int64_t ppw;        // element pairs per workgroup
  int64_t npairs;
  int kind, transpose;
  double cx, cy, cx2, cy2, adx, ady, react, ba, bb;
  int orth, fixed_m, fixed_substeps, max_substeps, m_max;
  int persistent;
  int basis_f32;
  int pad_;
  double h, tol, delta, eps_bd;
  int64_t wait_ticks;  // bound of a grid-wide wait, steady-counter ticks
};

// ---- reductions ------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum over the workgroup; every thread gets the result.  `red` holds kWaves
// doubles of LDS.  Deterministic (fixed order).
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s += red[w];
  return s;
}

__device__ inline double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) s = fmax(s, red[w]);
  return s;
}

// ---- grid synchronisation --------------------------------------------------
//
// Arrival at a grid-wide point.  Every workgroup has already written its
// partial results.  Thread 0 publishes them (release at agent scope) and takes
// a ticket; the workgroup holding the last ticket becomes the leader, sees all
// partials (acquire) and does the reduction and the serial work of the phase.
// In a persistent launch the other workgroups then wait for the leader's
// release; in per-phase kernels the kernel boundary is the release.

__device__ inline unsigned atomic_load_acq(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in every thread of the leader workgroup.
__device__ inline bool arrive(const Args& a, unsigned* gen0_out) {
  __shared__ int s_last;
  __shared__ unsigned s_gen;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned g = atomic_load_acq(a.sync + 1);
    __threadfence();
    unsigned prev = __hip_atomic_fetch_add(a.sync, 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    int last = (prev == (unsigned)(a.nwg - 1));
    if (last) __threadfence();
    s_last = last;
    s_gen = g;
  }
  __syncthreads();
  *gen0_out = s_gen;
  return s_last != 0;
}

// Called by the leader after its serial work: reset the ticket counter and
// (persistent launches) open the barrier.
__device__ inline void leader_release(const Args& a, unsigned gen0) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(a.sync, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    __hip_atomic_store(a.sync + 1, gen0 + 1u, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// Non-leaders of a persistent launch wait here.  The wait is bounded: after
// a.wait_ticks of the steady counter (a few seconds) without the generation
// moving, the abort flag is raised and every workgroup leaves its main loop at
// the next check.
__device__ inline void wait_release(const Args& a, unsigned gen0) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t t0 = wall_clock64();
    while (atomic_load_acq(a.sync + 1) == gen0) {
      if (atomic_load_acq(a.sync + 2) != 0u) break;
      __builtin_amdgcn_s_sleep(2);
      if (wall_clock64() - t0 > a.wait_ticks) {
        __hip_atomic_store(a.sync + 2, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}

__device__ inline bool aborted(const Args& a) {
  __shared__ int s_ab;
  __syncthreads();
  if (threadIdx.x == 0) s_ab = (atomic_load_acq(a.sync + 2) != 0u);
  __syncthreads();
  return s_ab != 0;
}

}  // namespace kp
