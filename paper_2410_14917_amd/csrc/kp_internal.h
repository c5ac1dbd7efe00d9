// Internal definitions of libkrylov_phi: layouts, device state, kernel
// arguments, reductions and the grid-wide barrier.  gfx950 (CDNA4), wave64.
//
// Coherence model used throughout.  A workgroup of the persistent kernel stays
// on one CU for the whole launch, and the L2 caches of the XCDs are not kept
// coherent with each other inside a kernel: a plain store can sit in the
// writer's L2 for the rest of the launch.  Therefore no plain-stored data ever
// crosses workgroups inside a launch.  Each workgroup owns a range of grid
// rows (in every species plane) and reads/writes only its own elements with
// plain accesses; everything another workgroup needs -- the first and last row
// of the range (stencil halo), the augmented tail, partial sums and the
// published control block -- goes through agent-scope atomic stores and loads
// (cstore / cload), which write through to and read from the coherent level.
// The barrier itself is a pair of monotone counters updated with relaxed
// agent-scope atomics; no cache-wide fence is executed inside the hot loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krylov_phi.h"

namespace kp {

// threadIdx.x, re-read at every use (an opaque move), so that per-lane values
// derived from it are computed where they are used and are not hoisted out of
// the persistent kernel's phase loop (where they would stay live throughout).
__device__ __forceinline__ int kp_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

constexpr int kThreads = 512;             // threads per workgroup (one per CU)
constexpr int kWaves = kThreads / 64;
constexpr int kMMax = KP_MMAX;
constexpr int kPMax = KP_PMAX;
constexpr int kKStride = 2 * kMMax + 8;   // partial-sum slots per workgroup
// The partial-sum area holds three [part_rows][kKStride] buffers: buffer 0 for the
// phases whose arrivals are counted (stage, close), buffers 1 and 2 for the
// Arnoldi steps, alternating with the barrier number (see step_part).
constexpr int kPartBuffers = 3;
// Marks a step-buffer slot that has not been written since it was consumed:
// a signalling NaN, which no arithmetic produces (results are quiet NaNs).
constexpr unsigned long long kPartEmpty = 0xFFF4A5A5A5A5A5A5ull;
constexpr int kLdh = kMMax + 1;           // leading dimension of H in the state
constexpr int kLdt = kMMax;               // leading dimension of L, M^{-1}
constexpr int kLogMax = 8192;             // logged substeps
constexpr int kNmPad = 68;                // small-exponential matrices, padded
constexpr int kExSlots = 6;               // scratch matrices of the small exp
constexpr int kTailPad = 64;              // augmented tail region (>= KP_PMAX)
constexpr int kPlaneAlign = 128;          // plane offset alignment (elements)
// Two-species operators: the second plane starts kPlaneSkew elements past the
// rounded plane size, so that the two planes' elements at one grid point
// (which the joint matvec tiles read together) are not a power of two apart
// in memory (2048^2 planes otherwise sit exactly 2^22 elements apart; 17
// alignment units measured best of 9..129: 2.6 % on the 2 x 2048^2 call).
constexpr int kPlaneSkew = 17 * kPlaneAlign;

// Phases of one call (uniform across the grid).
enum Phase : int {
  PH_STAGE = 0,
  PH_STEP = 1,     // [pending update] + matvec + grouped dots + scalar step
  PH_CLOSE = 2,    // pending update + exact norm of the newest vector
  PH_EXPM = 3,
  PH_COMBINE = 4,
  PH_FINISH = 5,
  PH_DONE = 6,
  // the processes with one reduction per inner product (Algorithm 1) or per
  // window (ioCGS): a plain matvec with its first products, then projection
  // phases, each ending in a grid-wide reduction
  PH_MVEC = 7,     // w = Atilde x_j and the first inner products
  PH_PROJ = 8,     // w -= h_i x_i for the pending columns, then x_i' . w or ||w||^2
};

// Orthogonalisations that take one grid-wide reduction per inner product
// (MGS) or per window (ioCGS) run the PH_MVEC / PH_PROJ phases; the hybrid
// forms of Algorithm 4 run PH_STEP / PH_CLOSE.
__host__ __device__ inline bool orth_multi_sync(int orth) {
  return orth == KP_ORTH_MGS || orth == KP_ORTH_IOCGS;
}

constexpr int kFlagStride = 16;           // unsigned per workgroup flag (64 B)

// Control block published by the leader (rank 0) after every grid-wide sync
// and read by every workgroup of the problem with coherent loads.
struct Pub {
  int phase;
  int j;            // completed Arnoldi steps of the current substep
  int upd;          // the update producing x_j is still pending (PH_STEP/CLOSE)
  int m_eff;        // Krylov dimension available (combine uses it)
  int last;         // the accepted substep ends at h
  int status;
  int pad_[2];
  double inv_mu;
  double xscale;            // MGS / ioCGS: unit scale of the column the next matvec multiplies
  double coef[kMMax + 2];   // coefficients of the pending update / of the combine
};

// Private state of the call, read and written only by the leader (and by the
// host between launches).
struct State {
  int m_target;       // steps to reach before the small exponential
  int m_cur;          // current Krylov dimension choice of the controller
  int breakdown;      // lucky breakdown in this substep
  int fallback_cur;   // the exact norm replaced the estimate at the last step
  int substeps, rejected, arnoldi_steps, expm_evals, n_fallback, breakdowns;
  int nlog;
  int zero;           // the start vector is zero
  int m_last;
  int onchip;         // vector passes of the two-pass count kept in LDS (keep_xw)
  int pad_[2];
  double t, tau, beta, mu, err_max, omega, err, last_nrm2;
  double omega_prev;  // normalised error of the last accepted substep (PI control)
  double sigma[kMMax + 2];   // unit scale of stored basis column i
  double gamma[kMMax + 2];   // divisor applied to column i+1 when it was written
  double wn2[kMMax + 2];     // ||A u_j||^2 of step j
  double F[kNmPad];          // exp(tau Hbar) e_1
  double H[kLdh * kMMax];    // Hessenberg, column-major
  double Lm[kLdt * kMMax];   // L (strictly lower), column-major
  double Minv[kLdt * kMMax]; // (I + L)^{-1}, column-major
  double log_tau[kLogMax];
  int log_m[kLogMax];
};

// Arguments of the kernels (passed by value).
//
// Internal vector layout (length ld): plane s (s < nplanes) at s*npt_pad,
// row-major nx x ny inside the plane; the augmented tail (p entries) at
// tail_off; zero padding elsewhere.  The caller's B, fields and out use the
// plain layout (plane s at s*npt).  In tangent mode the vector is the pair
// [a; c] of two augmented vectors of a one-plane operator: plane 0 = a_top,
// plane 1 = c_top, tail = [a_tail (pb entries); c_tail (pb entries)]; both
// planes read B and the fields at the plain in-plane index.
struct Args {
  void* V;            // basis, ld x (m_max + 2), element type per basis_f32
  double* u;          // substep state vector, float64, length ld
  const double* B;    // caller layout, N x (p+1), column-major
  int64_t ldb;
  const double* f0;
  const double* f1;
  double* out;
  double* dout;       // tangent mode: the directional derivative (plane 0)
  double* part;       // [kPartBuffers][part_rows][kKStride] partial sums (coherent)
  unsigned* sync;     // [0] arrivals, [1] releases, [2] abort (coherent)
  State* st;          // the leader only
  Pub* pub;           // coherent
  double* ex;         // small-exponential scratch (the leader)
  double* hx;         // halo rows [nwg][nplanes][2][nx]      (coherent)
  double* tx;         // tail values [kTailPad]               (coherent)
  unsigned* flags;    // per-workgroup production counters, kFlagStride apart
  int64_t ld, npt_pad, tail_off;
  int N, p, npt, nx, ny, nplanes;   // p: tail length (2 pb in tangent mode)
  int pb;             // number of phi terms beyond b_0 (columns b_1..b_pb of B)
  int tangent;        // 1: Van Loan block operator [[Atilde, dAtilde], [0, Atilde]]
  int nwg, rows_per_wg;   // workgroups that own rows; rows per workgroup
  int part_rows;      // rows of each partial-sum buffer (>= nwg, the same for every team class)
  int nteam, wg0;     // workgroups meeting at the barriers (>= nwg); first workgroup of the run of such teams
  int kind, transpose;
  double cx, cy, cx2, cy2, adx, ady, react, ba, bb;
  double dcx, dcy, dadx, dady, dreact;   // tangent mode: the direction dA
  int orth, fixed_m, fixed_substeps, max_substeps, m_max;
  int controller;     // KP_CTRL_POWER or KP_CTRL_PI
  int m0;             // Krylov dimension of the first substep
  double tau0;        // length of the first substep
  int stop_j;         // pause when this many steps are completed (INT_MAX: never)
  int basis_f32;
  int halo_lds;       // the stencil halo rows fit the LDS copy of the matvec
  int keep_xw;        // one plane, one sub-tile per workgroup, one-reduction form: the
                      // matvec pass leaves x_j and w in LDS for the next update
#ifdef KP_TIMELINE
  long long* ts;      // device timeline (see KP_TS), null when not recording
  int ts_kmax;        // phases the timeline holds
#endif
  double inv_nx;      // 1 / nx (row of an in-plane index, corrected exactly)
  double h, tol, delta, eps_bd;
  int64_t wait_ticks; // bound of a grid-wide wait, steady-counter ticks
};

// Rank of this workgroup in the set that solves the problem: the whole grid
// for a single call (wg0 = 0, nteam = grid size); for a batched call, the
// teams of one size are consecutive runs of nteam workgroups from wg0.
// Rank 0 leads.
__device__ inline int wg_rank(const Args& a) {
  return (int)(((unsigned)blockIdx.x - (unsigned)a.wg0) % (unsigned)a.nteam);
}

// ---- coherent (agent-scope) accesses ---------------------------------------

template <typename T>
__device__ inline T cload(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void cstore(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- reductions ------------------------------------------------------------

template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ inline double readlane_d(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the 64 lanes of a wave, result in every lane.  Rows of 16 lanes are
// reduced with DPP (quad permutations, half-row and row mirrors); the four row
// sums are combined through readlane, in a fixed order.
__device__ inline double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum over the workgroup; every thread gets the result.  `red` holds kWaves
// doubles of LDS.  Deterministic (fixed order).
__device__ inline double block_sum(double v, double* red) {
  const int lane = kp_tid() & 63, wv = kp_tid() >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ inline double block_max(double v, double* red) {
  const int lane = kp_tid() & 63, wv = kp_tid() >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// ---- grid-wide synchronisation ---------------------------------------------
//
// Sync block (64 bytes): arrival counter (u32 word 0), release word (u64 at
// byte 8: barrier number in the high half, the packed control of the phase it
// opens in the low half), abort flag (u32 word 4).
//
// Barrier number k (counted identically by every workgroup): every workgroup
// increments the arrival counter; the leader (rank 0) waits until it reads
// k * nteam,
// does the serial work of the phase, and stores the release word (k, control);
// the others wait until they read k and take the control of the next phase
// from the same word.  Each wait is bounded by a.wait_ticks of the steady
// counter: past it the abort flag is raised and all workgroups leave their
// main loop, so a launch always ends.

constexpr int kSyncArrive = 0;
constexpr int kSyncAbort = 4;

// Control of one phase, uniform across the grid.
struct Ctl {
  int phase;
  int j;        // completed Arnoldi steps of the current substep
  int upd;      // the update producing x_j is still pending (PH_STEP/CLOSE)
  int m_eff;    // Krylov dimension available (small exponential, combine)
  int last;     // the accepted substep ends at h
  int status;
  int i;        // PH_PROJ: column of the next inner product (j + 1: the norm)
};

__device__ inline unsigned ctl_pack(const Ctl& c) {
  return (unsigned)c.phase | ((unsigned)c.j << 4) | ((unsigned)c.upd << 11) |
         ((unsigned)c.m_eff << 12) | ((unsigned)c.last << 19) | ((unsigned)c.status << 20) |
         ((unsigned)c.i << 22);
}
__device__ inline Ctl ctl_unpack(unsigned w) {
  Ctl c;
  c.phase = (int)(w & 15u);
  c.j = (int)((w >> 4) & 127u);
  c.upd = (int)((w >> 11) & 1u);
  c.m_eff = (int)((w >> 12) & 127u);
  c.last = (int)((w >> 19) & 1u);
  c.status = (int)((w >> 20) & 3u);
  c.i = (int)((w >> 22) & 127u);
  return c;
}

__device__ inline unsigned long long* release_word(const Args& a) {
  return reinterpret_cast<unsigned long long*>(a.sync + 2);
}

__device__ inline void wait_all_stores() { __builtin_amdgcn_s_waitcnt(0); }

// Device timeline, compiled in with KP_TIMELINE only (a separate build of the
// library): thread 0 of workgroup w < kTsWgs stores the 100 MHz constant clock
// at fixed points of phase k into ts[(k * kTsWgs + w) * kTsSlots + slot], at
// existing barriers, so the recording adds no synchronisation.  Slots: 0
// phase start; 1 update done and its stores complete; 2 neighbours' halo
// flags seen; 3 streaming part done; 4 release seen (workgroup 0: the phase
// code, phase * 1000 + j); 5 workgroup 0's reduction done; 6 its serial work
// done; 7 its release published.
constexpr int kTsSlots = 8, kTsWgs = 256;
#ifdef KP_TIMELINE
#define KP_TSV(a, k, slot, v)                                                             \
  do {                                                                                    \
    if ((a).ts && (int)(k) < (a).ts_kmax && wg_rank(a) < kTsWgs && kp_tid() == 0)         \
      (a).ts[((int64_t)(k) * kTsWgs + wg_rank(a)) * kTsSlots + (slot)] = (long long)(v);  \
  } while (0)
#define KP_TS(a, k, slot) KP_TSV(a, k, slot, wall_clock64())
#else
#define KP_TSV(a, k, slot, v) ((void)0)
#define KP_TS(a, k, slot) ((void)0)
#endif

__device__ inline bool aborted(const Args& a) { return cload(a.sync + kSyncAbort) != 0u; }

__device__ inline bool wait_expired(const Args& a, int64_t t0) {
  if (wall_clock64() - t0 > a.wait_ticks) {
    cstore(a.sync + kSyncAbort, 1u);
    return true;
  }
  return false;
}

// Spin until *ctr >= target (false: the launch is aborting).
__device__ inline bool spin_until(const Args& a, const unsigned* ctr, unsigned target) {
  if (cload(ctr) >= target) return true;
  const int64_t t0 = wall_clock64();
  for (unsigned it = 1;; ++it) {
    __builtin_amdgcn_s_sleep(1);          // back off: fewer polls of the shared line
    if (cload(ctr) >= target) return true;
    if ((it & 31u) == 0u && (aborted(a) || wait_expired(a, t0))) return false;
  }
}

__device__ inline void bar_arrive(const Args& a) {
  wait_all_stores();
  __syncthreads();
  if (kp_tid() == 0)
    __hip_atomic_fetch_add(a.sync + kSyncArrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrival at an Arnoldi-step barrier: the leader detects the data itself (the
// partial sums replace kPartEmpty in the step buffer), so nothing waits for
// this workgroup's stores; the count is kept so that the targets of the
// counted barriers stay k * nteam.
__device__ inline void bar_count(const Args& a) {
  if (kp_tid() == 0)
    __hip_atomic_fetch_add(a.sync + kSyncArrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Step buffer of barrier k ([part_rows][kKStride], rows < nwg used).  A workgroup resets its row of
// the buffer of barrier k + 1 to kPartEmpty at the start of phase k (the
// leader consumed that buffer at barrier k - 1, before releasing it), and the
// reset reaches the coherent level before any of its later stores does.
__device__ inline double* step_part(const Args& a, unsigned k) {
  return a.part + (int64_t)(1 + (int)(k & 1u)) * a.part_rows * kKStride;
}

// Leader: wait for every arrival at barrier k.  *ok (LDS) = false when
// the launch is aborting.
__device__ inline void bar_gather(const Args& a, unsigned k, int* ok) {
  if (kp_tid() == 0) *ok = spin_until(a, a.sync + kSyncArrive, k * (unsigned)a.nteam) ? 1 : 0;
  __syncthreads();
}

// Leader: open barrier k, announcing the control of the next phase,
// after its coherent stores completed.  The control is mirrored in the Pub
// block for the host.
__device__ inline void bar_release(const Args& a, unsigned k, const Ctl& nxt, Pub* pb) {
  wait_all_stores();
  __syncthreads();
  if (kp_tid() == 0) {
    cstore(&pb->phase, nxt.phase);
    cstore(&pb->j, nxt.j);
    cstore(&pb->upd, nxt.upd);
    cstore(&pb->m_eff, nxt.m_eff);
    cstore(&pb->last, nxt.last);
    cstore(&pb->status, nxt.status);
    cstore(release_word(a), ((unsigned long long)k << 32) | ctl_pack(nxt));
  }
}

// Other workgroups: wait for the release of barrier k and take the control of
// the next phase (cur, LDS); *ok = false when the launch is aborting.
__device__ inline void bar_wait(const Args& a, unsigned k, Ctl* cur, int* ok) {
  if (kp_tid() == 0) {
    unsigned long long* rw = release_word(a);
    unsigned long long w = cload(rw);
    int good = 1;
    if ((unsigned)(w >> 32) < k) {
      const int64_t t0 = wall_clock64();
      for (unsigned it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        w = cload(rw);
        if ((unsigned)(w >> 32) >= k) break;
        if ((it & 31u) == 0u && (aborted(a) || wait_expired(a, t0))) {
          good = 0;
          break;
        }
      }
    }
    *ok = good;
    if (good) *cur = ctl_unpack((unsigned)w);
  }
  __syncthreads();
}

// Point-to-point: this workgroup has published the halo rows / tail of the
// vector it produced in the phase of barrier k.
__device__ inline void flag_publish(const Args& a, unsigned k) {
  wait_all_stores();
  __syncthreads();
  KP_TS(a, k, 1);
  if (kp_tid() == 0) cstore(a.flags + (int64_t)wg_rank(a) * kFlagStride, k);
}

// Wait until the two row neighbours (halo) and workgroup 0 (tail) have
// published the vector of barrier k (the three flags are polled together).
__device__ inline void flag_wait_neighbours(const Args& a, unsigned k) {
  if (kp_tid() == 0) {
    const int b = wg_rank(a), nw = a.nwg;
    const unsigned* fp = a.flags + (int64_t)((b == 0) ? nw - 1 : b - 1) * kFlagStride;
    const unsigned* fn = a.flags + (int64_t)((b + 1 == nw) ? 0 : b + 1) * kFlagStride;
    const unsigned* f0 = a.flags;
    int64_t t0 = 0;
    for (unsigned it = 0;; ++it) {
      if (it) __builtin_amdgcn_s_sleep(1);
      const unsigned vp = cload(fp), vn = cload(fn), v0 = cload(f0);
      if (vp >= k && vn >= k && v0 >= k) break;
      if (it == 0) t0 = wall_clock64();
      if ((it & 31u) == 31u && (aborted(a) || wait_expired(a, t0))) break;
    }
  }
  __syncthreads();
  KP_TS(a, k, 2);
}

}  // namespace kp
