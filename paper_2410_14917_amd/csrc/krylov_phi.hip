// libkrylov_phi: kernels and the C ABI declared in include/krylov_phi.h.
//
// Execution model (one MI355X, gfx950):
//  * Every phase of a phi_combo call is a device function over the whole grid:
//    stage, Arnoldi step (matvec + grouped dots, then update + norm), small
//    exponential + controller, combine, finish.  The grid-wide reduction of a
//    step is the paper's single global synchronisation (Algorithm 4): each
//    workgroup writes partial sums, the last workgroup to arrive reduces them
//    and runs the serial O(m^2) work.
//  * KP_EXEC_PERSISTENT runs the whole call in ONE cooperative launch: the
//    workgroups loop over the phases recorded in device memory and meet at
//    grid barriers; the adaptive controller never returns to the host.
//  * KP_EXEC_STREAM enqueues one kernel per phase (the kernel boundary is the
//    barrier); it serves fixed schedules and the step-by-step test entry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "kp_internal.h"
#include "kp_leader.h"
#include "kp_passes.h"

namespace kp {

constexpr int kLdsDoubles = 2 * kNmPad * kNmPad;
static_assert(kWaves * kKStride + kKStride + 8 * kKStride + (kMMax + 8) + kWaves <= kLdsDoubles,
              "LDS carve-up exceeds the shared buffer");

struct Ctrl {
  int phase, sub, j, m_eff, last, status, abort_;
  double inv_mu;
};

__device__ inline void read_ctrl(const Args& a, Ctrl* c) {
  __syncthreads();
  if (threadIdx.x == 0) {
    State* st = a.st;
    c->phase = __hip_atomic_load(&st->phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c->sub = __hip_atomic_load(&st->sub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c->j = __hip_atomic_load(&st->j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c->m_eff = __hip_atomic_load(&st->m_eff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c->last = __hip_atomic_load(&st->last_substep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c->status = __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c->abort_ = (int)atomic_load_acq(a.sync + 2);
    c->inv_mu = st->inv_mu;
  }
  __syncthreads();
}

__device__ inline void sync_point(const Args& a, unsigned gen0, bool leader) {
  if (leader) {
    leader_release(a, gen0);
  } else if (a.persistent) {
    wait_release(a, gen0);
  }
}

template <typename TB>
__device__ void run_phase(const Args& a, double* lds, const Ctrl& c) {
  double* sacc = lds;
  double* tv = sacc + kWaves * kKStride;
  double* grp = tv + kKStride;
  double* coef = grp + 8 * kKStride;
  double* red = coef + (kMMax + 8);
  unsigned gen0 = 0;
  bool leader = false;
  switch (c.phase) {
    case PH_STAGE:
      stage_pass(a, red);
      leader = arrive(a, &gen0);
      if (leader) leader_stage(a);
      sync_point(a, gen0, leader);
      break;
    case PH_STEP:
      if (c.sub == 0) {
        matvec_dots_pass<TB>(a, c.j, c.inv_mu, sacc);
        leader = arrive(a, &gen0);
        if (leader) {
          reduce_partials(a, 2 * c.j + 3, tv, grp);
          scalar_step(a, c.j, tv);
        }
        sync_point(a, gen0, leader);
      } else {
        for (int k = threadIdx.x; k < c.j + 2; k += kThreads) coef[k] = a.st->coef[k];
        __syncthreads();
        update_pass<TB>(a, c.j, coef, red);
        leader = arrive(a, &gen0);
        if (leader) {
          reduce_partials(a, 1, tv, grp);
          leader_norm(a, c.j, tv[0]);
        }
        sync_point(a, gen0, leader);
      }
      break;
    case PH_EXPM:
      if (!a.persistent) {
        if (blockIdx.x == 0) expm_phase(a, lds);
        break;
      }
      if (blockIdx.x == 0) expm_phase(a, lds);
      leader = arrive(a, &gen0);
      sync_point(a, gen0, leader);
      break;
    case PH_COMBINE:
      for (int k = threadIdx.x; k < c.m_eff; k += kThreads) coef[k] = a.st->coef[k];
      __syncthreads();
      combine_pass<TB>(a, c.m_eff, coef, c.last != 0);
      leader = arrive(a, &gen0);
      if (leader) leader_combine(a);
      sync_point(a, gen0, leader);
      break;
    case PH_FINISH:
      finish_pass(a, c.status == KP_STATUS_NONFINITE);
      leader = arrive(a, &gen0);
      if (leader && threadIdx.x == 0) a.st->phase = PH_DONE;
      sync_point(a, gen0, leader);
      break;
    default:
      break;
  }
}

// Whole call in one cooperative launch.
template <typename TB>
__global__ __launch_bounds__(kThreads) void k_persistent(Args a) {
  __shared__ double lds[kLdsDoubles];
  __shared__ Ctrl c;
  for (;;) {
    read_ctrl(a, &c);
    if (c.phase == PH_DONE || c.abort_) break;
    run_phase<TB>(a, lds, c);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && atomic_load_acq(a.sync + 2) != 0u)
    a.st->status = KP_STATUS_ABORTED;
}

// One phase per launch; a launch whose phase is not due does nothing.
template <typename TB, int PH, int SUB>
__global__ __launch_bounds__(kThreads) void k_phase(Args a) {
  __shared__ double lds[kLdsDoubles];
  __shared__ Ctrl c;
  read_ctrl(a, &c);
  if (c.phase != PH) return;
  if (PH == PH_STEP && c.sub != SUB) return;
  run_phase<TB>(a, lds, c);
}

// Reset of the call state; the Hessenberg and correction matrices are zeroed
// so that entries outside their triangles read as zero.
__global__ __launch_bounds__(256) void k_init(Args a, int m_target) {
  State* st = a.st;
  for (int i = threadIdx.x; i < kLdh * kMMax; i += blockDim.x) st->H[i] = 0.0;
  for (int i = threadIdx.x; i < kLdt * kMMax; i += blockDim.x) {
    st->Lm[i] = 0.0;
    st->Minv[i] = 0.0;
  }
  if (threadIdx.x != 0) return;
  a.sync[0] = 0u;
  a.sync[1] = 0u;
  a.sync[2] = 0u;
  st->phase = PH_STAGE;
  st->sub = 0;
  st->status = KP_STATUS_OK;
  st->j = 0;
  st->m_target = m_target;
  st->m_cur = m_target;
  st->m_eff = 0;
  st->breakdown = 0;
  st->fallback_cur = 0;
  st->last_substep = 0;
  st->substeps = st->rejected = st->arnoldi_steps = st->expm_evals = 0;
  st->n_fallback = st->breakdowns = st->nlog = st->zero = st->aborted = 0;
  st->m_last = 0;
  st->t = 0.0;
  st->tau = (a.fixed_m > 0) ? a.h / (double)a.fixed_substeps : a.h;
  st->beta = 0.0;
  st->mu = 1.0;
  st->inv_mu = 1.0;
  st->err_max = st->omega = st->err = st->last_nrm2 = 0.0;
}

// Small exponential alone (test entry): F = exp(tau Hbar_m) e_1 from st->H.
__global__ __launch_bounds__(kThreads) void k_expm_test(Args a, int m, double tau) {
  __shared__ double lds[kLdsDoubles];
  expm_hbar(a, a.st->H, kLdh, m, tau, false, a.st->F, lds);
}

}  // namespace kp

// ============================================================================
// Host side
// ============================================================================

using kp::Args;
using kp::State;

struct kp_ctx {
  kp_config cfg;
  hipStream_t stream = nullptr;
  int device = 0;
  int ncu = 0;
  int64_t wait_ticks = 0;
  void* V = nullptr;
  size_t v_bytes = 0;
  double* u = nullptr;
  size_t u_bytes = 0;
  double* part = nullptr;
  size_t part_bytes = 0;
  unsigned* sync = nullptr;
  State* st = nullptr;
  double* ex = nullptr;
  int occ[2] = {-1, -1};
  Args last{};
  int have_begin = 0;
  char err[512] = {0};
};

namespace {

int hip_fail(kp_ctx* c, hipError_t e, const char* what) {
  if (c) snprintf(c->err, sizeof(c->err), "%s: %s", what, hipGetErrorString(e));
  return KP_EHIP;
}

#define KP_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);  \
  } while (0)

int check_config(const kp_config* c) {
  if (c->orth < 0 || c->orth > KP_ORTH_H_NCWY) return KP_EINVAL;
  if (c->basis_dtype != KP_BASIS_F64 && c->basis_dtype != KP_BASIS_F32) return KP_EINVAL;
  if (c->exec_mode != KP_EXEC_PERSISTENT && c->exec_mode != KP_EXEC_STREAM) return KP_EINVAL;
  if (c->max_substeps < 0 || c->fixed_m < 0 || c->fixed_m > KP_MMAX) return KP_EINVAL;
  if (c->fixed_m > 0 && c->fixed_substeps < 1) return KP_EINVAL;
  if (c->fixed_substeps < 0) return KP_EINVAL;
  if (!std::isfinite(c->fallback_delta) || !std::isfinite(c->breakdown_eps)) return KP_EINVAL;
  if (c->breakdown_eps < 0.0) return KP_EINVAL;
  return KP_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

// Validate the operator and problem; fill the problem part of Args.
// No HIP call happens here.
int build_args(const kp_ctx* ctx, const kp_op* A, const double* B, int p, int64_t ldb,
               double h, double tol, int m_max, double* out, bool need_out, Args* a) {
  if (!ctx || !A || !B) return KP_EINVAL;
  if (need_out && !out) return KP_EINVAL;
  if (A->kind < KP_OP_ADR || A->kind > KP_OP_BRUSSELATOR) return KP_EINVAL;
  if (A->nx < 1 || A->ny < 1) return KP_EINVAL;
  if (!(A->dx > 0.0) || !(A->dy > 0.0) || !std::isfinite(A->dx) || !std::isfinite(A->dy))
    return KP_EINVAL;
  const double coefs[] = {A->nu, A->nu2, A->ax, A->ay, A->react, A->brus_a, A->brus_b};
  for (double v : coefs)
    if (!std::isfinite(v)) return KP_EINVAL;
  if (A->kind == KP_OP_ALLEN_CAHN && !A->field0) return KP_EINVAL;
  if (A->kind == KP_OP_BRUSSELATOR && (!A->field0 || !A->field1)) return KP_EINVAL;
  const int64_t npt = (int64_t)A->nx * A->ny;
  const int64_t N = npt * (A->kind == KP_OP_BRUSSELATOR ? 2 : 1);
  if (N > (int64_t)1 << 30) return KP_EINVAL;
  if (p < 0 || p > KP_PMAX) return KP_EINVAL;
  if (ldb < N) return KP_EINVAL;
  if (m_max < 1 || m_max > KP_MMAX) return KP_EINVAL;
  if (!(h >= 0.0) || !std::isfinite(h)) return KP_EINVAL;
  const kp_config& cfg = ctx->cfg;
  if (cfg.fixed_m == 0 && !(tol > 0.0 && std::isfinite(tol))) return KP_EINVAL;
  if (cfg.fixed_m > m_max) return KP_EINVAL;
  if (need_out) {
    const size_t ob = (size_t)N * sizeof(double);
    const size_t bb = (size_t)ldb * (p + 1) * sizeof(double);
    if (overlaps(out, ob, B, bb)) return KP_EINVAL;
    if (overlaps(out, ob, A->field0, (size_t)npt * sizeof(double))) return KP_EINVAL;
    if (overlaps(out, ob, A->field1, (size_t)npt * sizeof(double))) return KP_EINVAL;
  }
  Args r{};
  r.B = B;
  r.ldb = ldb;
  r.f0 = A->field0;
  r.f1 = A->field1;
  r.out = out;
  r.N = (int)N;
  r.L = (int)(N + p);
  r.p = p;
  r.npt = (int)npt;
  r.nx = A->nx;
  r.ny = A->ny;
  r.ld = ((int64_t)r.L + 63) / 64 * 64;
  r.npairs = r.ld / 2;
  r.kind = A->kind;
  r.transpose = A->transpose ? 1 : 0;
  r.cx = A->nu / (A->dx * A->dx);
  r.cy = A->nu / (A->dy * A->dy);
  r.cx2 = A->nu2 / (A->dx * A->dx);
  r.cy2 = A->nu2 / (A->dy * A->dy);
  r.adx = A->ax / (2.0 * A->dx);
  r.ady = A->ay / (2.0 * A->dy);
  r.react = A->react;
  r.ba = A->brus_a;
  r.bb = A->brus_b;
  r.orth = cfg.orth;
  r.fixed_m = cfg.fixed_m;
  r.fixed_substeps = cfg.fixed_m > 0 ? cfg.fixed_substeps : 0;
  r.max_substeps = cfg.max_substeps > 0 ? cfg.max_substeps : 2000;
  r.m_max = m_max;
  r.persistent = cfg.exec_mode == KP_EXEC_PERSISTENT ? 1 : 0;
  r.basis_f32 = cfg.basis_dtype == KP_BASIS_F32 ? 1 : 0;
  r.h = h;
  r.tol = tol > 0.0 ? tol : 1.0;
  r.delta = cfg.fallback_delta == 0.0 ? 1e-10 : (cfg.fallback_delta < 0.0 ? 0.0 : cfg.fallback_delta);
  r.eps_bd = cfg.breakdown_eps == 0.0 ? 1e-12 : cfg.breakdown_eps;
  *a = r;
  return KP_OK;
}

template <typename TB>
int occupancy(kp_ctx* ctx, int which) {
  if (ctx->occ[which] < 0) {
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, reinterpret_cast<const void*>(&kp::k_persistent<TB>), kp::kThreads, 0);
    if (e != hipSuccess) return -1;
    ctx->occ[which] = occ;
  }
  return ctx->occ[which];
}

int device_setup(kp_ctx* ctx) {
  if (ctx->ncu > 0) return KP_OK;
  KP_HIP(ctx, hipGetDevice(&ctx->device));
  int ncu = 0, rate_khz = 0;
  KP_HIP(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  KP_HIP(ctx, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device));
  ctx->ncu = ncu;
  if (rate_khz <= 0) rate_khz = 100000;
  ctx->wait_ticks = (int64_t)rate_khz * 1000 * 4;   // 4 s
  return KP_OK;
}

int grow(kp_ctx* ctx, void** p, size_t* have, size_t need) {
  if (*have >= need) return KP_OK;
  if (*p) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    hipFree(*p);
    *p = nullptr;
    *have = 0;
  }
  hipError_t e = hipMalloc(p, need);
  if (e != hipSuccess) {
    *p = nullptr;
    snprintf(ctx->err, sizeof(ctx->err), "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    return KP_ENOMEM;
  }
  *have = need;
  return KP_OK;
}

// Allocate the workspace for a problem and finish Args (grid geometry).
int prepare(kp_ctx* ctx, Args* a) {
  int rc = device_setup(ctx);
  if (rc) return rc;
  const size_t esz = a->basis_f32 ? sizeof(float) : sizeof(double);
  const size_t vneed = (size_t)a->ld * (size_t)(a->m_max + 2) * esz;
  if ((rc = grow(ctx, &ctx->V, &ctx->v_bytes, vneed))) return rc;
  if ((rc = grow(ctx, reinterpret_cast<void**>(&ctx->u), &ctx->u_bytes,
                 (size_t)a->ld * sizeof(double))))
    return rc;
  const int occ = a->basis_f32 ? occupancy<float>(ctx, 1) : occupancy<double>(ctx, 0);
  if (occ <= 0) {
    snprintf(ctx->err, sizeof(ctx->err), "persistent kernel does not fit on a CU");
    return KP_EHIP;
  }
  const int64_t per_wg = (int64_t)kp::kThreads * kp::kR;
  int64_t nwg = (a->npairs + per_wg - 1) / per_wg;
  nwg = std::max<int64_t>(1, std::min<int64_t>(nwg, (int64_t)ctx->ncu * occ));
  a->nwg = (int)nwg;
  a->ppw = (a->npairs + nwg - 1) / nwg;
  if ((rc = grow(ctx, reinterpret_cast<void**>(&ctx->part), &ctx->part_bytes,
                 (size_t)nwg * kp::kKStride * sizeof(double))))
    return rc;
  if (!ctx->st) {
    KP_HIP(ctx, hipMalloc(&ctx->st, sizeof(State)));
    KP_HIP(ctx, hipMalloc(&ctx->sync, 64));
    KP_HIP(ctx, hipMalloc(&ctx->ex, sizeof(double) * kp::kExSlots * kp::kNmPad * kp::kNmPad));
  }
  a->V = ctx->V;
  a->u = ctx->u;
  a->part = ctx->part;
  a->sync = ctx->sync;
  a->st = ctx->st;
  a->ex = ctx->ex;
  a->wait_ticks = ctx->wait_ticks;
  return KP_OK;
}

template <typename TB, int PH, int SUB>
int launch_phase(kp_ctx* ctx, const Args& a, int grid) {
  hipLaunchKernelGGL((kp::k_phase<TB, PH, SUB>), dim3(grid), dim3(kp::kThreads), 0,
                     ctx->stream, a);
  KP_HIP(ctx, hipGetLastError());
  return KP_OK;
}

template <typename TB>
int run_stream(kp_ctx* ctx, const Args& a) {
  int rc;
  if ((rc = launch_phase<TB, kp::PH_STAGE, 0>(ctx, a, a.nwg))) return rc;
  for (int s = 0; s < a.fixed_substeps; ++s) {
    for (int j = 0; j < a.fixed_m; ++j) {
      if ((rc = launch_phase<TB, kp::PH_STEP, 0>(ctx, a, a.nwg))) return rc;
      if ((rc = launch_phase<TB, kp::PH_STEP, 1>(ctx, a, a.nwg))) return rc;
    }
    if ((rc = launch_phase<TB, kp::PH_EXPM, 0>(ctx, a, 1))) return rc;
    if ((rc = launch_phase<TB, kp::PH_COMBINE, 0>(ctx, a, a.nwg))) return rc;
  }
  return launch_phase<TB, kp::PH_FINISH, 0>(ctx, a, a.nwg);
}

template <typename TB>
int run_persistent(kp_ctx* ctx, Args a) {
  void* args[] = {&a};
  KP_HIP(ctx, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&kp::k_persistent<TB>),
                                         dim3(a.nwg), dim3(kp::kThreads), args, 0,
                                         ctx->stream));
  return KP_OK;
}

int fill_info(kp_ctx* ctx, kp_info* info) {
  KP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  State h;
  KP_HIP(ctx, hipMemcpy(&h, ctx->st, offsetof(State, sigma), hipMemcpyDeviceToHost));
  unsigned flags[3] = {0, 0, 0};
  KP_HIP(ctx, hipMemcpy(flags, ctx->sync, sizeof(flags), hipMemcpyDeviceToHost));
  std::memset(info, 0, sizeof(*info));
  info->status = flags[2] ? KP_STATUS_ABORTED : h.status;
  info->substeps = h.substeps;
  info->rejected = h.rejected;
  info->arnoldi_steps = h.arnoldi_steps;
  info->expm_evals = h.expm_evals;
  info->m_last = h.m_last;
  info->n_fallback = h.n_fallback;
  info->breakdowns = h.breakdowns;
  info->schedule_len = std::min(h.nlog, kp::kLogMax);
  info->err_max = h.err_max;
  info->mu = h.mu;
  info->t_end = h.t;
  return KP_OK;
}

}  // namespace

extern "C" {

int kp_version(void) { return 10000; }

const char* kp_strerror(int code) {
  switch (code) {
    case KP_OK: return "ok";
    case KP_EINVAL: return "invalid argument";
    case KP_ENOMEM: return "device allocation failed";
    case KP_EHIP: return "HIP runtime error";
    case KP_EUNSUPPORTED: return "unsupported combination of options";
    case KP_ESTATE: return "call out of order";
    default: return "unknown error";
  }
}

const char* kp_last_error(kp_ctx* ctx) { return ctx ? ctx->err : ""; }

int kp_create(kp_ctx** out, const kp_config* cfg) {
  if (!out) return KP_EINVAL;
  kp_config c{};
  if (cfg) c = *cfg;
  int rc = check_config(&c);
  if (rc) return rc;
  kp_ctx* ctx = new (std::nothrow) kp_ctx();
  if (!ctx) return KP_ENOMEM;
  ctx->cfg = c;
  ctx->stream = static_cast<hipStream_t>(c.stream);
  *out = ctx;
  return KP_OK;
}

int kp_set_config(kp_ctx* ctx, const kp_config* cfg) {
  if (!ctx || !cfg) return KP_EINVAL;
  int rc = check_config(cfg);
  if (rc) return rc;
  ctx->cfg = *cfg;
  ctx->stream = static_cast<hipStream_t>(cfg->stream);
  ctx->have_begin = 0;
  return KP_OK;
}

int kp_destroy(kp_ctx* ctx) {
  if (!ctx) return KP_EINVAL;
  if (ctx->ncu > 0) hipStreamSynchronize(ctx->stream);
  if (ctx->V) hipFree(ctx->V);
  if (ctx->u) hipFree(ctx->u);
  if (ctx->part) hipFree(ctx->part);
  if (ctx->st) hipFree(ctx->st);
  if (ctx->sync) hipFree(ctx->sync);
  if (ctx->ex) hipFree(ctx->ex);
  delete ctx;
  return KP_OK;
}

int kp_phi_combo(kp_ctx* ctx, const kp_op* A, const double* B, int32_t p, int64_t ldb,
                 double h, double tol, int32_t m_max, double* out, kp_info* info) {
  Args a;
  int rc = build_args(ctx, A, B, p, ldb, h, tol, m_max, out, true, &a);
  if (rc) return rc;
  if (ctx->cfg.exec_mode == KP_EXEC_STREAM && ctx->cfg.fixed_m == 0) return KP_EUNSUPPORTED;
  if ((rc = prepare(ctx, &a))) return rc;
  const int m0 = a.fixed_m > 0 ? a.fixed_m : std::min(16, a.m_max);
  hipLaunchKernelGGL(kp::k_init, dim3(1), dim3(256), 0, ctx->stream, a, m0);
  KP_HIP(ctx, hipGetLastError());
  if (a.persistent) {
    rc = a.basis_f32 ? run_persistent<float>(ctx, a) : run_persistent<double>(ctx, a);
  } else {
    rc = a.basis_f32 ? run_stream<float>(ctx, a) : run_stream<double>(ctx, a);
  }
  if (rc) return rc;
  ctx->last = a;
  ctx->have_begin = 0;
  if (info) return fill_info(ctx, info);
  return KP_OK;
}

int kp_get_schedule(kp_ctx* ctx, double* tau_host, int32_t* m_host, int32_t cap) {
  if (!ctx || cap < 0 || (cap > 0 && (!tau_host || !m_host))) return KP_EINVAL;
  if (!ctx->st) return KP_ESTATE;
  KP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int nlog = 0;
  KP_HIP(ctx, hipMemcpy(&nlog, &ctx->st->nlog, sizeof(int), hipMemcpyDeviceToHost));
  const int n = std::min(std::min(nlog, kp::kLogMax), cap);
  if (n > 0) {
    KP_HIP(ctx, hipMemcpy(tau_host, ctx->st->log_tau, n * sizeof(double), hipMemcpyDeviceToHost));
    KP_HIP(ctx, hipMemcpy(m_host, ctx->st->log_m, n * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  return n;
}

int kp_arnoldi_begin(kp_ctx* ctx, const kp_op* A, const double* B, int32_t p, int64_t ldb,
                     int32_t m_max) {
  if (!ctx) return KP_EINVAL;
  Args a;
  kp_config saved = ctx->cfg;
  ctx->cfg.fixed_m = 0;
  int rc = build_args(ctx, A, B, p, ldb, 1.0, 1.0, m_max, nullptr, false, &a);
  ctx->cfg = saved;
  if (rc) return rc;
  a.persistent = 0;
  if ((rc = prepare(ctx, &a))) return rc;
  hipLaunchKernelGGL(kp::k_init, dim3(1), dim3(256), 0, ctx->stream, a, m_max);
  KP_HIP(ctx, hipGetLastError());
  rc = a.basis_f32 ? launch_phase<float, kp::PH_STAGE, 0>(ctx, a, a.nwg)
                   : launch_phase<double, kp::PH_STAGE, 0>(ctx, a, a.nwg);
  if (rc) return rc;
  ctx->last = a;
  ctx->have_begin = 1;
  return KP_OK;
}

int kp_arnoldi_step(kp_ctx* ctx, int32_t nsteps) {
  if (!ctx || nsteps < 0) return KP_EINVAL;
  if (!ctx->have_begin) return KP_ESTATE;
  const Args& a = ctx->last;
  for (int s = 0; s < nsteps; ++s) {
    int rc;
    if (a.basis_f32) {
      if ((rc = launch_phase<float, kp::PH_STEP, 0>(ctx, a, a.nwg))) return rc;
      if ((rc = launch_phase<float, kp::PH_STEP, 1>(ctx, a, a.nwg))) return rc;
    } else {
      if ((rc = launch_phase<double, kp::PH_STEP, 0>(ctx, a, a.nwg))) return rc;
      if ((rc = launch_phase<double, kp::PH_STEP, 1>(ctx, a, a.nwg))) return rc;
    }
  }
  return KP_OK;
}

int kp_arnoldi_read(kp_ctx* ctx, double* H_host, double* V_host, int32_t* j_host,
                    double* beta_host, int32_t* flags_host) {
  if (!ctx) return KP_EINVAL;
  if (!ctx->have_begin) return KP_ESTATE;
  const Args& a = ctx->last;
  KP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<char> buf(sizeof(State));
  State* h = reinterpret_cast<State*>(buf.data());
  KP_HIP(ctx, hipMemcpy(h, ctx->st, sizeof(State), hipMemcpyDeviceToHost));
  const int j = h->j;
  if (j_host) *j_host = j;
  if (beta_host) *beta_host = h->beta;
  if (flags_host) {
    flags_host[0] = h->breakdown;
    flags_host[1] = h->n_fallback;
  }
  if (H_host) {
    const int mm = a.m_max;
    for (int c = 0; c < mm; ++c)
      for (int r = 0; r <= mm; ++r) H_host[(size_t)c * (mm + 1) + r] = h->H[(size_t)c * kp::kLdh + r];
  }
  if (V_host) {
    const int ncol = j + 1;
    const size_t L = (size_t)a.L;
    const size_t esz = a.basis_f32 ? sizeof(float) : sizeof(double);
    std::vector<char> raw((size_t)a.ld * ncol * esz);
    KP_HIP(ctx, hipMemcpy(raw.data(), ctx->V, raw.size(), hipMemcpyDeviceToHost));
    for (int c = 0; c < ncol; ++c) {
      double scale;
      if (c < j) scale = h->sigma[c];
      else scale = (h->last_nrm2 > 0.0 && !h->breakdown) ? 1.0 / std::sqrt(h->last_nrm2) : 0.0;
      for (size_t e = 0; e < L; ++e) {
        const double v = a.basis_f32 ? (double)reinterpret_cast<float*>(raw.data())[(size_t)c * a.ld + e]
                                     : reinterpret_cast<double*>(raw.data())[(size_t)c * a.ld + e];
        V_host[(size_t)c * L + e] = v * scale;
      }
    }
  }
  return KP_OK;
}

int kp_expm_hbar(kp_ctx* ctx, const double* H_host, int32_t ldh, int32_t m, double tau,
                 double* F_host) {
  if (!ctx || !H_host || !F_host || m < 1 || m > KP_MMAX || ldh < m + 1 || !std::isfinite(tau))
    return KP_EINVAL;
  int rc = device_setup(ctx);
  if (rc) return rc;
  if (!ctx->st) {
    KP_HIP(ctx, hipMalloc(&ctx->st, sizeof(State)));
    KP_HIP(ctx, hipMalloc(&ctx->sync, 64));
    KP_HIP(ctx, hipMalloc(&ctx->ex, sizeof(double) * kp::kExSlots * kp::kNmPad * kp::kNmPad));
  }
  std::vector<double> Hs((size_t)kp::kLdh * kp::kMMax, 0.0);
  for (int c = 0; c < m; ++c)
    for (int r = 0; r <= m; ++r) Hs[(size_t)c * kp::kLdh + r] = H_host[(size_t)c * ldh + r];
  KP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  KP_HIP(ctx, hipMemcpy(ctx->st->H, Hs.data(), Hs.size() * sizeof(double), hipMemcpyHostToDevice));
  Args a{};
  a.st = ctx->st;
  a.ex = ctx->ex;
  hipLaunchKernelGGL(kp::k_expm_test, dim3(1), dim3(kp::kThreads), 0, ctx->stream, a, m, tau);
  KP_HIP(ctx, hipGetLastError());
  KP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  KP_HIP(ctx, hipMemcpy(F_host, ctx->st->F, (m + 1) * sizeof(double), hipMemcpyDeviceToHost));
  return KP_OK;
}

}  // extern "C"
