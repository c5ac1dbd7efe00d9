// libkrylov_phi: kernels and the C ABI declared in include/krylov_phi.h.
//
// Execution model (one MI355X, gfx950).  A whole phi_combo call is ONE
// cooperative launch of k_run: every workgroup loops over the phases published
// by workgroup 0 (stage, Arnoldi step = matvec+dots then update+norm, small
// exponential + controller, combine, finish) and meets the others at
// grid-wide barriers.  The grid-wide reduction of an Arnoldi step is the
// paper's single global synchronisation (Algorithm 4): every workgroup
// publishes its partial inner products, workgroup 0 reduces them and runs the
// O(m^2) scalar step, then releases the grid.  The adaptive substep controller
// runs on the device; nothing returns to the host until the call is done.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "kp_internal.h"
#include "kp_leader.h"
#include "kp_passes.h"

namespace kp {

// Carve-up of the shared phase buffer (doubles).  Streaming phases: per-wave
// partial sums (sacc), coefficients, block-reduction scratch and the LDS copy
// of the stencil halo rows (hl).  Leader work, after sacc is dead: group sums
// of the partial reduction (grp), then the scalar-step work arrays (wk), and
// the reduced inner products tv.  The small exponential uses the whole buffer
// (it runs in a phase of its own).  The correction-matrix tables of the leader
// live in a separate buffer for the whole launch.
constexpr int kOffSacc = 0;
constexpr int kOffGrp = 0;
constexpr int kOffWk = 0;
constexpr int kOffCoef = kWaves * kKStride;
constexpr int kOffRed = kOffCoef + kMMax + 8;
constexpr int kOffTv = kOffRed + kWaves;
constexpr int kOffHl = 1536;
constexpr int kHaloCap = 8192;            // 2 * nplanes * nx doubles at most
constexpr int kLdsDoubles = (2 * kNmPad * kNmPad > kOffHl + kHaloCap) ? 2 * kNmPad * kNmPad
                                                                      : kOffHl + kHaloCap;
static_assert(kOffGrp + kRg * kKStride <= kOffCoef, "grp overlaps coef");
static_assert(kOffWk + kWkDoubles <= kOffCoef, "wk overlaps coef");
static_assert(kOffTv + kKStride <= kOffHl, "tv overlaps the halo copy");
static_assert(kLdsDoubles >= kNmPad * kGjLd, "the small exponential does not fit the phase buffer");

// One phase of the call for this workgroup.  cur: control of the phase (LDS,
// identical in every workgroup); nxt: the leader's control of the next phase;
// ok: cleared when a bounded wait gives up (the launch is aborting).  On
// return cur holds the control of the next phase.
template <typename TB>
__device__ __attribute__((always_inline)) inline void run_phase(const Args& a, double* lds, LeadLds& L, Ctl& cur, Ctl& nxt, int& ok,
                          unsigned k) {
  double* sacc = lds + kOffSacc;
  double* grp = lds + kOffGrp;
  double* wk = lds + kOffWk;
  double* red = lds + kOffRed;
  double* tv = lds + kOffTv;
  double* hl = lds + kOffHl;
  const bool lead = blockIdx.x == 0;
  const Ctl c = cur;
  // streaming part of the phase (every workgroup)
  switch (c.phase) {
    case PH_STAGE:
      stage_pass(a, red);
      break;
    case PH_STEP:
      // the update that produces x_j (coefficients of the previous scalar
      // step), then the matvec + grouped dots of step j: one grid-wide sync
      if (c.upd) {
        update_pass<TB>(a, c.j - 1, a.pub->coef, red, false);
        flag_publish(a, k);
        flag_wait_neighbours(a, k);
      }
      if (a.halo_lds)
        matvec_dots_pass<TB, true>(a, c.j, sacc, hl);
      else
        matvec_dots_pass<TB, false>(a, c.j, sacc, hl);
      break;
    case PH_CLOSE:
      update_pass<TB>(a, c.j - 1, a.pub->coef, red, true);
      break;
    case PH_COMBINE:
      combine_pass<TB>(a, c.m_eff, a.pub->coef, c.last != 0);
      break;
    case PH_FINISH:
      finish_pass(a, c.status == KP_STATUS_NONFINITE);
      break;
    default:
      break;
  }
  bar_arrive(a);
  if (!lead) {
    bar_wait(a, k, &cur, &ok);
    return;
  }
  // serial part (workgroup 0)
  bar_gather(a, k, &ok);
  if (!ok) return;
  if (kp_tid() == 0) nxt = c;
  switch (c.phase) {
    case PH_STAGE:
      leader_stage(a, red, nxt);
      break;
    case PH_STEP:
      reduce_partials(a, 2 * c.j + 3, tv, grp);
      scalar_step(a, c.j, tv, L, wk, nxt);
      break;
    case PH_CLOSE:
      reduce_partials(a, 1, tv, grp);
      leader_close(a, tv[0], L, nxt);
      break;
    case PH_EXPM:
      expm_phase(a, lds, L, nxt);
      break;
    case PH_COMBINE:
      leader_combine(a, L, nxt);
      break;
    case PH_FINISH:
      if (kp_tid() == 0) nxt.phase = PH_DONE;
      break;
    default:
      break;
  }
  bar_release(a, k, nxt, a.pub);
  if (kp_tid() == 0) cur = nxt;
}

// The whole call (or, for the step-by-step entry, the steps up to stop_j).
template <typename TB>
__global__ __launch_bounds__(kThreads) void k_run(Args a, int arnoldi_only) {
  __shared__ double lds[kLdsDoubles];
  __shared__ LeadLds lead;
  __shared__ Ctl cur, nxt;
  __shared__ int ok;
  __shared__ unsigned s_k;
  if (kp_tid() == 0) {
    // barriers released by earlier launches, and the control they announced
    const unsigned long long w = cload(release_word(a));
    s_k = (unsigned)(w >> 32);
    cur = ctl_unpack((unsigned)w);
    ok = aborted(a) ? 0 : 1;
  }
  if (blockIdx.x == 0) load_tables(a, lead);
  __syncthreads();
  unsigned k = s_k;
  for (;;) {
    __syncthreads();
    if (!ok || cur.phase == PH_DONE) break;
    if (arnoldi_only &&
        (cur.phase >= PH_EXPM || (cur.phase == PH_STEP && cur.j >= a.stop_j)))
      break;
    ++k;
    run_phase<TB>(a, lds, lead, cur, nxt, ok, k);
  }
}

// Reset of the call state; the Hessenberg and correction matrices are zeroed
// so that entries outside their triangles read as zero.
__global__ __launch_bounds__(256) void k_init(Args a, int m_target) {
  State* st = a.st;
  for (int i = kp_tid(); i < kLdh * kMMax; i += blockDim.x) st->H[i] = 0.0;
  for (int i = kp_tid(); i < kLdt * kMMax; i += blockDim.x) {
    st->Lm[i] = 0.0;
    st->Minv[i] = 0.0;
  }
  for (int i = kp_tid(); i < kMMax + 2; i += blockDim.x) a.pub->coef[i] = 0.0;
  for (int i = kp_tid(); i < a.nwg * kFlagStride; i += blockDim.x) a.flags[i] = 0u;
  if (kp_tid() != 0) return;
  for (int i = 0; i < 16; ++i) a.sync[i] = 0u;   // counters, release word (STAGE), abort
  Pub* pb = a.pub;
  pb->phase = PH_STAGE;
  pb->upd = 0;
  pb->j = 0;
  pb->m_eff = 0;
  pb->last = 0;
  pb->status = KP_STATUS_OK;
  pb->inv_mu = 1.0;
  st->m_target = m_target;
  st->m_cur = m_target;
  st->breakdown = 0;
  st->fallback_cur = 0;
  st->substeps = st->rejected = st->arnoldi_steps = st->expm_evals = 0;
  st->n_fallback = st->breakdowns = st->nlog = st->zero = 0;
  st->m_last = 0;
  st->t = 0.0;
  st->tau = (a.fixed_m > 0) ? a.h / (double)a.fixed_substeps : a.h;
  st->beta = 0.0;
  st->mu = 1.0;
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
using kp::Pub;
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
  double* hx = nullptr;
  size_t hx_bytes = 0;
  unsigned* flags = nullptr;
  size_t flags_bytes = 0;
  unsigned* sync = nullptr;
  State* st = nullptr;
  Pub* pub = nullptr;
  double* ex = nullptr;
  double* tx = nullptr;
  int occ[2] = {-1, -1};
  Args last{};
  int have_begin = 0;
  int arn_target = 0;
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
  if (c->reserved0 != 0) return KP_EINVAL;
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
  const int nplanes = A->kind == KP_OP_BRUSSELATOR ? 2 : 1;
  const int64_t npt = (int64_t)A->nx * A->ny;
  const int64_t N = npt * nplanes;
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
  r.p = p;
  r.pb = p;
  r.tangent = 0;
  r.dout = nullptr;
  r.npt = (int)npt;
  r.nx = A->nx;
  r.ny = A->ny;
  r.nplanes = nplanes;
  r.npt_pad = (npt + kp::kPlaneAlign - 1) / kp::kPlaneAlign * kp::kPlaneAlign;
  r.tail_off = r.npt_pad * nplanes;
  r.ld = r.tail_off + kp::kTailPad;
  r.kind = A->kind;
  r.transpose = A->transpose ? 1 : 0;
  r.cx = A->nu / (A->dx * A->dx);
  r.cy = A->nu / (A->dy * A->dy);
  r.cx2 = A->nu2 / (A->dx * A->dx);
  r.cy2 = A->nu2 / (A->dy * A->dy);
  r.inv_nx = 1.0 / (double)A->nx;
  r.halo_lds = (2 * nplanes * (int64_t)A->nx <= kp::kHaloCap) ? 1 : 0;
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
  r.stop_j = INT_MAX;
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
        &occ, reinterpret_cast<const void*>(&kp::k_run<TB>), kp::kThreads, 0);
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

// Grid geometry: workgroup b owns rows [b*rows, (b+1)*rows) of every plane.
// At least one full sub-tile (kThreads * kR pairs) of elements per workgroup,
// at most one workgroup per co-resident slot; an even row count when nx is
// odd keeps every segment start even (pair alignment).
void geometry(int ncu_slots, Args* a) {
  const int64_t per_wg_min = (int64_t)kp::kThreads * kp::kR * 2;
  int64_t rows = (per_wg_min + (int64_t)a->nx * a->nplanes - 1) / ((int64_t)a->nx * a->nplanes);
  rows = std::max<int64_t>(rows, (a->ny + ncu_slots - 1) / ncu_slots);
  rows = std::max<int64_t>(1, std::min<int64_t>(rows, a->ny));
  if ((a->nx & 1) && (rows & 1) && rows < a->ny) ++rows;
  a->rows_per_wg = (int)rows;
  a->nwg = (int)((a->ny + rows - 1) / rows);
}

// Allocate the workspace for a problem and finish Args.
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
    snprintf(ctx->err, sizeof(ctx->err), "the persistent kernel does not fit on a CU");
    return KP_EHIP;
  }
  geometry(ctx->ncu * occ, a);
  if ((rc = grow(ctx, reinterpret_cast<void**>(&ctx->part), &ctx->part_bytes,
                 (size_t)a->nwg * kp::kKStride * sizeof(double))))
    return rc;
  if ((rc = grow(ctx, reinterpret_cast<void**>(&ctx->hx), &ctx->hx_bytes,
                 (size_t)a->nwg * a->nplanes * 2 * a->nx * sizeof(double))))
    return rc;
  if ((rc = grow(ctx, reinterpret_cast<void**>(&ctx->flags), &ctx->flags_bytes,
                 (size_t)a->nwg * kp::kFlagStride * sizeof(unsigned))))
    return rc;
  if (!ctx->st) {
    KP_HIP(ctx, hipMalloc(&ctx->st, sizeof(State)));
    KP_HIP(ctx, hipMalloc(&ctx->pub, sizeof(Pub)));
    KP_HIP(ctx, hipMalloc(&ctx->sync, 64));
    KP_HIP(ctx, hipMalloc(&ctx->ex, sizeof(double) * kp::kExSlots * kp::kNmPad * kp::kNmPad));
    KP_HIP(ctx, hipMalloc(&ctx->tx, sizeof(double) * kp::kTailPad));
  }
  a->V = ctx->V;
  a->u = ctx->u;
  a->part = ctx->part;
  a->hx = ctx->hx;
  a->tx = ctx->tx;
  a->flags = ctx->flags;
  a->sync = ctx->sync;
  a->st = ctx->st;
  a->pub = ctx->pub;
  a->ex = ctx->ex;
  a->wait_ticks = ctx->wait_ticks;
  return KP_OK;
}

template <typename TB>
int launch_run(kp_ctx* ctx, Args a, int arnoldi_only) {
  void* args[] = {&a, &arnoldi_only};
  KP_HIP(ctx, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&kp::k_run<TB>),
                                         dim3(a.nwg), dim3(kp::kThreads), args, 0,
                                         ctx->stream));
  return KP_OK;
}

int launch(kp_ctx* ctx, const Args& a, int arnoldi_only) {
  return a.basis_f32 ? launch_run<float>(ctx, a, arnoldi_only)
                     : launch_run<double>(ctx, a, arnoldi_only);
}

int launch_init(kp_ctx* ctx, const Args& a, int m_target) {
  hipLaunchKernelGGL(kp::k_init, dim3(1), dim3(256), 0, ctx->stream, a, m_target);
  KP_HIP(ctx, hipGetLastError());
  return KP_OK;
}

int fill_info(kp_ctx* ctx, kp_info* info) {
  KP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  State h;
  KP_HIP(ctx, hipMemcpy(&h, ctx->st, offsetof(State, sigma), hipMemcpyDeviceToHost));
  Pub pb;
  KP_HIP(ctx, hipMemcpy(&pb, ctx->pub, sizeof(Pub), hipMemcpyDeviceToHost));
  unsigned flags[16] = {0};
  KP_HIP(ctx, hipMemcpy(flags, ctx->sync, sizeof(flags), hipMemcpyDeviceToHost));
  std::memset(info, 0, sizeof(*info));
  info->status = flags[kp::kSyncAbort] ? KP_STATUS_ABORTED : pb.status;
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

int kp_version(void) { return 10100; }

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
  void* bufs[] = {ctx->V,  ctx->u,    ctx->part, ctx->hx, ctx->flags,
                  ctx->st, ctx->pub, ctx->sync, ctx->ex, ctx->tx};
  for (void* b : bufs)
    if (b) hipFree(b);
  delete ctx;
  return KP_OK;
}

int kp_phi_combo(kp_ctx* ctx, const kp_op* A, const double* B, int32_t p, int64_t ldb,
                 double h, double tol, int32_t m_max, double* out, kp_info* info) {
  Args a;
  int rc = build_args(ctx, A, B, p, ldb, h, tol, m_max, out, true, &a);
  if (rc) return rc;
  if ((rc = prepare(ctx, &a))) return rc;
  const int m0 = a.fixed_m > 0 ? a.fixed_m : std::min(16, a.m_max);
  if ((rc = launch_init(ctx, a, m0))) return rc;
  if ((rc = launch(ctx, a, 0))) return rc;
  ctx->last = a;
  ctx->have_begin = 0;
  if (info) return fill_info(ctx, info);
  return KP_OK;
}

int kp_phi_combo_tangent(kp_ctx* ctx, const kp_op* A, const kp_op* dA, const double* B,
                         int32_t p, int64_t ldb, double h, double tol, int32_t m_max,
                         double* out, double* dout, kp_info* info) {
  if (!ctx || !A || !dA || !dout) return KP_EINVAL;
  if (A->kind != KP_OP_ADR && A->kind != KP_OP_ALLEN_CAHN) return KP_EUNSUPPORTED;
  if (dA->kind != A->kind || dA->nx != A->nx || dA->ny != A->ny || dA->dx != A->dx ||
      dA->dy != A->dy || (dA->transpose != 0) != (A->transpose != 0))
    return KP_EINVAL;
  if (dA->field0 || dA->field1) return KP_EUNSUPPORTED;
  const double dc[] = {dA->nu, dA->ax, dA->ay, dA->react};
  for (double v : dc)
    if (!std::isfinite(v)) return KP_EINVAL;
  if (p < 0 || 2 * p > KP_PMAX) return KP_EUNSUPPORTED;
  Args a;
  int rc = build_args(ctx, A, B, p, ldb, h, tol, m_max, out, true, &a);
  if (rc) return rc;
  const size_t ob = (size_t)a.N * sizeof(double);
  if (overlaps(dout, ob, out, ob) || overlaps(dout, ob, B, (size_t)ldb * (p + 1) * sizeof(double)) ||
      overlaps(dout, ob, A->field0, ob))
    return KP_EINVAL;
  // the pair [a; c] of augmented vectors: two planes, tail of 2p entries
  a.tangent = 1;
  a.dout = dout;
  a.nplanes = 2;
  a.pb = p;
  a.p = 2 * p;
  a.tail_off = a.npt_pad * 2;
  a.ld = a.tail_off + kp::kTailPad;
  a.halo_lds = (2 * 2 * (int64_t)A->nx <= kp::kHaloCap) ? 1 : 0;
  a.dcx = dA->nu / (A->dx * A->dx);
  a.dcy = dA->nu / (A->dy * A->dy);
  a.dadx = dA->ax / (2.0 * A->dx);
  a.dady = dA->ay / (2.0 * A->dy);
  a.dreact = dA->react;
  if ((rc = prepare(ctx, &a))) return rc;
  const int m0 = a.fixed_m > 0 ? a.fixed_m : std::min(16, a.m_max);
  if ((rc = launch_init(ctx, a, m0))) return rc;
  if ((rc = launch(ctx, a, 0))) return rc;
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
  if ((rc = prepare(ctx, &a))) return rc;
  a.stop_j = 0;
  if ((rc = launch_init(ctx, a, m_max))) return rc;
  if ((rc = launch(ctx, a, 1))) return rc;
  ctx->last = a;
  ctx->have_begin = 1;
  ctx->arn_target = 0;
  return KP_OK;
}

int kp_arnoldi_step(kp_ctx* ctx, int32_t nsteps) {
  if (!ctx || nsteps < 0) return KP_EINVAL;
  if (!ctx->have_begin) return KP_ESTATE;
  ctx->arn_target = std::min(ctx->arn_target + nsteps, ctx->last.m_max);
  Args a = ctx->last;
  a.stop_j = ctx->arn_target;
  return launch(ctx, a, 1);
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
  Pub pb;
  KP_HIP(ctx, hipMemcpy(&pb, ctx->pub, sizeof(Pub), hipMemcpyDeviceToHost));
  const int j = pb.j;
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
    const size_t L = (size_t)a.N + a.p;
    const size_t esz = a.basis_f32 ? sizeof(float) : sizeof(double);
    std::vector<char> raw((size_t)a.ld * ncol * esz);
    KP_HIP(ctx, hipMemcpy(raw.data(), ctx->V, raw.size(), hipMemcpyDeviceToHost));
    for (int c = 0; c < ncol; ++c) {
      double scale;
      if (c < j) scale = h->sigma[c];
      else scale = (h->last_nrm2 > 0.0 && !h->breakdown) ? 1.0 / std::sqrt(h->last_nrm2) : 0.0;
      auto at = [&](int64_t e) {
        return a.basis_f32 ? (double)reinterpret_cast<float*>(raw.data())[(size_t)c * a.ld + e]
                           : reinterpret_cast<double*>(raw.data())[(size_t)c * a.ld + e];
      };
      for (int s = 0; s < a.nplanes; ++s)
        for (int64_t q = 0; q < a.npt; ++q)
          V_host[(size_t)c * L + (size_t)s * a.npt + q] = at(s * a.npt_pad + q) * scale;
      for (int k = 0; k < a.p; ++k)
        V_host[(size_t)c * L + a.N + k] = at(a.tail_off + k) * scale;
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
    KP_HIP(ctx, hipMalloc(&ctx->pub, sizeof(Pub)));
    KP_HIP(ctx, hipMalloc(&ctx->sync, 64));
    KP_HIP(ctx, hipMalloc(&ctx->ex, sizeof(double) * kp::kExSlots * kp::kNmPad * kp::kNmPad));
    KP_HIP(ctx, hipMalloc(&ctx->tx, sizeof(double) * kp::kTailPad));
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
