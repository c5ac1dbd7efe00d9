// A client of libkrylov_phi through its C ABI only (HIP runtime + the header,
// no Python, no torch): reads an advection-diffusion problem from a raw file,
// runs kp_phi_combo, kp_phi_combo_batched (the same problem twice) and
// kp_phi_combo_backward, and writes the results for the test to compare.
//
// usage: c_abi_client <in.bin> <out.bin>
//   in.bin : int32 nx, ny, p, m, nsub; double nu, ax, ay, react, h, tol;
//            B (N x (p+1), column-major); g (N)
//   out.bin: int32 status x4; y (N); y_batched (2N); grad_B (N x (p+1));
//            grad_coef (4)
// Fixed schedule when m > 0 (nsub substeps of m steps), adaptive otherwise.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "krylov_phi.h"

#define CHECK_HIP(x)                                                     \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      return 2;                                                          \
    }                                                                    \
  } while (0)

static kp_ctx* g_ctx = nullptr;   // for the detail of a failure

#define CHECK_KP(x)                                                      \
  do {                                                                   \
    int r_ = (x);                                                        \
    if (r_ != KP_OK) {                                                   \
      fprintf(stderr, "%s: %s (%s)\n", #x, kp_strerror(r_),              \
              kp_last_error(g_ctx));                                     \
      return 3;                                                          \
    }                                                                    \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
    return 1;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 1;
  int32_t hdr[5];
  double par[6];
  if (fread(hdr, sizeof(hdr), 1, f) != 1 || fread(par, sizeof(par), 1, f) != 1) return 1;
  const int nx = hdr[0], ny = hdr[1], p = hdr[2], m = hdr[3], nsub = hdr[4];
  const size_t N = (size_t)nx * ny;
  std::vector<double> B(N * (p + 1)), g(N);
  if (fread(B.data(), sizeof(double), B.size(), f) != B.size()) return 1;
  if (fread(g.data(), sizeof(double), N, f) != N) return 1;
  fclose(f);

  double *dB, *dg, *dy, *dyb, *dgB, *dgc;
  CHECK_HIP(hipMalloc(&dB, B.size() * sizeof(double)));
  CHECK_HIP(hipMalloc(&dg, N * sizeof(double)));
  CHECK_HIP(hipMalloc(&dy, N * sizeof(double)));
  CHECK_HIP(hipMalloc(&dyb, 2 * N * sizeof(double)));
  CHECK_HIP(hipMalloc(&dgB, B.size() * sizeof(double)));
  CHECK_HIP(hipMalloc(&dgc, 4 * sizeof(double)));
  CHECK_HIP(hipMemcpy(dB, B.data(), B.size() * sizeof(double), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dg, g.data(), N * sizeof(double), hipMemcpyHostToDevice));

  kp_config cfg = {};
  if (m > 0) {
    cfg.fixed_m = m;
    cfg.fixed_substeps = nsub;
  }
  kp_ctx* ctx = nullptr;
  CHECK_KP(kp_create(&ctx, &cfg));
  g_ctx = ctx;
  kp_op A = {};
  A.kind = KP_OP_ADR;
  A.nx = nx;
  A.ny = ny;
  A.dx = 1.0 / nx;
  A.dy = 1.0 / ny;
  A.nu = par[0];
  A.ax = par[1];
  A.ay = par[2];
  A.react = par[3];
  const double h = par[4], tol = par[5];
  const int m_max = m > 0 ? m : 48;
  kp_info info[4] = {};
  CHECK_KP(kp_phi_combo(ctx, &A, dB, p, (int64_t)N, h, tol, m_max, dy, &info[0]));

  kp_op ops[2] = {A, A};
  const double* Bs[2] = {dB, dB};
  int32_t ps[2] = {p, p};
  int64_t lds[2] = {(int64_t)N, (int64_t)N};
  double hs[2] = {h, h};
  double* outs[2] = {dyb, dyb + N};
  kp_info binfo[2];
  CHECK_KP(kp_phi_combo_batched(ctx, 2, ops, Bs, ps, lds, hs, tol, m_max, outs, binfo));
  info[1] = binfo[0].status > binfo[1].status ? binfo[0] : binfo[1];

  CHECK_KP(kp_phi_combo_backward(ctx, &A, dB, p, (int64_t)N, h, tol, m_max, dg, dgB,
                                 (int64_t)N, 15, dgc, &info[2]));
  // the planner on the host, as a caller would inspect it
  int32_t team_of[2], wg0[256], sz[256], nteams = 0;
  double makespan = 0.0;
  CHECK_KP(kp_batch_plan(2, ops, ps, hs, m_max, 256, team_of, wg0, sz, &nteams, &makespan,
                         nullptr));
  info[3].status = (nteams >= 2 && team_of[0] != team_of[1] && makespan > 0.0) ? 0 : 9;

  std::vector<double> y(N), yb(2 * N), gB(B.size()), gc(4);
  CHECK_HIP(hipMemcpy(y.data(), dy, N * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(yb.data(), dyb, 2 * N * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(gB.data(), dgB, B.size() * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(gc.data(), dgc, 4 * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_KP(kp_destroy(ctx));
  hipFree(dB);
  hipFree(dg);
  hipFree(dy);
  hipFree(dyb);
  hipFree(dgB);
  hipFree(dgc);

  f = fopen(argv[2], "wb");
  if (!f) return 1;
  const int32_t st[4] = {info[0].status, info[1].status, info[2].status, info[3].status};
  fwrite(st, sizeof(st), 1, f);
  fwrite(y.data(), sizeof(double), N, f);
  fwrite(yb.data(), sizeof(double), 2 * N, f);
  fwrite(gB.data(), sizeof(double), gB.size(), f);
  fwrite(gc.data(), sizeof(double), 4, f);
  fclose(f);
  printf("c_abi_client: N=%zu p=%d statuses %d %d %d %d\n", N, p, st[0], st[1], st[2], st[3]);
  return 0;
}
