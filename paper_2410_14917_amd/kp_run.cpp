// kp_run: a native runner of libkrylov_phi (the C ABI alone, the system HIP
// runtime, no Python), for profiling a process that maps exactly one HIP
// runtime.  It reads a problem's arrays from raw float64 files, makes
// --warmup untimed and --steps timed kp_phi_combo calls on one stream, times
// each with HIP events and prints one JSON line.
//
//   kp_run --kind K --nx NX --ny NY [--nu NU --nu2 NU2 --ax AX --ay AY
//          --react R --brus-a A --brus-b B --dx DX --dy DY]
//          --p P --h H --tol TOL --m-max M --B file [--field0 f --field1 f]
//          [--orth O] [--basis 0|1] [--fixed-m M --fixed-substeps S]
//          [--controller 0|1] [--steps K] [--warmup W] [--out file]
//          [--calib-copy]
//
// B holds N x (p+1) float64 column-major (columns b_0..b_p); fields hold
// nx*ny float64.  --calib-copy first runs one elementwise kernel that reads
// and writes 1 GiB (dst = -src), the reference of the HBM counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "krylov_phi.h"

namespace {

__global__ void k_neg(const double* __restrict__ src, double* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = -src[i];
}

bool read_file(const std::string& path, std::vector<double>* v, size_t n) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  v->resize(n);
  const size_t got = std::fread(v->data(), sizeof(double), n, f);
  const bool extra = std::fgetc(f) != EOF;
  std::fclose(f);
  return got == n && !extra;
}

int fail(const char* what, const char* detail) {
  std::fprintf(stderr, "kp_run: %s%s%s\n", what, detail ? ": " : "", detail ? detail : "");
  return 1;
}

#define HIPCHK(x)                                                   \
  do {                                                              \
    hipError_t e_ = (x);                                            \
    if (e_ != hipSuccess) return fail(#x, hipGetErrorString(e_));   \
  } while (0)

}  // namespace

int main(int argc, char** argv) {
  kp_op op{};
  op.brus_a = 1.0;
  op.brus_b = 3.0;
  kp_config cfg{};
  int p = 0, m_max = 64, steps = 5, warmup = 1;
  double h = 0.0, tol = 1e-8;
  bool calib = false;
  std::string fB, f0, f1, fout;
  for (int i = 1; i < argc; ++i) {
    const std::string k = argv[i];
    if (k == "--calib-copy") {
      calib = true;
      continue;
    }
    if (i + 1 >= argc) return fail("missing value for", k.c_str());
    const char* v = argv[++i];
    if (k == "--kind") op.kind = std::atoi(v);
    else if (k == "--nx") op.nx = std::atoi(v);
    else if (k == "--ny") op.ny = std::atoi(v);
    else if (k == "--nu") op.nu = std::atof(v);
    else if (k == "--nu2") op.nu2 = std::atof(v);
    else if (k == "--ax") op.ax = std::atof(v);
    else if (k == "--ay") op.ay = std::atof(v);
    else if (k == "--react") op.react = std::atof(v);
    else if (k == "--brus-a") op.brus_a = std::atof(v);
    else if (k == "--brus-b") op.brus_b = std::atof(v);
    else if (k == "--dx") op.dx = std::atof(v);
    else if (k == "--dy") op.dy = std::atof(v);
    else if (k == "--p") p = std::atoi(v);
    else if (k == "--h") h = std::atof(v);
    else if (k == "--tol") tol = std::atof(v);
    else if (k == "--m-max") m_max = std::atoi(v);
    else if (k == "--B") fB = v;
    else if (k == "--field0") f0 = v;
    else if (k == "--field1") f1 = v;
    else if (k == "--out") fout = v;
    else if (k == "--orth") cfg.orth = std::atoi(v);
    else if (k == "--basis") cfg.basis_dtype = std::atoi(v);
    else if (k == "--fixed-m") cfg.fixed_m = std::atoi(v);
    else if (k == "--fixed-substeps") cfg.fixed_substeps = std::atoi(v);
    else if (k == "--controller") cfg.controller = std::atoi(v);
    else if (k == "--steps") steps = std::atoi(v);
    else if (k == "--warmup") warmup = std::atoi(v);
    else return fail("unknown option", k.c_str());
  }
  if (op.nx < 1 || op.ny < 1 || p < 0 || fB.empty() || steps < 1 || warmup < 0)
    return fail("need --nx, --ny, --p, --B and positive --steps", nullptr);
  if (op.dx == 0.0) op.dx = 1.0 / op.nx;
  if (op.dy == 0.0) op.dy = 1.0 / op.ny;
  const size_t npt = (size_t)op.nx * op.ny;
  const size_t n = npt * (op.kind == KP_OP_BRUSSELATOR ? 2 : 1);
  std::vector<double> hB, h0, h1;
  if (!read_file(fB, &hB, n * (p + 1))) return fail("cannot read N x (p+1) doubles from", fB.c_str());
  if (!f0.empty() && !read_file(f0, &h0, npt)) return fail("cannot read nx*ny doubles from", f0.c_str());
  if (!f1.empty() && !read_file(f1, &h1, npt)) return fail("cannot read nx*ny doubles from", f1.c_str());

  hipStream_t stream;
  HIPCHK(hipStreamCreate(&stream));
  double *dB = nullptr, *d0 = nullptr, *d1 = nullptr, *dout = nullptr;
  HIPCHK(hipMalloc(&dB, hB.size() * sizeof(double)));
  HIPCHK(hipMemcpy(dB, hB.data(), hB.size() * sizeof(double), hipMemcpyHostToDevice));
  if (!h0.empty()) {
    HIPCHK(hipMalloc(&d0, npt * sizeof(double)));
    HIPCHK(hipMemcpy(d0, h0.data(), npt * sizeof(double), hipMemcpyHostToDevice));
  }
  if (!h1.empty()) {
    HIPCHK(hipMalloc(&d1, npt * sizeof(double)));
    HIPCHK(hipMemcpy(d1, h1.data(), npt * sizeof(double), hipMemcpyHostToDevice));
  }
  HIPCHK(hipMalloc(&dout, n * sizeof(double)));
  op.field0 = d0;
  op.field1 = d1;

  if (calib) {
    const size_t cn = (size_t)1 << 27;   // 1 GiB of float64
    double *src = nullptr, *dst = nullptr;
    HIPCHK(hipMalloc(&src, cn * sizeof(double)));
    HIPCHK(hipMalloc(&dst, cn * sizeof(double)));
    HIPCHK(hipMemsetAsync(src, 0, cn * sizeof(double), stream));
    hipLaunchKernelGGL(k_neg, dim3(4096), dim3(256), 0, stream, src, dst, cn);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    HIPCHK(hipFree(src));
    HIPCHK(hipFree(dst));
  }

  cfg.stream = stream;
  kp_ctx* ctx = nullptr;
  int rc = kp_create(&ctx, &cfg);
  if (rc) return fail("kp_create", kp_strerror(rc));
  kp_info info{};
  for (int w = 0; w < warmup; ++w) {
    rc = kp_phi_combo(ctx, &op, dB, p, (int64_t)n, h, tol, m_max, dout, &info);
    if (rc) return fail("kp_phi_combo", kp_last_error(ctx));
  }
  std::vector<hipEvent_t> e0(steps), e1(steps);
  for (int k = 0; k < steps; ++k) {
    HIPCHK(hipEventCreate(&e0[k]));
    HIPCHK(hipEventCreate(&e1[k]));
  }
  HIPCHK(hipStreamSynchronize(stream));
  for (int k = 0; k < steps; ++k) {
    HIPCHK(hipEventRecord(e0[k], stream));
    rc = kp_phi_combo(ctx, &op, dB, p, (int64_t)n, h, tol, m_max, dout, nullptr);
    if (rc) return fail("kp_phi_combo", kp_last_error(ctx));
    HIPCHK(hipEventRecord(e1[k], stream));
  }
  rc = kp_phi_combo(ctx, &op, dB, p, (int64_t)n, h, tol, m_max, dout, &info);
  if (rc) return fail("kp_phi_combo", kp_last_error(ctx));
  std::vector<double> ms(steps);
  for (int k = 0; k < steps; ++k) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0[k], e1[k]));
    ms[k] = t;
  }
  if (!fout.empty()) {
    std::vector<double> y(n);
    HIPCHK(hipMemcpy(y.data(), dout, n * sizeof(double), hipMemcpyDeviceToHost));
    FILE* f = std::fopen(fout.c_str(), "wb");
    if (!f || std::fwrite(y.data(), sizeof(double), n, f) != n) return fail("cannot write", fout.c_str());
    std::fclose(f);
  }
  std::vector<double> sorted = ms;
  std::sort(sorted.begin(), sorted.end());
  double mean = 0.0;
  for (double t : ms) mean += t / steps;
  int rv = 0, dv = 0;
  kp_runtime_version(&rv, &dv);
  std::printf("{\"N\": %zu, \"steps\": %d, \"avg_launch_ms\": %.4f, \"median_launch_ms\": %.4f, "
              "\"min_launch_ms\": %.4f, \"max_launch_ms\": %.4f, \"status\": %d, \"substeps\": %d, "
              "\"rejected\": %d, \"arnoldi_steps\": %d, \"hip_runtime_version\": %d}\n",
              n, steps, mean, sorted[steps / 2], sorted.front(), sorted.back(), info.status,
              info.substeps, info.rejected, info.arnoldi_steps, rv);
  std::fflush(stdout);  // a profiler may end the process abnormally at exit
  kp_destroy(ctx);
  hipFree(dB);
  hipFree(d0);
  hipFree(d1);
  hipFree(dout);
  hipStreamDestroy(stream);
  return info.status == KP_STATUS_OK ? 0 : 2;
}
