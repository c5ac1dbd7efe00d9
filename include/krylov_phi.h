/*
 * libkrylov_phi: Krylov evaluation of a linear combination of phi-functions
 * on one MI355X (gfx950).
 *
 *     out = sum_{k=0}^{p} h^k phi_k(h A) b_k
 *
 * phi_0(z) = e^z, phi_k(z) = int_0^1 e^{(1-s)z} s^{k-1}/(k-1)! ds (arXiv:2410.14917,
 * Section 2, eq. phi_int_def; the combination is eq. ansatz with the step h of
 * eq. philincomb).  The combination is the top block of exp(h Atilde) [b_0; e_p]
 * for the augmented matrix Atilde = [[A, B], [0, K]], B = [b_p, ..., b_1], K the
 * p x p upper shift (Section 2.1).  That exponential is applied by substepping
 * (Section 2.2, eq. substep); each substep is a Krylov projection (eq. kryexp)
 * whose basis comes from the hybrid low-synchronisation Arnoldi process
 * (Section 3.3, Algorithm 4) with one grid-wide reduction per step and the
 * correction matrix of Algorithm 5 (H-CWY), 6 (H-NCWY) or 7 (H-GSMGS).
 *
 * Conventions
 *  - All vectors and matrices passed as `const double*` / `double*` are DEVICE
 *    pointers (hipMalloc'd or equivalent) unless the parameter name ends in
 *    `_host`.  Device pointers are borrowed: the library never frees them, and
 *    the caller keeps them alive until the context's stream has passed the call.
 *  - Matrices are column-major with an explicit leading dimension.
 *  - Calls enqueue work on the context's stream and return; they are ordered
 *    with other work on that stream.  A call that fills a `kp_info` or copies
 *    results to host memory synchronises the stream before it returns.
 *  - Return codes are synchronous (argument and runtime errors).  Outcomes of
 *    the computation (not converged, non-finite data) are reported in
 *    kp_info.status.  No C++ exception crosses this interface.
 *  - A context is not thread-safe; use one context per stream/thread.
 *  - The solves are cooperative kernel launches.  On the ROCm runtime this
 *    library is built for, once a process has made such a launch (as
 *    kp_phi_combo does directly; the batched call's graph node does not), a
 *    cooperative launch from another process on the same GPU is refused while
 *    the first process lives: that call returns KP_EHIP, and kp_last_error
 *    reports "the operation cannot be performed in the present state".  Drive
 *    one GPU from one process.
 *  - Every device-wide wait is bounded (4 s; the environment variable
 *    KP_WAIT_LIMIT_US, read when a context first uses the device, sets
 *    another bound in microseconds).  A wait that exceeds it ends the launch
 *    cleanly and the call reports KP_STATUS_ABORTED.
 *  - The library links the system HIP runtime.  In a process that also uses a
 *    second copy (PyTorch ships its own), load that copy first: loaded after
 *    this library, its initialisation leaves this library's first device
 *    query reporting no device (KP_EHIP from the first call that touches
 *    the device).
 */
#ifndef KRYLOV_PHI_H
#define KRYLOV_PHI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define KP_OK            0
#define KP_EINVAL       -1  /* invalid argument (null, out of range, mismatch) */
#define KP_ENOMEM       -2  /* device allocation failed */
#define KP_EHIP         -3  /* HIP runtime error (message via kp_last_error) */
#define KP_EUNSUPPORTED -4  /* combination of options not supported */
#define KP_ESTATE       -5  /* call out of order (e.g. step before begin) */
#define KP_ETOOLARGE    -6  /* the problem exceeds a fixed capacity */

/* ---- kp_info.status ------------------------------------------------------ */
#define KP_STATUS_OK            0
#define KP_STATUS_NOT_CONVERGED 1  /* max_substeps reached or step size underflow */
#define KP_STATUS_NONFINITE     2  /* NaN/Inf in the input or the iteration */
#define KP_STATUS_ABORTED       3  /* a device-wide wait exceeded its limit */

/* ---- orthogonalisation ---------------------------------------------------
 * The hybrid one-reduction forms of Algorithm 4 (correction matrix
 * T ~ (V^T V)^{-1}): one grid-wide reduction per Arnoldi step. */
#define KP_ORTH_H_GSMGS 0  /* Algorithm 7: T = M^{-1}[I + N M^{-1}], default */
#define KP_ORTH_H_CWY   1  /* Algorithm 5: T = (I + L)^{-1} by recursion    */
#define KP_ORTH_H_NCWY  2  /* Algorithm 6: T = I - L (Neumann, two terms)   */
/* The comparators of Sections 2.3 and 4.2, in the same persistent kernel and
 * controller: */
#define KP_ORTH_MGS     3  /* Algorithm 1: modified Gram-Schmidt, j + 1 grid
                              reductions at step j (j inner products, 1 norm) */
#define KP_ORTH_IOCGS   4  /* ioCGS (Section 2.3.1): classical Gram-Schmidt
                              against the previous two vectors only, then the
                              norm: 2 grid reductions per step; V is not
                              orthonormal */

/* ---- substep-size controller -------------------------------------------- */
#define KP_CTRL_POWER 0    /* tau *= clamp(0.9 w^(-1/(q+1)), 0.2, 4) (default) */
#define KP_CTRL_PI    1    /* proportional-integral control after accepted
                              substeps (the Conclusion's future work; gains of
                              Gustafsson's PI controller): tau *= clamp(0.9
                              w^(-0.7/(q+1)) w_prev^(0.4/(q+1)), 0.2, 4) */

/* ---- operator kinds (matrix-free, 2D periodic, second-order FD) --------- */
#define KP_OP_ADR         0 /* nu Lap u - ax Dx u - ay Dy u + react u (+ field0 .* u) */
#define KP_OP_ALLEN_CAHN  1 /* nu Lap u + (1 - 3 field0^2) .* u                       */
#define KP_OP_BRUSSELATOR 2 /* Jacobian of the 2-species Brusselator at (field0, field1) */

/* ---- basis storage ------------------------------------------------------ */
#define KP_BASIS_F64 0
#define KP_BASIS_F32 1   /* basis streamed in FP32; H, T, exp, combination in FP64 */

/* Limits. */
#define KP_MMAX 64   /* largest Krylov dimension m_max */
#define KP_PMAX 8    /* largest number of phi terms p  */

/*
 * Operator description, copied at call time.  Grid point (ix, iy) is vector
 * index iy*nx + ix; neighbours wrap periodically.  Lap = 5-point Laplacian
 * with spacings dx, dy; Dx, Dy = centred first differences.  For the
 * Brusselator the state vector is [u-plane; v-plane] (N = 2 nx ny) and the
 * operator is the Jacobian of
 *     u' = nu Lap u + brus_a - (brus_b + 1) u + u^2 v,
 *     v' = nu2 Lap v + brus_b u - u^2 v     at (u, v) = (field0, field1).
 * transpose != 0 applies A^T instead of A.  field0/field1 are device arrays of
 * nx*ny doubles (field0 optional for KP_OP_ADR: pass NULL for none).
 */
typedef struct kp_op {
    int32_t kind;
    int32_t nx, ny;
    int32_t transpose;
    double dx, dy;
    double nu, nu2;
    double ax, ay;
    double react;
    double brus_a, brus_b;
    const double* field0;
    const double* field1;
} kp_op;

/* Context configuration.  Zero-initialise and set what you need; zero fields
 * take the defaults given. */
typedef struct kp_config {
    void*   stream;          /* hipStream_t; NULL = the null stream            */
    int32_t orth;            /* KP_ORTH_*, default KP_ORTH_H_GSMGS            */
    int32_t basis_dtype;     /* KP_BASIS_*, default KP_BASIS_F64              */
    int32_t m_init;          /* first Krylov dimension of the adaptive controller;
                                0 -> min(16, m_max)                             */
    int32_t max_substeps;    /* 0 -> 2000                                     */
    int32_t fixed_m;         /* >0: every substep uses exactly this m          */
    int32_t fixed_substeps;  /* with fixed_m: number of equal substeps (>=1)   */
    double  fallback_delta;  /* exact norm replaces the estimate when
                                ||w||^2 - ss <= delta ||w||^2; 0 -> 1e-10,
                                negative -> 0 (the printed rule)              */
    double  breakdown_eps;   /* lucky breakdown when ||v|| <= eps ||A v_j||;
                                0 -> 1e-12                                     */
    double  tau_init;        /* first substep length of the adaptive controller;
                                0 -> h (clipped to h)                           */
    int32_t controller;      /* KP_CTRL_*, default KP_CTRL_POWER              */
    int32_t rows_per_wg;     /* grid rows owned by each workgroup of a single
                                call; 0 -> automatic (at least 4096 elements per
                                workgroup, one workgroup per CU at most).  A
                                smaller value spreads a small grid over more
                                CUs (raised to what the CU count needs).      */
} kp_config;

/* Outcome of a call (filled after the stream is synchronised). */
typedef struct kp_info {
    int32_t status;          /* KP_STATUS_* */
    int32_t substeps;        /* accepted substeps */
    int32_t rejected;        /* rejected trials (m growth or tau reduction) */
    int32_t arnoldi_steps;   /* Arnoldi steps = operator applications */
    int32_t expm_evals;      /* small exponentials evaluated */
    int32_t m_last;          /* Krylov dimension of the last substep */
    int32_t n_fallback;      /* steps where the exact norm replaced the estimate */
    int32_t breakdowns;      /* lucky breakdowns */
    int32_t schedule_len;    /* entries available through kp_get_schedule */
    int32_t onchip_passes;   /* vector passes (N elements each) of the two-pass
                                count of Algorithm 4 that stayed in LDS: where
                                each workgroup's rows fit one sub-tile (one
                                plane, at most 4096 elements and rows of at
                                most 2048, a one-reduction form) the update
                                takes x_j and w from the matvec pass before
                                it, that pass reads the updated x_{j+1} from
                                LDS, and w is never stored; 0 otherwise */
    double  err_max;         /* largest substep error estimate */
    double  mu;              /* power-of-two balance of the augmented block */
    double  t_end;           /* time reached (h on success) */
} kp_info;

typedef struct kp_ctx kp_ctx;

/* Create a context bound to cfg->stream (cfg may be NULL for defaults).
 * Allocates nothing on the device until the first call that needs memory.
 * Errors: KP_EINVAL (out == NULL or an option out of range). */
int kp_create(kp_ctx** out, const kp_config* cfg);

/* Free the context's device workspace (after synchronising its stream). */
int kp_destroy(kp_ctx* ctx);

/* Replace the configuration (same validation as kp_create). */
int kp_set_config(kp_ctx* ctx, const kp_config* cfg);

/*
 * out[0..N) = sum_{k=0}^{p} h^k phi_k(h A) b_k.
 *   B    : device, N x (p+1) column-major, leading dimension ldb >= N,
 *          columns b_0..b_p.  N = nx*ny (x2 for the Brusselator).
 *   out  : device, N doubles, must not overlap B or the operator fields.
 *   tol  : relative accuracy target of the adaptive substep controller
 *          (ignored with a fixed schedule); tol > 0.
 *   m_max: Krylov dimension cap, 1 <= m_max <= KP_MMAX.
 *   info : optional; when non-NULL the stream is synchronised and filled.
 * The whole call (staging, every Arnoldi step, small exponentials, substep
 * control, combination) is ONE cooperative kernel launch on the context's
 * stream; control never returns to the host in between.  Asynchronous unless
 * info is requested.  The context grows its workspace on demand.
 * Errors: KP_EINVAL, KP_ENOMEM, KP_EHIP.
 */
int kp_phi_combo(kp_ctx* ctx, const kp_op* A, const double* B, int32_t p,
                 int64_t ldb, double h, double tol, int32_t m_max,
                 double* out, kp_info* info);

/*
 * kp_phi_combo for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same computation, kernels and arguments as kp_phi_combo (the same result to
 * the bit), but the whole workspace (basis, state vector, partial sums, halo
 * rows, control and state blocks, small-exponential scratch) is carved from
 * one static device array of KP_NOALLOC_BYTES per GPU, which the loaded
 * library holds until the process ends; the call makes no allocation.
 * The workspace needs about (m_max + 2) (N + 64 + 128 planes) elements of the
 * basis type plus 8 (N + 64) bytes and ~1.3 MB of fixed blocks (float64 basis,
 * m_max = 64: N up to about 115,000).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other contexts or streams of the process) race and must be ordered by the
 * caller.  The array keeps the last call's contents; each call resets what it
 * reads before writing it.  kp_get_schedule afterwards reads this call's log.
 * The context must be used on the device that was current when it first
 * touched the device.
 * Errors: those of kp_phi_combo except KP_ENOMEM; KP_ETOOLARGE when the
 * workspace exceeds KP_NOALLOC_BYTES (nothing is enqueued).
 */
#define KP_NOALLOC_BYTES (64u << 20)
int kp_phi_combo_noalloc(kp_ctx* ctx, const kp_op* A, const double* B, int32_t p,
                         int64_t ldb, double h, double tol, int32_t m_max, double* out,
                         kp_info* info);

/*
 * Directional derivative of the phi combination with respect to the operator
 * (tangent mode, for gradients with respect to operator coefficients):
 *     out  = sum_{k=0}^{p} h^k phi_k(h A) b_k                (as kp_phi_combo)
 *     dout = d/de sum_{k=0}^{p} h^k phi_k(h (A + e dA)) b_k   at e = 0.
 * With Atilde the augmented matrix of Section 2.1 and Etilde = [[dA, 0], [0, 0]],
 * out and dout are the top blocks of the two halves of exp(h M) [0; z] for the
 * block matrix M = [[Atilde, Etilde], [0, Atilde]] (the block-triangular
 * exponential whose upper-right block is the Frechet derivative of exp, Van
 * Loan, IEEE Trans. Automat. Control 23 (1978)); one Krylov solve of Section 3
 * on vectors of length 2(N + p), substepped and controlled as kp_phi_combo.
 *   A  : KP_OP_ADR or KP_OP_ALLEN_CAHN (one species plane).
 *   dA : same kind, grid and transpose flag as A; its nu, ax, ay, react give
 *        the direction (dA = nu Lap - ax Dx - ay Dy + react I; transposed with
 *        A); field0/field1 must be NULL.
 *   p  : 0 <= 2p <= KP_PMAX.
 *   out, dout: device, N doubles each, disjoint from B, the fields and each other.
 * Errors: KP_EINVAL, KP_EUNSUPPORTED (other kinds, fields in dA, p too large),
 * KP_ENOMEM, KP_EHIP.
 */
int kp_phi_combo_tangent(kp_ctx* ctx, const kp_op* A, const kp_op* dA, const double* B,
                         int32_t p, int64_t ldb, double h, double tol, int32_t m_max,
                         double* out, double* dout, kp_info* info);

/*
 * Gradients of a loss L(y) of the phi combination y = sum_k h^k phi_k(h A) b_k
 * (kp_phi_combo's arguments A, B, p, ldb, h, tol, m_max), given g = dL/dy:
 *   grad_B[:, k]  = h^k phi_k(h A^T) g,  k = 0..p: the phi combination of the
 *                   transposed operator with B = [0, ..., 0, g] (the phi
 *                   functions of A^T are the transposes of those of A);
 *                   p + 1 solves as in kp_phi_combo.
 *   grad_coef[c]  = <g, dy/dtheta_c> for every bit c of coef_mask, theta =
 *                   (nu, ax, ay, react) (bits 0..3), with the unit direction
 *                   L of that coefficient (Lap, -Dx, -Dy or I; transposed
 *                   with A), then a fixed-order device inner product.  For a
 *                   constant-coefficient ADR operator (no field) L and A
 *                   commute (both circulant) and dy/dtheta is one phi
 *                   combination of A with the p+2 right-hand sides
 *                   c_j = h L b_j - (j-1) L b_{j-1} (from phi_k' = phi_k -
 *                   k phi_{k+1}); otherwise one kp_phi_combo_tangent solve.
 *   g       : device, N doubles.
 *   grad_B  : device, N x (p+1) column-major with leading dimension
 *             ldgb >= N, or NULL (no B-gradient); disjoint from B and g.
 *   grad_coef: device, 4 doubles (entries of unset bits untouched), NULL
 *             only when coef_mask = 0.
 *   Coefficient gradients need KP_OP_ADR or KP_OP_ALLEN_CAHN, and p + 1 <=
 *   KP_PMAX (constant-coefficient ADR) or 2p <= KP_PMAX (otherwise).
 *   info    : optional; when non-NULL every solve is synchronised and info
 *             gets the worst status and the summed work of all the solves.
 * Asynchronous unless info is requested; no tape of the forward call is
 * needed (the solves recompute what they need).  The context keeps a
 * workspace of at most (2p + 5) N doubles for it.
 * Errors: KP_EINVAL, KP_EUNSUPPORTED, KP_ENOMEM, KP_EHIP.
 */
int kp_phi_combo_backward(kp_ctx* ctx, const kp_op* A, const double* B, int32_t p,
                          int64_t ldb, double h, double tol, int32_t m_max, const double* g,
                          double* grad_B, int64_t ldgb, int32_t coef_mask, double* grad_coef,
                          kp_info* info);

/*
 * Many independent phi combinations in one call (the uneven-batch form):
 *     out[i][0..N_i) = sum_{k=0}^{p_i} h_i^k phi_k(h_i A_i) b_{i,k},  i < nprob,
 * each computed exactly as kp_phi_combo computes it (Section 3's hybrid
 * low-synchronisation Arnoldi, Section 2.1's augmented matrix, the adaptive
 * substeps of the KIOPS-type controller), with the context's configuration
 * and the common tol and m_max.
 *   ops, B, p, ldb, h, out: host arrays of nprob entries; B[i] and out[i] are
 *          device pointers with the layouts of kp_phi_combo; ops[i].field*
 *          are device pointers.  Outputs of different problems must not
 *          overlap.
 *   infos: optional host array of nprob records; when non-NULL the stream is
 *          synchronised and filled.  A problem that did not finish reports
 *          KP_STATUS_ABORTED.
 * The grid of one cooperative launch is split into teams of workgroups; a
 * team solves its problems one after another with its own barriers.  Every
 * problem keeps its own basis and state vector for the launch (device memory
 * ~ sum_i (N_i + padding) (m_max + 3) elements of the basis type), so that no
 * cache line written by one workgroup is handed to another during the launch.
 * The
 * team sizes and the problem-to-team assignment come from the built-in
 * planner (see kp_batch_plan), computed when the set of problem shapes
 * (kind, nx, ny, p per problem, nprob, m_max, configuration) differs from the
 * previous batched call on this context; the plan, the workspace and a HIP
 * graph (reset kernel -> batched kernel -> outcome records) are kept and the
 * graph is replayed while the shapes repeat.  The Args of every call
 * (pointers, coefficients, h, tol) are copied to the device before the
 * replay, so they may change between calls.  Asynchronous unless infos is
 * requested.
 * Errors: KP_EINVAL, KP_ENOMEM, KP_EHIP.
 */
int kp_phi_combo_batched(kp_ctx* ctx, int32_t nprob, const kp_op* ops,
                         const double* const* B, const int32_t* p, const int64_t* ldb,
                         const double* h, double tol, int32_t m_max,
                         double* const* out, kp_info* infos);

/*
 * Exponential integrators (Section 4.1) for u' = f(u) on a periodic grid,
 * each step one or two phi combinations of the Jacobian J_n = f'(u_n):
 *   KP_EPI4, KP_EPI5 (multistep, the coefficient matrices A_4, A_5 printed
 *     in Section 4.1; P = 2, 3 previous states):
 *       u_{n+1} = u_n + phi_1(h J_n) h f_n + sum_m phi_m(h J_n) v_m,
 *       v_m = sum_i alpha_{m,i} h R(u_{n-i}),  R(v) = f(v) - f_n - J_n (v - u_n);
 *     one kp_phi_combo per step (b_1 = f_n, b_m = v_m / h^m).  The first P
 *     steps are SRERK3 steps, each taken as start_substeps equal substeps.
 *   KP_SRERK3: z = u_n + phi_1(3/4 h J_n) 3/4 h f_n,
 *       u_{n+1} = u_n + phi_1(h J_n) h f_n + phi_3(h J_n) 32/9 h R(z):
 *     two calls per step.
 * Right-hand sides (kp_rhs, second-order differences as the operators):
 *   KP_RHS_ALLEN_CAHN  f = nu Lap u + u - u^3 (J: KP_OP_ALLEN_CAHN, field u_n)
 *   KP_RHS_ADR         f = nu Lap u - ax Dx u - ay Dy u + gamma u (u - 1/2)(1 - u)
 *                      (J: KP_OP_ADR with the field gamma (-3 u_n^2 + 3 u_n - 1/2))
 *   u     : device, nx*ny doubles: the initial state, overwritten with the state
 *           after nsteps steps of size dt.
 *   tol, m_max: of every phi combination (the context's configuration applies:
 *           orthogonalisation, controller, basis type, fixed schedule).
 *   start_substeps: >= 1 (EPI only).
 *   info  : optional; when non-NULL every call is synchronised and info gets
 *           the worst status and the summed work of all the phi combinations.
 * The context keeps a workspace of about (2P + M + 6) N doubles for it.
 * Errors: KP_EINVAL, KP_ENOMEM, KP_EHIP.
 */
#define KP_RHS_ALLEN_CAHN 0
#define KP_RHS_ADR        1
#define KP_EPI4   0
#define KP_EPI5   1
#define KP_SRERK3 2

typedef struct kp_rhs {
    int32_t kind;
    int32_t nx, ny;
    int32_t reserved;
    double dx, dy;
    double nu, ax, ay, gamma;
} kp_rhs;

int kp_integrate(kp_ctx* ctx, const kp_rhs* f, int32_t method, double dt, int32_t nsteps,
                 int32_t start_substeps, double* u, double tol, int32_t m_max, kp_info* info);

/* Copy the (tau, m) of the accepted substeps of problem i of the last batched
 * call into host arrays of capacity cap; returns the number copied (>= 0) or
 * a KP_E code (KP_ESTATE: no batched call yet; KP_EINVAL: i out of range). */
int kp_get_batch_schedule(kp_ctx* ctx, int32_t i, double* tau_host, int32_t* m_host,
                          int32_t cap);

/*
 * The planner of kp_phi_combo_batched on its own (host only; no device call,
 * the operators' field pointers are only tested for NULL).  For a grid of
 * n_wg workgroups it returns the teams (team_wg0[t], team_size[t],
 * t < *nteams; arrays of capacity n_wg), the team of every problem
 * (team_of_problem, nprob entries), the predicted makespan and the predicted
 * single-workgroup time of all problems (work; may be NULL), in seconds.
 * Cost model: Arnoldi steps ~ max(16, 8 sqrt(h rho)) with rho a bound of
 * ||A||; streaming bytes per step ~ 8 N (m + p + c + 6); a serial cost per
 * step and per small exponential; problems, heaviest first, go to the team
 * that finishes them earliest, over a search of team-size mixes.
 * Errors: KP_EINVAL.
 */
int kp_batch_plan(int32_t nprob, const kp_op* ops, const int32_t* p, const double* h,
                  int32_t m_max, int32_t n_wg, int32_t* team_of_problem, int32_t* team_wg0,
                  int32_t* team_size, int32_t* nteams, double* makespan, double* work);

/*
 * Calibration of kp_batch_plan's cost model on this device (the batched
 * call's autotuner): the small exponential's time at m = 64 is measured
 * directly, and the streaming rate of one workgroup with the whole grid
 * streaming, the serial time per Arnoldi step, per step of a multi-workgroup
 * team and per doubling of a team come from a least-squares fit of the model
 * to seven fixed-schedule advection-diffusion solves (one substep, m = 8..24,
 * 64 x 64 to 2048 x 1024 grids, one to 256 workgroups).  The context's later
 * batched calls plan with the result.  With the environment variable
 * KP_AUTOTUNE_CACHE naming a file, a cached result for this device (GPU
 * architecture, CU count, library version) is read instead of measuring
 * unless force != 0, and a measured one is stored there.
 *   model_host: optional, 5 doubles: bytes/s per workgroup, serial seconds
 *               per step, per team step, per team doubling, and seconds per
 *               small exponential at m = 64.
 * Returns 0 (measured) or 1 (read from the cache), or a KP_E code.  About
 * 0.1 s of device work on the context's stream; synchronises it.
 */
int kp_calibrate(kp_ctx* ctx, int32_t force, double* model_host);

/* Copy the (tau_i, m_i) of the accepted substeps of the last call into host
 * arrays of capacity cap; returns the number copied (>= 0) or a KP_E code. */
int kp_get_schedule(kp_ctx* ctx, double* tau_host, int32_t* m_host, int32_t cap);

/*
 * Step-by-step Arnoldi (Algorithm 4) for inspection and tests.
 * kp_arnoldi_begin stages z = [b_0; mu e_p] for (A, B, p) and resets the
 * process with capacity m_max; kp_arnoldi_step advances it by nsteps steps
 * (fewer on lucky breakdown; each call is one launch of the same persistent
 * kernel, paused at a step boundary); kp_arnoldi_read synchronises and copies:
 *   H_host    : (m_max+1) x m_max column-major (may be NULL),
 *   V_host    : (N+p) x (j+1) column-major unit basis vectors, the last one
 *               normalised by its exact norm (may be NULL),
 *   j_host    : number of completed steps, beta_host: ||z||,
 *   flags_host: [breakdown, n_fallback] (may be NULL).
 */
int kp_arnoldi_begin(kp_ctx* ctx, const kp_op* A, const double* B, int32_t p,
                     int64_t ldb, int32_t m_max);
int kp_arnoldi_step(kp_ctx* ctx, int32_t nsteps);
int kp_arnoldi_read(kp_ctx* ctx, double* H_host, double* V_host, int32_t* j_host,
                    double* beta_host, int32_t* flags_host);

/*
 * Small phi evaluation on its own, for tests: F = exp(tau * Hbar) e_1 with the
 * (m+1) x (m+1) matrix Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]] read from the
 * host array H_host ((m+1) x m column-major, leading dimension ldh >= m+1).
 * Runs the device's small-exponential routine (degree-19 Taylor polynomial
 * with scaling and squaring) in one workgroup and copies F (m+1 doubles) to
 * F_host.
 */
int kp_expm_hbar(kp_ctx* ctx, const double* H_host, int32_t ldh, int32_t m,
                 double tau, double* F_host);

/*
 * Practical HBM read rate, for reporting a kernel's bandwidth against what
 * streaming reads reach (diagnostic; allocates and frees a buffer of `bytes`
 * device bytes, 1 MiB..64 GiB).  One workgroup of 512 threads per compute
 * unit, the persistent kernels' launch shape, reads the buffer with 16-byte
 * loads, four in flight per thread; *gbps_host = bytes / median time of
 * `reps` (1..1000) launches after one warm-up, in GB/s (1e9 B/s).  On the
 * context's stream; synchronises it.
 */
int kp_read_bandwidth(kp_ctx* ctx, int64_t bytes, int32_t reps, double* gbps_host);

/*
 * Device timeline of single calls, for profiling (the library built with
 * KP_TIMELINE, libkrylov_phi_timeline.so; the default build returns
 * KP_EUNSUPPORTED and records nothing).  During every later kp_phi_combo on
 * ctx, thread 0 of each workgroup w < workgroups (kp_timeline_layout) stores
 * the GPU's 100 MHz constant clock at fixed points of phase k < kmax into
 * ts[(k * workgroups + w) * slots + slot] (device memory, int64, owned by
 * the caller, at least kmax * workgroups * slots entries; entries that no
 * workgroup reaches keep their value).  Slots: 0 phase start; 1 the basis
 * update done and its stores complete; 2 the neighbours' halo flags seen;
 * 3 the streaming part done; 4 the release seen (workgroup 0: the phase
 * code phase * 1000 + j, phases numbered as in the kernel: 0 start vector,
 * 1 Arnoldi step, 2 close, 3 small exponential, 4 combination, 5 finish,
 * 7 and 8 matvec and projection of MGS / ioCGS); 5 workgroup 0's reduction
 * done; 6 its serial work done; 7 its release published.  The points sit at
 * existing barriers, so recording adds no synchronisation.  kmax = 0 stops
 * recording.
 */
int kp_set_timeline(kp_ctx* ctx, long long* ts, int32_t kmax);

/* Slots per workgroup and workgroups of the timeline layout; returns 1 when
 * the library records timelines (KP_TIMELINE build), else 0. */
int kp_timeline_layout(int32_t* slots_host, int32_t* workgroups_host);

/* Static description of a return code. */
const char* kp_strerror(int code);

/* Text of the last KP_EHIP error on this context (or "" ). */
const char* kp_last_error(kp_ctx* ctx);

/* Library version, major*10000 + minor*100 + patch. */
int kp_version(void);

/* Versions of the HIP runtime and driver this library is bound to in the
 * calling process (hipRuntimeGetVersion, hipDriverGetVersion), for reports:
 * a process that loads another copy of the runtime first (PyTorch ships one)
 * binds the library to that copy.  Either pointer may be NULL.
 * Errors: KP_EHIP. */
int kp_runtime_version(int32_t* runtime_host, int32_t* driver_host);

#ifdef __cplusplus
}
#endif

#endif /* KRYLOV_PHI_H */
