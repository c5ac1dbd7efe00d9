"""Parity of the HIP library (through the C ABI) with the CPU oracle."""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import arnoldi, closed_form, krylov, operators, phi
import paper_2410_14917_amd as kp

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10          # relative 2-norm parity bound for float64 results


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(pr):
    op = kp.Operator.from_host(pr.op, device="cuda")
    B = torch.as_tensor(np.ascontiguousarray(pr.B[:, :pr.p + 1].T), device="cuda")
    return op, B


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


# ---- small exponential -----------------------------------------------------

def _krylov_H(kind, m, seed):
    pr = W.random_problem(seed, kind=kind, nx=24, ny=20, p=2, with_diag=True)
    mu = krylov.balance_scale(pr.B, pr.p)
    a = arnoldi.MGSArnoldi(lambda x: krylov.aug_apply(pr.op, pr.B, pr.p, mu, x),
                           krylov.start_vector(pr.B, pr.p, mu), m)
    a.extend(m)
    return a.H


@pytest.mark.parametrize("m", [1, 2, 7, 16, 40, 64])
@pytest.mark.parametrize("tau", [1e-4, 0.01, 0.05, 0.2])
def test_expm_matches_oracle_taylor(m, tau):
    say(f"expm m={m} tau={tau}")
    H = _krylov_H(W.OP_ADR, m, 100 + m)
    with kp.Context() as ctx:
        F = ctx.expm_hbar(H, m, tau)
    ref = phi.expm_taylor(tau * krylov.hbar(H, m))[:, 0]
    assert rel(F, ref) <= 1e-12


@pytest.mark.parametrize("scale", [0.5, 8.0, 300.0])
def test_expm_random_hessenberg(scale):
    rng = np.random.default_rng(int(scale * 10))
    m = 48
    H = np.triu(rng.standard_normal((m + 1, m)), -1)
    H[np.arange(m), np.arange(m)] -= 2.0
    with kp.Context() as ctx:
        F = ctx.expm_hbar(H, m, scale / m)
    ref = phi.expm_taylor((scale / m) * krylov.hbar(H, m))[:, 0]
    assert rel(F, ref) <= 1e-11


# ---- Arnoldi steps -----------------------------------------------------------

CASES = [
    (W.OP_ADR, 37, 29, 3),          # one workgroup, ragged tail
    (W.OP_ALLEN_CAHN, 96, 70, 2),   # two workgroups
    (W.OP_BRUSSELATOR, 130, 97, 1), # several workgroups, two species
    (W.OP_ADR, 300, 257, 0),        # 38 workgroups, no augmentation
]
ORTHS = [("h-gsmgs", "gsmgs"), ("h-cwy", "cwy"), ("h-ncwy", "ncwy")]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("orth", ORTHS)
def test_arnoldi_steps_match_oracle(case, orth):
    kind, nx, ny, p = case
    say(f"arnoldi kind={kind} {nx}x{ny} p={p} orth={orth[0]}")
    pr = W.random_problem(7, kind=kind, nx=nx, ny=ny, p=p, with_diag=True, react=0.2)
    m = 30
    op, B = dev(pr)
    mu = krylov.balance_scale(pr.B, p)
    apply = lambda x: krylov.aug_apply(pr.op, pr.B, p, mu, x)
    z = krylov.start_vector(pr.B, p, mu)
    with kp.Context(orth=orth[0]) as ctx:
        ctx.arnoldi_begin(op, B, m)
        ctx.arnoldi_step(5)
        r5 = ctx.arnoldi_read()
        ctx.arnoldi_step(m - 5)
        r = ctx.arnoldi_read()
    hyb = arnoldi.HybridArnoldi(apply, z, m, tform=orth[1])
    hyb.extend(5)
    assert r5["j"] == 5
    assert rel(r5["H"][:6, :5], hyb.H[:6, :5]) <= 1e-12
    hyb.extend(m)
    mgs = arnoldi.MGSArnoldi(apply, z, m)
    mgs.extend(m)
    assert r["j"] == m and not r["breakdown"]
    assert r["beta"] == pytest.approx(mgs.beta, rel=1e-13)
    assert rel(r["H"][:m + 1, :m], hyb.H[:m + 1, :m]) <= 1e-12
    assert rel(r["H"][:m + 1, :m], mgs.H[:m + 1, :m]) <= 1e-11
    V = r["V"]
    assert rel(V, hyb.basis()) <= 1e-10
    assert np.linalg.norm(np.eye(m + 1) - V.T @ V, 2) <= 1e-12
    assert r["n_fallback"] == hyb.n_fallback


# ---- phi_combo, fixed schedule ----------------------------------------------

FIXED = [
    (W.OP_ADR, 64, 64, 3, 40, 1),
    (W.OP_ADR, 45, 33, 0, 20, 3),
    (W.OP_ALLEN_CAHN, 80, 72, 2, 32, 2),
    (W.OP_BRUSSELATOR, 50, 41, 2, 24, 2),
    (W.OP_ADR, 128, 100, 8, 16, 4),
]


@pytest.mark.parametrize("case", FIXED)
@pytest.mark.parametrize("orth", ["h-gsmgs", "h-cwy", "h-ncwy"])
def test_phi_combo_fixed_schedule(case, orth):
    kind, nx, ny, p, m, nsub = case
    say(f"fixed kind={kind} {nx}x{ny} p={p} m={m} nsub={nsub} {orth}")
    pr = W.random_problem(11, kind=kind, nx=nx, ny=ny, p=p, h=0.05, with_diag=True)
    op, B = dev(pr)
    with kp.Context(orth=orth, fixed_m=m, fixed_substeps=nsub) as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, m_max=m, info=True)
        sched = ctx.schedule()
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, p, fixed_m=m, fixed_substeps=nsub, m_max=m)
    assert info["status"] == 0
    assert info["substeps"] == nsub and info["arnoldi_steps"] == rinfo.arnoldi_steps
    assert [s[1] for s in sched] == [s[1] for s in rinfo.schedule]
    assert rel(y.cpu().numpy(), ref) <= FP64_TOL
    # the estimate beta |F_m| is an entry of the small exponential: where it
    # lies far below u ||F|| (no accuracy request here) the two exponential
    # methods agree only to that absolute level, relative to the solution
    assert info["err_max"] == pytest.approx(rinfo.err_max, rel=1e-6,
                                            abs=1e-15 * float(np.abs(ref).max()))


def test_config1_matches_dft_closed_form():
    pr = W.config1()
    op, B = dev(pr)
    with kp.Context(fixed_m=40, fixed_substeps=1) as ctx:
        y = ctx.phi_combo(op, B, pr.h, m_max=40)
    ref = closed_form.adr_phi_combo(pr.op, pr.B, pr.h, pr.p)
    assert rel(y.cpu().numpy(), ref) <= 1e-12


# ---- phi_combo, adaptive ----------------------------------------------------

ADAPT = [
    (W.OP_ADR, 48, 40, 3, 1e-8, 24, 0.1, 0.1),
    (W.OP_ALLEN_CAHN, 128, 128, 2, 1e-8, 64, 0.1, 0.01),
    (W.OP_BRUSSELATOR, 64, 64, 2, 1e-6, 32, 0.01, 0.02),
]


@pytest.mark.parametrize("case", ADAPT)
@pytest.mark.parametrize("orth", [("h-gsmgs", "gsmgs"), ("h-cwy", "cwy")])
def test_phi_combo_adaptive(case, orth):
    kind, nx, ny, p, tol, m_max, h, nu = case
    say(f"adaptive kind={kind} {nx}x{ny} p={p} tol={tol} m_max={m_max} {orth[0]}")
    pr = W.random_problem(13, kind=kind, nx=nx, ny=ny, p=p, h=h, nu=nu, react=-0.5)
    op, B = dev(pr)
    with kp.Context(orth=orth[0]) as ctx:
        y, info = ctx.phi_combo(op, B, h, tol=tol, m_max=m_max, info=True)
        sched = ctx.schedule()
    # the oracle runs the same algorithm (Algorithm 4 with the same T)
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, h, p, tol=tol, m_max=m_max, orth="hybrid",
                                  tform=orth[1])
    say(f"  gpu substeps={info['substeps']} rejected={info['rejected']} "
        f"oracle substeps={rinfo.substeps} rejected={rinfo.rejected}")
    say(f"  tau gpu {[s[0] for s in sched]}")
    say(f"  tau ora {[s[0] for s in rinfo.schedule]}")
    assert info["status"] == 0 and info["t_end"] == h
    # The controller takes the same decisions on both sides.  The step sizes
    # agree to ~1e-7 of h only: the error estimate is the last entry of
    # exp(tau Hbar) e_1, about tol times smaller than its first entry, so the
    # rounding of the Arnoldi process (~1e-15 of the vector) is ~1e-7 of its
    # value; and the last substep, clipped to h - t, inherits the absolute
    # differences of the earlier ones.
    assert [s[1] for s in sched] == [s[1] for s in rinfo.schedule]
    assert np.allclose([s[0] for s in sched], [s[0] for s in rinfo.schedule], rtol=0,
                       atol=1e-6 * h)
    assert info["rejected"] == rinfo.rejected
    assert rel(y.cpu().numpy(), ref) <= FP64_TOL


def test_adaptive_against_closed_form():
    op_h = W.Operator(kind=W.OP_ADR, nx=96, ny=80, nu=0.05, ax=1.0, ay=0.5, react=-0.5)
    rng = np.random.default_rng(17)
    Bh = rng.standard_normal((op_h.n, 4))
    ref = closed_form.adr_phi_combo(op_h, Bh, 0.1, 3)
    op = kp.Operator.from_host(op_h)
    B = torch.as_tensor(np.ascontiguousarray(Bh.T), device="cuda")
    for tol in (1e-6, 1e-10):
        with kp.Context() as ctx:
            y, info = ctx.phi_combo(op, B, 0.1, tol=tol, m_max=32, info=True)
        assert info["status"] == 0 and info["substeps"] >= 2
        assert rel(y.cpu().numpy(), ref) <= 10 * tol


# ---- edge cases -------------------------------------------------------------

def test_h_zero_returns_b0():
    pr = W.random_problem(21, nx=20, ny=18, p=2)
    op, B = dev(pr)
    with kp.Context() as ctx:
        y, info = ctx.phi_combo(op, B, 0.0, tol=1e-8, m_max=10, info=True)
    assert np.array_equal(y.cpu().numpy(), pr.B[:, 0]) and info["substeps"] == 0


def test_nonfinite_input_reported():
    pr = W.random_problem(22, nx=20, ny=18, p=2)
    Bh = pr.B.copy()
    Bh[5, 2] = np.inf
    op = kp.Operator.from_host(pr.op)
    B = torch.as_tensor(np.ascontiguousarray(Bh.T), device="cuda")
    with kp.Context() as ctx:
        y, info = ctx.phi_combo(op, B, 0.05, tol=1e-8, m_max=10, info=True)
    assert info["status"] == 2
    assert np.all(np.isnan(y.cpu().numpy()))


def test_zero_input_gives_zero():
    pr = W.random_problem(23, nx=20, ny=18, p=0)
    op = kp.Operator.from_host(pr.op)
    B = torch.zeros((1, pr.op.n), dtype=torch.float64, device="cuda")
    with kp.Context() as ctx:
        y, info = ctx.phi_combo(op, B, 0.05, tol=1e-8, m_max=10, info=True)
    assert info["status"] == 0 and float(y.abs().max()) == 0.0


@pytest.mark.parametrize("orth", ["h-gsmgs", "h-cwy", "h-ncwy"])
def test_lucky_breakdown_diagonal_operator(orth):
    d_vals = np.array([-3.0, -1.0, -0.5, 0.2, 1.1])
    nx, ny = 70, 40
    diag = d_vals[np.random.default_rng(12).integers(0, len(d_vals), nx * ny)]
    op_h = W.Operator(kind=W.OP_ADR, nx=nx, ny=ny, field0=diag)
    p = 2
    Bh = np.random.default_rng(13).standard_normal((op_h.n, p + 1))
    ref = phi.phi_combo_diag(diag, Bh, 0.3, p)
    op = kp.Operator.from_host(op_h)
    B = torch.as_tensor(np.ascontiguousarray(Bh.T), device="cuda")
    with kp.Context(orth=orth) as ctx:
        y, info = ctx.phi_combo(op, B, 0.3, tol=1e-10, m_max=20, info=True)
    assert info["breakdowns"] >= 1 and info["m_last"] == len(d_vals) + p
    assert info["n_fallback"] >= 1
    assert rel(y.cpu().numpy(), ref) <= 1e-12


def test_m_max_one():
    """m = 1: with a loose tolerance it converges; with a tight one the error
    per unit step (h_21 h / tol) cannot be met by shrinking tau, and both sides
    stop with NOT_CONVERGED after the same trials."""
    pr = W.random_problem(24, nx=16, ny=16, p=1, h=1e-3, nu=1e-4, ax=0.0, ay=0.0)
    op, B = dev(pr)
    for tol, status in ((1e-1, 0), (1e-6, 1)):
        with kp.Context() as ctx:
            y, info = ctx.phi_combo(op, B, pr.h, tol=tol, m_max=1, info=True)
        ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, 1, tol=tol, m_max=1)
        assert info["status"] == rinfo.status == status
        assert info["substeps"] == rinfo.substeps and info["rejected"] == rinfo.rejected
        assert rel(y.cpu().numpy(), ref) <= FP64_TOL


def test_small_grids_and_single_row():
    for nx, ny in [(1, 7), (3, 1), (2, 2), (5, 3)]:
        pr = W.random_problem(25, nx=nx, ny=ny, p=2, with_diag=True)
        op, B = dev(pr)
        n = pr.op.n + 2
        with kp.Context(fixed_m=n, fixed_substeps=1) as ctx:
            y = ctx.phi_combo(op, B, pr.h, m_max=n)
        ref = phi.phi_combo_dense(operators.dense(pr.op), pr.B, pr.h, 2)
        assert rel(y.cpu().numpy(), ref) <= 1e-12, (nx, ny)


def test_transpose_operator():
    pr = W.random_problem(26, kind=W.OP_BRUSSELATOR, nx=40, ny=33, p=2)
    opt = pr.op.with_transpose()
    op = kp.Operator.from_host(opt)
    B = torch.as_tensor(np.ascontiguousarray(pr.B.T), device="cuda")
    with kp.Context(fixed_m=24, fixed_substeps=2) as ctx:
        y = ctx.phi_combo(op, B, pr.h, m_max=24)
    ref, _ = krylov.phi_combo(opt, pr.B, pr.h, 2, fixed_m=24, fixed_substeps=2, m_max=24)
    assert rel(y.cpu().numpy(), ref) <= FP64_TOL


def test_deterministic_and_exact_power_of_two_scaling():
    pr = W.random_problem(27, kind=W.OP_ALLEN_CAHN, nx=150, ny=120, p=2)
    op, B = dev(pr)
    with kp.Context() as ctx:
        y1 = ctx.phi_combo(op, B, pr.h, tol=1e-9, m_max=32).cpu().numpy()
        y2 = ctx.phi_combo(op, B, pr.h, tol=1e-9, m_max=32).cpu().numpy()
        y4 = ctx.phi_combo(op, 4.0 * B, pr.h, tol=1e-9, m_max=32).cpu().numpy()
    assert np.array_equal(y1, y2)
    assert np.array_equal(y4, 4.0 * y1)


# ---- FP32 basis (float32 storage and streams, float64 arithmetic) -----------

FP32_TOL = 1e-5           # relative 2-norm bound of the FP32-basis results

FP32_FIXED = [
    (W.OP_BRUSSELATOR, 64, 48, 2, 32, 2),
    (W.OP_ADR, 96, 80, 3, 40, 1),
    (W.OP_ALLEN_CAHN, 80, 72, 2, 32, 2),
]


@pytest.mark.parametrize("case", FP32_FIXED)
def test_fp32_basis_fixed_schedule(case):
    kind, nx, ny, p, m, nsub = case
    say(f"fp32 basis fixed kind={kind} {nx}x{ny} p={p} m={m} nsub={nsub}")
    pr = W.random_problem(31, kind=kind, nx=nx, ny=ny, p=p, h=0.05, with_diag=True)
    op, B = dev(pr)
    with kp.Context(basis="f32", fixed_m=m, fixed_substeps=nsub) as ctx:
        y32, info = ctx.phi_combo(op, B, pr.h, m_max=m, info=True)
    with kp.Context(fixed_m=m, fixed_substeps=nsub) as ctx:
        y64 = ctx.phi_combo(op, B, pr.h, m_max=m)
    ref, _ = krylov.phi_combo(pr.op, pr.B, pr.h, p, fixed_m=m, fixed_substeps=nsub, m_max=m)
    e_ref, e_64 = rel(y32.cpu().numpy(), ref), rel(y32.cpu().numpy(), y64.cpu().numpy())
    say(f"  fp32 basis: rel err vs oracle {e_ref:.2e}, vs fp64 path {e_64:.2e}")
    assert info["status"] == 0 and info["substeps"] == nsub
    assert e_ref <= FP32_TOL and e_64 <= FP32_TOL


# The FP32-basis Brusselator pass takes both species of a grid point together
# (joint sub-tiles): the geometries that reach its other branches.
FP32_BRUSSELATOR = [
    (63, 41, 3, False),    # odd row width: pairs across rows, a padding element per plane; p = 3
    (2051, 4, 1, False),   # rows too wide for the LDS halo copy: coherent halo loads
    (130, 97, 2, True),    # the transposed operator, several workgroups
    (64, 48, 0, False),    # p = 0: no columns of B in the matvec
]


@pytest.mark.parametrize("case", FP32_BRUSSELATOR)
def test_fp32_basis_brusselator_joint_tiles(case):
    nx, ny, p, tr = case
    say(f"fp32 basis brusselator joint tiles {nx}x{ny} p={p} transpose={tr}")
    pr = W.random_problem(33, kind=W.OP_BRUSSELATOR, nx=nx, ny=ny, p=p, h=0.02, nu=0.02)
    opn = pr.op.with_transpose() if tr else pr.op
    op = kp.Operator.from_host(opn)
    B = torch.as_tensor(np.ascontiguousarray(pr.B[:, :p + 1].T), device="cuda")
    with kp.Context(basis="f32", fixed_m=24, fixed_substeps=2) as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, m_max=24, info=True)
    ref, _ = krylov.phi_combo(opn, pr.B[:, :p + 1], pr.h, p, fixed_m=24, fixed_substeps=2,
                              m_max=24)
    e = rel(y.cpu().numpy(), ref)
    ea = float(np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    say(f"  rel err vs oracle {e:.2e}, max-abs {ea:.2e}")
    assert info["status"] == 0 and info["substeps"] == 2
    assert e <= FP32_TOL and ea <= FP32_TOL


def test_fp32_basis_adaptive_brusselator():
    """Brusselator Jacobian (the FP32-basis workload's operator, small grid),
    adaptive, tol 1e-6."""
    pr = W.random_problem(32, kind=W.OP_BRUSSELATOR, nx=96, ny=80, p=2, h=0.01, nu=0.02)
    op, B = dev(pr)
    with kp.Context(basis="f32") as ctx:
        y32, info = ctx.phi_combo(op, B, pr.h, tol=1e-6, m_max=64, info=True)
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, 2, tol=1e-12, m_max=64)
    e = rel(y32.cpu().numpy(), ref)
    say(f"  fp32 basis adaptive: substeps {info['substeps']} rejected {info['rejected']} "
        f"rel err vs oracle(tol 1e-12) {e:.2e}")
    assert info["status"] == 0 and info["t_end"] == pr.h
    assert e <= FP32_TOL


def test_full_size_config2_fixed_substep():
    """Allen-Cahn 1024^2, one substep of exactly m = 64 (the microbenchmark's
    launch configuration), against the oracle element by element."""
    pr = W.config2()
    say("full-size cfg2: GPU")
    op, B = dev(pr)
    with kp.Context(fixed_m=64, fixed_substeps=1) as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, m_max=64, info=True)
    y = y.cpu().numpy()
    say("full-size cfg2: oracle")
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, fixed_m=64, fixed_substeps=1,
                                  m_max=64)
    say(f"  rel={rel(y, ref):.3e} err_est gpu={info['err_max']:.3e} oracle={rinfo.err_max:.3e}")
    assert info["arnoldi_steps"] == 64
    assert rel(y, ref) <= FP64_TOL


def test_full_size_config2_adaptive_against_oracle_replay():
    """The benchmark's adaptive call (Allen-Cahn 1024^2, tol 1e-8, m <= 64, the
    launch configuration bench.py times): the oracle's hybrid Arnoldi
    (H-GSMGS) replaying the GPU's accepted substeps gives the same result
    element by element.  About a minute of CPU work for the oracle."""
    pr = W.config2()
    say("full-size cfg2 adaptive: GPU")
    op, B = dev(pr)
    with kp.Context() as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, tol=pr.tol, m_max=64, info=True)
        sched = ctx.schedule()
    y = y.cpu().numpy()
    say(f"  {info['substeps']} substeps ({info['rejected']} rejected), "
        f"{info['arnoldi_steps']} Arnoldi steps; oracle replay of {len(sched)} substeps")
    assert info["status"] == 0 and info["t_end"] == pr.h and len(sched) == info["substeps"]
    assert abs(sum(t for t, _ in sched) - pr.h) <= 1e-12 * pr.h
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, orth="hybrid", tform="gsmgs",
                                  schedule=sched)
    say(f"  rel err vs oracle replay {rel(y, ref):.3e}")
    assert rinfo.substeps == len(sched)
    assert rel(y, ref) <= FP64_TOL


def test_full_size_fp32_basis_brusselator():
    """The FP32-basis workload at full size (2 x 2048^2 Brusselator Jacobian,
    N = 8,388,608, p = 2, h = 0.01, tol 1e-6, m <= 64): the adaptive FP32-basis
    result against the FP64 path (the task's 1e-5), and one substep at fixed
    m = 64 of both bases against the oracle element by element (every
    workgroup streams several sub-tiles per plane at this size): float64 to
    1e-10, float32 to 1e-5, in the 2-norm and in max |y - ref| / max |ref|."""
    import numpy as np
    pr = W.config3()
    say("full-size cfg3: GPU")
    op, B = dev(pr)
    with kp.Context(basis="f32") as ctx:
        y32, i32 = ctx.phi_combo(op, B, pr.h, tol=pr.tol, m_max=pr.m_max, info=True)
        s32 = ctx.schedule()
    with kp.Context() as ctx:
        y64, i64 = ctx.phi_combo(op, B, pr.h, tol=pr.tol, m_max=pr.m_max, info=True)
        s64 = ctx.schedule()
    e = rel(y32.cpu().numpy(), y64.cpu().numpy())
    say(f"  f32 vs f64 rel {e:.2e} (substeps f32 {i32['substeps']} f64 {i64['substeps']})")
    say(f"  schedule f64 {[(round(t, 6), m) for t, m in s64]}")
    say(f"  schedule f32 {[(round(t, 6), m) for t, m in s32]}")
    assert i32["status"] == 0 and i64["status"] == 0 and e <= FP32_TOL
    fixed = {}
    for basis in ("f64", "f32"):
        with kp.Context(basis=basis, fixed_m=64, fixed_substeps=1) as ctx:
            fixed[basis] = ctx.phi_combo(op, B, pr.h, m_max=64).cpu().numpy()
    say("full-size cfg3: oracle, fixed m = 64")
    ref, _ = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, fixed_m=64, fixed_substeps=1, m_max=64)
    for basis, tol in (("f64", FP64_TOL), ("f32", FP32_TOL)):
        y = fixed[basis]
        r2, ra = rel(y, ref), float(np.abs(y - ref).max() / np.abs(ref).max())
        say(f"  fixed m=64 {basis}: rel {r2:.2e} max-abs {ra:.2e}")
        assert r2 <= tol and ra <= tol


@pytest.mark.parametrize("case", [(W.OP_ADR, 4101, 6, 2), (W.OP_ALLEN_CAHN, 4200, 5, 1),
                                  (W.OP_BRUSSELATOR, 2051, 4, 2)])
def test_wide_grids_halo_rows_through_coherent_loads(case):
    """Grids whose two halo rows per plane do not fit the matvec's LDS copy
    (2 * planes * nx > 8192): the stencil reads them with coherent loads."""
    kind, nx, ny, p = case
    say(f"wide kind={kind} {nx}x{ny}")
    pr = W.random_problem(61, kind=kind, nx=nx, ny=ny, p=p, h=0.02, with_diag=True)
    op, B = dev(pr)
    with kp.Context(fixed_m=24, fixed_substeps=2) as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, m_max=24, info=True)
    ref, _ = krylov.phi_combo(pr.op, pr.B, pr.h, p, fixed_m=24, fixed_substeps=2, m_max=24)
    say(f"  rel {rel(y.cpu().numpy(), ref):.2e}")
    assert info["status"] == 0 and rel(y.cpu().numpy(), ref) <= FP64_TOL


@pytest.mark.parametrize("m_init,tau_init", [(8, 0.0), (32, 0.02), (4, 0.5)])
def test_controller_start_values(m_init, tau_init):
    """m_init and tau_init (tau_init > h is clipped to h): the same decisions
    and result as the oracle with the same start values, single and batched."""
    pr = W.random_problem(81, kind=W.OP_ADR, nx=72, ny=60, p=2, h=0.1, nu=0.05, react=-0.3)
    op, B = dev(pr)
    with kp.Context(m_init=m_init, tau_init=tau_init) as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, tol=1e-8, m_max=48, info=True)
        sched = ctx.schedule()
        (yb,), (ib,) = ctx.phi_combo_batched([op], [B], [pr.h], tol=1e-8, m_max=48, info=True)
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, 2, tol=1e-8, m_max=48, orth="hybrid",
                                  m_init=m_init, tau_init=tau_init)
    say(f"  m_init={m_init} tau_init={tau_init}: first {sched[0]} oracle {rinfo.schedule[0]}")
    assert info["status"] == 0 and ib["status"] == 0
    assert [s[1] for s in sched] == [s[1] for s in rinfo.schedule]
    assert np.allclose([s[0] for s in sched], [s[0] for s in rinfo.schedule], rtol=0,
                       atol=1e-6 * pr.h)
    assert rel(y.cpu().numpy(), ref) <= FP64_TOL and rel(yb.cpu().numpy(), ref) <= FP64_TOL


@pytest.mark.parametrize("delta,oracle_delta", [(1.0, 1.0), (-1.0, 0.0), (1e-4, 1e-4)])
def test_norm_estimate_fallback_settings(delta, oracle_delta):
    """The estimate's fallback threshold: 1.0 takes the exact norm at every
    step (the exact-norm mode, at no extra pass), a negative value the printed
    rule (delta = 0); decisions, fallback counts and results as the oracle's."""
    pr = W.random_problem(91, kind=W.OP_ALLEN_CAHN, nx=64, ny=56, p=2, h=0.05)
    op, B = dev(pr)
    with kp.Context(fallback_delta=delta, fixed_m=32, fixed_substeps=2) as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, m_max=32, info=True)
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, 2, fixed_m=32, fixed_substeps=2, m_max=32,
                                  orth="hybrid", delta=oracle_delta)
    say(f"  delta={delta}: n_fallback gpu {info['n_fallback']} oracle {rinfo.n_fallback}")
    assert info["n_fallback"] == rinfo.n_fallback
    if delta == 1.0:
        assert info["n_fallback"] == info["arnoldi_steps"]         # every step
    assert rel(y.cpu().numpy(), ref) <= FP64_TOL
