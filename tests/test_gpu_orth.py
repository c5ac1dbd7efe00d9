"""Parity of the comparator processes with the CPU oracle: modified
Gram-Schmidt (Algorithm 1, one grid-wide reduction per inner product) and the
incomplete classical Gram-Schmidt over the previous two vectors (ioCGS,
Section 2.3.1), run by the same persistent kernel and controller as the
one-reduction forms; the PI substep controller; small grids spread over many
workgroups."""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import arnoldi, closed_form, krylov, phi
import paper_2410_14917_amd as kp

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


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


CASES = [
    (W.OP_ADR, 37, 29, 3),          # one workgroup, ragged tail
    (W.OP_ALLEN_CAHN, 96, 70, 2),   # two workgroups
    (W.OP_BRUSSELATOR, 130, 97, 1), # several workgroups, two species
    (W.OP_ADR, 300, 257, 0),        # 38 workgroups, no augmentation
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("orth", ["mgs", "iocgs"])
def test_arnoldi_steps_match_oracle(case, orth):
    """H and V after 5 steps and after m = 30 (a paused and resumed launch)
    against the oracle's process of the same kind."""
    kind, nx, ny, p = case
    say(f"arnoldi {orth} kind={kind} {nx}x{ny} p={p}")
    pr = W.random_problem(7, kind=kind, nx=nx, ny=ny, p=p, with_diag=True, react=0.2)
    m = 30
    op, B = dev(pr)
    mu = krylov.balance_scale(pr.B, p)
    apply = lambda x: krylov.aug_apply(pr.op, pr.B, p, mu, x)
    z = krylov.start_vector(pr.B, p, mu)
    with kp.Context(orth=orth) as ctx:
        ctx.arnoldi_begin(op, B, m)
        ctx.arnoldi_step(5)
        r5 = ctx.arnoldi_read()
        ctx.arnoldi_step(m - 5)
        r = ctx.arnoldi_read()
    ref = (arnoldi.MGSArnoldi(apply, z, m) if orth == "mgs"
           else arnoldi.IOPArnoldi(apply, z, m, window=2))
    ref.extend(5)
    assert r5["j"] == 5
    assert rel(r5["H"][:6, :5], ref.H[:6, :5]) <= 1e-12
    ref.extend(m)
    assert r["j"] == m and not r["breakdown"]
    assert r["beta"] == pytest.approx(ref.beta, rel=1e-13)
    eH = rel(r["H"][:m + 1, :m], ref.H[:m + 1, :m])
    eV = rel(r["V"], ref.V[:, :m + 1])
    say(f"  H rel {eH:.2e}  V rel {eV:.2e}")
    assert eH <= 1e-11 and eV <= 1e-10
    V = r["V"]
    loss = np.linalg.norm(np.eye(m + 1) - V.T @ V, 2)
    if orth == "mgs":
        assert loss <= 1e-12
        assert np.allclose(np.tril(r["H"][:m + 1, :m], -2), 0.0)
    else:
        # two-vector window: H is tridiagonal, each vector orthogonal to its
        # window, but not to the whole basis
        assert np.allclose(np.triu(r["H"][:m + 1, :m], 2), 0.0)
        for j in range(1, m + 1):
            assert np.all(np.abs(V[:, max(0, j - 2):j].T @ V[:, j]) <= 1e-12)
    assert r["n_fallback"] == 0


FIXED = [
    (W.OP_ADR, 64, 64, 3, 40, 1),
    (W.OP_ALLEN_CAHN, 80, 72, 2, 32, 2),
    (W.OP_BRUSSELATOR, 50, 41, 2, 24, 2),
    (W.OP_ADR, 128, 100, 8, 16, 4),
]


@pytest.mark.parametrize("case", FIXED)
@pytest.mark.parametrize("orth,oorth", [("mgs", "mgs"), ("iocgs", "iop")])
def test_phi_combo_fixed_schedule(case, orth, oorth):
    kind, nx, ny, p, m, nsub = case
    say(f"fixed {orth} kind={kind} {nx}x{ny} p={p} m={m} nsub={nsub}")
    pr = W.random_problem(11, kind=kind, nx=nx, ny=ny, p=p, h=0.05, with_diag=True)
    op, B = dev(pr)
    with kp.Context(orth=orth, fixed_m=m, fixed_substeps=nsub) as ctx:
        y, info = ctx.phi_combo(op, B, pr.h, m_max=m, info=True)
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, pr.h, p, fixed_m=m, fixed_substeps=nsub, m_max=m,
                                  orth=oorth)
    say(f"  rel {rel(y.cpu().numpy(), ref):.2e}")
    assert info["status"] == 0
    assert info["substeps"] == nsub and info["arnoldi_steps"] == rinfo.arnoldi_steps
    assert rel(y.cpu().numpy(), ref) <= FP64_TOL
    # (an estimate far below u ||F|| agrees only to that absolute level)
    assert info["err_max"] == pytest.approx(rinfo.err_max, rel=1e-6,
                                            abs=1e-15 * float(np.abs(ref).max()))


ADAPT = [
    (W.OP_ADR, 48, 40, 3, 1e-8, 24, 0.1, 0.1),
    (W.OP_ALLEN_CAHN, 128, 128, 2, 1e-8, 64, 0.1, 0.01),
    (W.OP_BRUSSELATOR, 64, 64, 2, 1e-6, 32, 0.01, 0.02),
]


def _adaptive(case, orth, oorth, controller):
    kind, nx, ny, p, tol, m_max, h, nu = case
    pr = W.random_problem(13, kind=kind, nx=nx, ny=ny, p=p, h=h, nu=nu, react=-0.5)
    op, B = dev(pr)
    with kp.Context(orth=orth, controller=controller) as ctx:
        y, info = ctx.phi_combo(op, B, h, tol=tol, m_max=m_max, info=True)
        sched = ctx.schedule()
    ref, rinfo = krylov.phi_combo(pr.op, pr.B, h, p, tol=tol, m_max=m_max, orth=oorth,
                                  controller=controller)
    say(f"  gpu substeps={info['substeps']} rejected={info['rejected']} "
        f"oracle substeps={rinfo.substeps} rejected={rinfo.rejected}")
    assert info["status"] == 0 and info["t_end"] == h
    assert [s[1] for s in sched] == [s[1] for s in rinfo.schedule]
    assert np.allclose([s[0] for s in sched], [s[0] for s in rinfo.schedule], rtol=0,
                       atol=1e-6 * h)
    assert info["rejected"] == rinfo.rejected
    assert rel(y.cpu().numpy(), ref) <= FP64_TOL


@pytest.mark.parametrize("case", ADAPT)
@pytest.mark.parametrize("orth,oorth", [("mgs", "mgs"), ("iocgs", "iop")])
def test_phi_combo_adaptive(case, orth, oorth):
    say(f"adaptive {orth} kind={case[0]} {case[1]}x{case[2]}")
    _adaptive(case, orth, oorth, "power")


@pytest.mark.parametrize("case", ADAPT)
@pytest.mark.parametrize("orth,oorth", [("h-gsmgs", "hybrid"), ("mgs", "mgs")])
def test_pi_controller_matches_oracle(case, orth, oorth):
    """The PI substep controller: the same decisions and step sizes as the
    oracle's, and the same result."""
    say(f"PI {orth} kind={case[0]} {case[1]}x{case[2]}")
    _adaptive(case, orth, oorth, "pi")


def test_pi_controller_against_closed_form():
    op_h = W.Operator(kind=W.OP_ADR, nx=96, ny=80, nu=0.05, ax=1.0, ay=0.5, react=-0.5)
    Bh = np.random.default_rng(17).standard_normal((op_h.n, 4))
    ref = closed_form.adr_phi_combo(op_h, Bh, 0.1, 3)
    op = kp.Operator.from_host(op_h)
    B = torch.as_tensor(np.ascontiguousarray(Bh.T), device="cuda")
    for orth in ("h-gsmgs", "mgs", "iocgs"):
        for tol in (1e-6, 1e-10):
            with kp.Context(orth=orth, controller="pi") as ctx:
                y, info = ctx.phi_combo(op, B, 0.1, tol=tol, m_max=32, info=True)
            assert info["status"] == 0 and info["substeps"] >= 2
            assert rel(y.cpu().numpy(), ref) <= 10 * tol, (orth, tol)


@pytest.mark.parametrize("orth", ["h-gsmgs", "h-cwy", "h-ncwy", "mgs", "iocgs"])
def test_config1_spread_over_64_workgroups(orth):
    """The 64 x 64 advection-diffusion workload (p = 3, m = 40) on one
    workgroup (the default geometry) and with one grid row per workgroup (64
    workgroups, the latency-bound regime): both equal the DFT closed form."""
    pr = W.config1()
    op, B = dev(pr)
    ref = closed_form.adr_phi_combo(pr.op, pr.B, pr.h, pr.p)
    ys = []
    for rows in (0, 1):
        with kp.Context(orth=orth, fixed_m=40, fixed_substeps=1, rows_per_wg=rows) as ctx:
            y, info = ctx.phi_combo(op, B, pr.h, m_max=40, info=True)
        ys.append(y.cpu().numpy())
        assert info["status"] == 0 and info["arnoldi_steps"] == 40
        # ioCGS loses orthogonality, its m = 40 projection is less accurate
        assert rel(ys[-1], ref) <= (1e-12 if orth != "iocgs" else 1e-9), (orth, rows)
    assert rel(ys[1], ys[0]) <= (1e-13 if orth != "iocgs" else 1e-11)


@pytest.mark.parametrize("orth", ["mgs", "iocgs"])
def test_lucky_breakdown_diagonal_operator(orth):
    """MGS on a diagonal operator with p = 2 (invariant after d + p steps);
    ioCGS with p = 0 (symmetric: the window is the Lanczos recurrence, so its
    breakdown is exact too)."""
    d_vals = np.array([-3.0, -1.0, -0.5, 0.2, 1.1])
    nx, ny = 70, 40
    diag = d_vals[np.random.default_rng(12).integers(0, len(d_vals), nx * ny)]
    op_h = W.Operator(kind=W.OP_ADR, nx=nx, ny=ny, field0=diag)
    p = 2 if orth == "mgs" else 0
    Bh = np.random.default_rng(13).standard_normal((op_h.n, p + 1))
    ref = phi.phi_combo_diag(diag, Bh, 0.3, p)
    op = kp.Operator.from_host(op_h)
    B = torch.as_tensor(np.ascontiguousarray(Bh.T), device="cuda")
    with kp.Context(orth=orth) as ctx:
        y, info = ctx.phi_combo(op, B, 0.3, tol=1e-10, m_max=20, info=True)
    assert info["breakdowns"] >= 1 and info["m_last"] == len(d_vals) + p
    assert rel(y.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("orth", ["mgs", "iocgs"])
def test_edge_cases(orth):
    """h = 0 returns b_0; a zero start vector gives zero; non-finite input is
    reported."""
    pr = W.random_problem(21, nx=20, ny=18, p=2)
    op, B = dev(pr)
    with kp.Context(orth=orth) as ctx:
        y, info = ctx.phi_combo(op, B, 0.0, tol=1e-8, m_max=10, info=True)
        assert np.array_equal(y.cpu().numpy(), pr.B[:, 0]) and info["substeps"] == 0
        Z = torch.zeros((1, pr.op.n), dtype=torch.float64, device="cuda")
        y, info = ctx.phi_combo(op, Z, 0.05, tol=1e-8, m_max=10, info=True)
        assert info["status"] == 0 and float(y.abs().max()) == 0.0
        Bn = B.clone()
        Bn[2, 5] = float("inf")
        y, info = ctx.phi_combo(op, Bn, 0.05, tol=1e-8, m_max=10, info=True)
        assert info["status"] == 2 and bool(torch.isnan(y).all())


def test_full_size_config2_fixed_substep_mgs_and_iocgs():
    """Allen-Cahn 1024^2, one substep of exactly m = 64 (the microbenchmark's
    launch configuration): the GPU's MGS against the oracle's MGS and the
    GPU's ioCGS against the oracle's ioCGS, element by element."""
    pr = W.config2()
    op, B = dev(pr)
    for orth, oorth in (("iocgs", "iop"), ("mgs", "mgs")):
        say(f"full-size cfg2 {orth}: GPU")
        with kp.Context(orth=orth, fixed_m=64, fixed_substeps=1) as ctx:
            y, info = ctx.phi_combo(op, B, pr.h, m_max=64, info=True)
        y = y.cpu().numpy()
        say(f"full-size cfg2 {orth}: oracle")
        ref, _ = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, fixed_m=64, fixed_substeps=1,
                                  m_max=64, orth=oorth)
        say(f"  {orth} rel {rel(y, ref):.3e}")
        assert info["arnoldi_steps"] == 64 and rel(y, ref) <= FP64_TOL
