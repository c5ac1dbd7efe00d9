"""The exponential integrators of Section 4.1 (EPI4, EPI5, SRERK3) on the GPU
(kp_integrate: right-hand side and remainder kernels around kp_phi_combo)
against the oracle's integrators with the same start and schedule."""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import closed_form, integrators as I
import paper_2410_14917_amd as kp

pytestmark = pytest.mark.gpu

METHODS = [("epi4", I.EPI4), ("epi5", I.EPI5), ("srerk3", I.SRERK3)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _ivps():
    ac = W.ivp_allen_cahn(side=48)
    adr = W.ivp_adr(side=40)
    return [("allen-cahn", ac), ("adr", adr)]


@pytest.mark.parametrize("name,iv", _ivps())
@pytest.mark.parametrize("method,om", METHODS)
def test_fixed_schedule_matches_oracle(name, iv, method, om):
    """Every phi combination with a fixed schedule (m = 24, two substeps) on
    both sides: the integrated state agrees to rounding."""
    say(f"integrate {method} {name}")
    nsteps, start = 6, 2
    u = torch.as_tensor(iv.u0, device="cuda").clone()
    with kp.Context(fixed_m=24, fixed_substeps=2) as ctx:
        _, info = ctx.integrate(iv.rhs, u, iv.dt, nsteps, method=method, m_max=24,
                                start_substeps=start, info=True)
    solve = I.krylov_solver(fixed_m=24, fixed_substeps=2, m_max=24, orth="hybrid")
    ref = I.integrate(iv.rhs, iv.u0, iv.dt, nsteps, om, solve, start_substeps=start)
    e = rel(u.cpu().numpy(), ref)
    say(f"  rel {e:.2e}  calls' substeps {info['substeps']}")
    assert info["status"] == 0 and e <= 1e-10


@pytest.mark.parametrize("method,om", METHODS)
def test_adaptive_matches_oracle(method, om):
    """The adaptive controller in every call (tol 1e-10, m <= 32): the same
    decisions on both sides, the same state to 1e-9."""
    iv = W.ivp_allen_cahn(side=40)
    u = torch.as_tensor(iv.u0, device="cuda").clone()
    with kp.Context() as ctx:
        _, info = ctx.integrate(iv.rhs, u, iv.dt, 5, method=method, tol=1e-10, m_max=32,
                                start_substeps=2, info=True)
    solve = I.krylov_solver(tol=1e-10, m_max=32, orth="hybrid")
    ref = I.integrate(iv.rhs, iv.u0, iv.dt, 5, om, solve, start_substeps=2)
    e = rel(u.cpu().numpy(), ref)
    say(f"  {method}: rel {e:.2e}, {info['substeps']} substeps {info['arnoldi_steps']} steps")
    assert info["status"] == 0 and e <= 1e-9


@pytest.mark.parametrize("method,om", METHODS)
def test_linear_problem_against_closed_form(method, om):
    """gamma = 0 (f = A u): every method propagates e^{hA} exactly; the DFT
    closed form of e^{T A} u0."""
    rhs = W.Rhs(W.RHS_ADR, 64, 48, 1 / 64, 1 / 48, nu=0.02, ax=0.7, ay=-0.4, gamma=0.0)
    u0 = np.random.default_rng(3).standard_normal(rhs.n)
    u = torch.as_tensor(u0, device="cuda").clone()
    with kp.Context() as ctx:
        ctx.integrate(rhs, u, 0.05, 6, method=method, tol=1e-13, m_max=48)
    op = W.Operator(kind=W.OP_ADR, nx=rhs.nx, ny=rhs.ny, nu=rhs.nu, ax=rhs.ax, ay=rhs.ay)
    ref = closed_form.adr_phi_combo(op, u0[:, None], 0.3, 0)
    assert rel(u.cpu().numpy(), ref) <= 1e-11


def test_scalar_allen_cahn_closed_form():
    """A spatially constant state follows u' = u - u^3 exactly.  EPI5 with its
    SRERK3 start (8 substeps) at h = 1/40: the oracle's scalar integration
    (pinned to converge at fifth order) is 2.4e-9 from the closed form; the
    GPU state equals it to rounding, uniform in space."""
    import math
    side, u0v, T, nsteps = 32, 0.3, 1.0, 40
    rhs = W.Rhs(W.RHS_ALLEN_CAHN, side, side, 1 / side, 1 / side, nu=0.1)
    exact = u0v * math.exp(T) / math.sqrt(1.0 + u0v * u0v * (math.exp(2 * T) - 1.0))
    u = torch.full((side * side,), u0v, dtype=torch.float64, device="cuda")
    with kp.Context() as ctx:
        ctx.integrate(rhs, u, T / nsteps, nsteps, method="epi5", tol=1e-13, m_max=16,
                      start_substeps=8)
    y = u.cpu().numpy()
    small = W.Rhs(W.RHS_ALLEN_CAHN, 4, 4, 1 / 4, 1 / 4, nu=0.1)
    ref = I.integrate(small, np.full(16, u0v), T / nsteps, nsteps, I.EPI5, I.dense_solver,
                      start_substeps=8)[0]
    say(f"  gpu - oracle {y[0] - ref:.2e}, oracle - exact {ref - exact:.2e}")
    assert np.ptp(y) <= 1e-14 and abs(y[0] - ref) <= 1e-13 and abs(y[0] - exact) <= 5e-9


def test_mgs_and_iocgs_inside_the_integrator():
    """The integrator with the comparator orthogonalisations (the paper's
    ioCGS baseline and MGS) reaches the oracle's state too."""
    iv = W.ivp_adr(side=40)
    solve = I.krylov_solver(fixed_m=24, fixed_substeps=2, m_max=24, orth="hybrid")
    ref = I.integrate(iv.rhs, iv.u0, iv.dt, 5, I.EPI4, solve, start_substeps=2)
    for orth in ("mgs", "iocgs"):
        u = torch.as_tensor(iv.u0, device="cuda").clone()
        with kp.Context(orth=orth, fixed_m=24, fixed_substeps=2) as ctx:
            ctx.integrate(iv.rhs, u, iv.dt, 5, method="epi4", m_max=24, start_substeps=2)
        e = rel(u.cpu().numpy(), ref)
        say(f"  {orth}: rel {e:.2e}")
        assert e <= 1e-10
