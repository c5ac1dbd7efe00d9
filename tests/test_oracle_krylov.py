"""Pins of oracle/krylov.py (no GPU): exactness, closed forms, special cases,
linearity and the adaptive controller's accuracy."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_form, krylov, operators, phi


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("kind", [W.OP_ADR, W.OP_ALLEN_CAHN, W.OP_BRUSSELATOR])
@pytest.mark.parametrize("orth", ["mgs", "hybrid"])
def test_exact_when_m_equals_dimension(kind, orth):
    pr = W.random_problem(41, kind=kind, nx=5, ny=4, p=2, h=0.2, with_diag=True)
    n = pr.op.n + pr.p
    ref = phi.phi_combo_dense(operators.dense(pr.op), pr.B, pr.h, pr.p)
    y, info = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, fixed_m=n, fixed_substeps=1,
                               m_max=n, orth=orth)
    assert rel(y, ref) <= 1e-12


def test_config1_matches_dft_closed_form():
    pr = W.config1()
    y, info = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, fixed_m=40, fixed_substeps=1,
                               m_max=40)
    ref = closed_form.adr_phi_combo(pr.op, pr.B, pr.h, pr.p)
    assert rel(y, ref) <= 1e-12


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_adaptive_meets_tolerance_against_closed_form(tol):
    op = W.Operator(kind=W.OP_ADR, nx=48, ny=40, nu=0.1, ax=1.0, ay=0.5, react=-0.5)
    rng = np.random.default_rng(42)
    B = rng.standard_normal((op.n, 4))
    h = 0.1
    ref = closed_form.adr_phi_combo(op, B, h, 3)
    for orth in ("mgs", "hybrid"):
        y, info = krylov.phi_combo(op, B, h, 3, tol=tol, m_max=24, orth=orth)
        assert info.status == krylov.STATUS_OK
        assert info.substeps >= 2             # hrho ~ 190: needs substepping
        assert rel(y, ref) <= 10 * tol


def test_zero_step_returns_b0():
    pr = W.random_problem(43)
    y, _ = krylov.phi_combo(pr.op, pr.B, 0.0, pr.p, tol=1e-8, m_max=10)
    assert np.array_equal(y, pr.B[:, 0])


def test_zero_operator_gives_taylor_weights():
    op = W.Operator(kind=W.OP_ADR, nx=6, ny=5)           # nu = a = r = 0
    rng = np.random.default_rng(44)
    p, h = 4, 0.7
    B = rng.standard_normal((op.n, p + 1))
    ref = sum(h ** k / math.factorial(k) * B[:, k] for k in range(p + 1))
    y, info = krylov.phi_combo(op, B, h, p, tol=1e-12, m_max=10)
    assert rel(y, ref) <= 1e-13
    assert info.breakdowns >= 1


def test_p0_is_plain_exponential_and_semigroup():
    pr = W.random_problem(45, nx=6, ny=5, p=0, h=0.3, with_diag=True)
    A = operators.dense(pr.op)
    ref = phi.expm_taylor(pr.h * A) @ pr.B[:, 0]
    y, _ = krylov.phi_combo(pr.op, pr.B, pr.h, 0, fixed_m=30, fixed_substeps=1, m_max=30)
    assert rel(y, ref) <= 1e-12
    y1, _ = krylov.phi_combo(pr.op, pr.B, 0.1, 0, fixed_m=30, fixed_substeps=1, m_max=30)
    y2, _ = krylov.phi_combo(pr.op, y1[:, None], 0.2, 0, fixed_m=30, fixed_substeps=1,
                             m_max=30)
    assert rel(y2, ref) <= 1e-12


def test_linearity_in_B_is_exact_for_power_of_two_scaling():
    pr = W.random_problem(46, nx=12, ny=10, p=2)
    kw = dict(fixed_m=12, fixed_substeps=2, m_max=12)
    y1, _ = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, **kw)
    y2, _ = krylov.phi_combo(pr.op, 4.0 * pr.B, pr.h, pr.p, **kw)
    assert np.array_equal(y2, 4.0 * y1)


def test_balance_scale_does_not_change_result():
    pr = W.random_problem(47, nx=10, ny=8, p=3)
    kw = dict(fixed_m=40, fixed_substeps=1, m_max=40)
    y1, _ = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, **kw)
    y2, _ = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, mu=1.0, **kw)
    y3, _ = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, mu=1024.0, **kw)
    assert rel(y2, y1) <= 1e-12 and rel(y3, y1) <= 1e-12
    assert krylov.balance_scale(pr.B, pr.p) == 2.0 ** math.floor(
        math.log2(np.max(np.abs(pr.B[:, 1:]))))


def test_nonfinite_input_is_reported():
    pr = W.random_problem(48)
    B = pr.B.copy()
    B[3, 1] = np.nan
    y, info = krylov.phi_combo(pr.op, B, pr.h, pr.p, tol=1e-8, m_max=10)
    assert info.status == krylov.STATUS_NONFINITE


def test_error_estimate_tracks_true_error():
    """The (m+1)-st entry of exp(tau Hbar) e_1 estimates the substep error."""
    pr = W.config1()
    ref = closed_form.adr_phi_combo(pr.op, pr.B, pr.h, pr.p)
    for m in (12, 16, 20):
        y, info = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, fixed_m=m, fixed_substeps=1,
                                   m_max=m)
        err = np.linalg.norm(y - ref)
        assert 0.01 * info.err_max <= err <= 100 * info.err_max


@pytest.mark.parametrize("m_init,tau_init", [(4, 0.0), (48, 0.0), (16, 0.01), (8, 0.2)])
def test_controller_start_values_keep_accuracy(m_init, tau_init):
    """Any first Krylov dimension and first step reach the closed form within
    tol (the controller corrects them); tau_init beyond h is clipped to h."""
    op = W.Operator(kind=W.OP_ADR, nx=48, ny=40, nu=0.05, ax=1.0, ay=0.5, react=-0.3)
    rng = np.random.default_rng(71)
    B = rng.standard_normal((op.n, 3))
    y, info = krylov.phi_combo(op, B, 0.1, 2, tol=1e-9, m_max=48, m_init=m_init,
                               tau_init=tau_init, orth="hybrid")
    assert info.status == 0
    assert np.linalg.norm(y - closed_form.adr_phi_combo(op, B, 0.1, 2)) <= \
        10 * 1e-9 * np.linalg.norm(y)
    if tau_init == 0.0 or tau_init >= 0.1:
        assert info.schedule[0][0] <= 0.1


# ---- replay of a logged schedule -------------------------------------------

def test_replay_of_equal_substeps_is_the_fixed_schedule():
    """Replaying n substeps of h/n with dimension m is the fixed schedule,
    to the bit (the same projections in the same order)."""
    pr = W.random_problem(7, kind=W.OP_ADR, nx=12, ny=10, p=2, h=0.3)
    for orth in ("mgs", "hybrid"):
        y_f, _ = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, fixed_m=12, fixed_substeps=3,
                                  m_max=12, orth=orth)
        y_r, info = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, orth=orth,
                                     schedule=[(pr.h / 3, 12)] * 3)
        assert np.array_equal(y_f, y_r) and info.substeps == 3 and info.arnoldi_steps == 36


def test_replay_of_uneven_substeps_matches_closed_form():
    """Substeps of 0.3 h, 0.5 h and 0.2 h (converged dimension 40) give the
    DFT closed form of the whole step (Section 3: the substeps compose the
    exponential of the augmented matrix)."""
    pr = W.config1()
    h = pr.h
    y, info = krylov.phi_combo(pr.op, pr.B, h, pr.p, orth="hybrid",
                               schedule=[(0.3 * h, 40), (0.5 * h, 40), (0.2 * h, 40)])
    ref = closed_form.adr_phi_combo(pr.op, pr.B, h, pr.p)
    assert info.substeps == 3 and rel(y, ref) <= 1e-12
    # a dropped substep is a different result
    y2, _ = krylov.phi_combo(pr.op, pr.B, h, pr.p, orth="hybrid",
                             schedule=[(0.3 * h, 40), (0.5 * h, 40)])
    assert rel(y2, ref) > 1e-3


def test_replay_of_an_adaptive_schedule_reproduces_the_run():
    """The accepted substeps of an adaptive run (with rejections and growth of
    m), replayed, give the run's result to rounding."""
    pr = W.random_problem(11, kind=W.OP_ADR, nx=24, ny=20, p=2, h=0.5)
    y_a, info_a = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, tol=1e-8, m_max=24,
                                   orth="hybrid")
    assert info_a.substeps >= 2
    y_r, info_r = krylov.phi_combo(pr.op, pr.B, pr.h, pr.p, orth="hybrid",
                                   schedule=info_a.schedule)
    assert info_r.schedule == info_a.schedule
    assert rel(y_r, y_a) <= 1e-13


# ---- ioCGS (Section 2.3.1) and the PI substep controller (Conclusion) -------

@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_iop_adaptive_meets_tolerance_against_closed_form(tol):
    """The incomplete process in the same controller reaches the DFT closed
    form within 10 tol on a non-normal advection-diffusion operator."""
    op = W.Operator(kind=W.OP_ADR, nx=48, ny=40, nu=0.1, ax=1.0, ay=0.5, react=-0.5)
    B = np.random.default_rng(42).standard_normal((op.n, 4))
    ref = closed_form.adr_phi_combo(op, B, 0.1, 3)
    y, info = krylov.phi_combo(op, B, 0.1, 3, tol=tol, m_max=24, orth="iop")
    assert info.status == krylov.STATUS_OK and info.substeps >= 2
    assert rel(y, ref) <= 10 * tol


@pytest.mark.parametrize("orth", ["mgs", "hybrid", "iop"])
@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_pi_controller_meets_tolerance_against_closed_form(orth, tol):
    op = W.Operator(kind=W.OP_ADR, nx=48, ny=40, nu=0.1, ax=1.0, ay=0.5, react=-0.5)
    B = np.random.default_rng(42).standard_normal((op.n, 4))
    ref = closed_form.adr_phi_combo(op, B, 0.1, 3)
    y, info = krylov.phi_combo(op, B, 0.1, 3, tol=tol, m_max=24, orth=orth, controller="pi")
    assert info.status == krylov.STATUS_OK and info.substeps >= 2
    assert rel(y, ref) <= 10 * tol


def test_pi_controller_uses_the_previous_error():
    """The PI factor depends on the previous accepted substep's error: with
    omega_prev = 1 it is the integral part alone; a more accurate previous
    substep (the error growing) gives a smaller factor; clipped to [0.2, 4]."""
    for m in (8, 33, 64):
        for om in (1e-3, 0.3, 0.9):
            f_pow = krylov.step_factor(om, m)
            q = (m + 3) // 4
            assert krylov.step_factor(om, m, 1.0, "pi") == pytest.approx(
                min(4.0, 0.9 * om ** (-0.7 / (q + 1))), rel=1e-15)
            if krylov.step_factor(om, m, 1.0, "pi") < 4.0:
                assert krylov.step_factor(om, m, 0.5, "pi") < krylov.step_factor(om, m, 1.0, "pi")
            assert 0.2 <= f_pow <= 4.0
        assert krylov.step_factor(0.0, m, 0.5, "pi") == 4.0
        assert krylov.step_factor(1e30, m) == 0.2
    # without a previous accepted substep the PI controller is the power law
    assert krylov.step_factor(0.3, 16, 0.0, "pi") == krylov.step_factor(0.3, 16)
