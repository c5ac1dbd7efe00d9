"""Pins of oracle/integrators.py (no GPU): the printed EPI coefficient
matrices against the classical order conditions, exactness on a linear
problem, the closed-form solution of the scalar Allen-Cahn ODE, and observed
convergence orders on a small grid."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import workloads as W
from oracle import closed_form, integrators as I


def order_of(alpha, qmax=8):
    """Largest q for which the multistep scheme sum_m phi_m(Z) v_m,
    v_m = h sum_i alpha_{m,i} R(t_n - i h), reproduces the exact remainder
    integral h int_0^1 e^{(1-s)Z} r(t_n + s h) ds = sum_k r_k h^{k+1}
    phi_{k+1}(Z) (variation of constants; r(t_n) = r'(t_n) = 0 for the
    remainder R) up to the terms r_k h^{k+1} Z^l with k + 1 + l <= q, using
    phi_m(Z) = sum_l Z^l / (l + m)!.  Exact rational arithmetic."""
    M, P = len(alpha), len(alpha[0])
    best = 2
    for q in range(3, qmax + 1):
        for k in range(2, q):
            for l in range(0, q - k):
                s = sum(Fr(alpha[m][i]) * Fr((-(i + 1)) ** k, math.factorial(k))
                        / math.factorial(l + m + 1) for m in range(M) for i in range(P))
                if s != Fr(1, math.factorial(l + k + 1)):
                    return best
        best = q
    return best


def test_printed_epi_tables_have_their_order():
    assert order_of(I.EPI_ALPHA[I.EPI4]) == 4
    assert order_of(I.EPI_ALPHA[I.EPI5]) == 5
    # the A_6 of the extracted text fails even the third-order conditions
    a6 = [[0, 0, 0, 0], [Fr(-49, 60), Fr(351, 560), Fr(-359, 12600), Fr(367, 6720)],
          [Fr(97, 7), Fr(-99, 14), Fr(176, 63), Fr(-1, 2)],
          [Fr(485, 21), Fr(-151, 14), Fr(23, 9), Fr(-31, 168)]]
    assert order_of(a6) == 2


def _scalar_ac(side=4, u0=0.3):
    """Allen-Cahn with a spatially constant state: the Laplacian vanishes and
    u' = u - u^3, u(t) = u0 e^t / sqrt(1 + u0^2 (e^{2t} - 1))."""
    rhs = W.Rhs(W.RHS_ALLEN_CAHN, side, side, 1.0 / side, 1.0 / side, nu=0.1)
    exact = lambda t: u0 * math.exp(t) / math.sqrt(1.0 + u0 * u0 * (math.exp(2 * t) - 1.0))
    return rhs, np.full(side * side, u0), exact


@pytest.mark.parametrize("method,q", [(I.EPI4, 4), (I.EPI5, 5), (I.SRERK3, 3)])
def test_scalar_allen_cahn_converges_at_the_method_order(method, q):
    rhs, u0, exact = _scalar_ac()
    T = 1.0
    errs = []
    for nsteps in (10, 20, 40):
        h = T / nsteps
        P = I.history_length(method)
        start = [np.full(rhs.n, exact((k + 1) * h)) for k in range(P)]
        u = I.integrate(rhs, u0, h, nsteps, method, I.dense_solver, start=start)
        errs.append(abs(u[0] - exact(T)))
        assert np.ptp(u) <= 1e-14                 # stays constant in space
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(rates) >= q - 0.35, (errs, rates)


@pytest.mark.parametrize("method", [I.EPI4, I.EPI5, I.SRERK3])
def test_linear_problem_is_propagated_exactly(method):
    """gamma = 0: f(u) = A u, the remainder vanishes and every step is
    u_{n+1} = u_n + h phi_1(hA) A u_n = e^{hA} u_n: the DFT closed form of
    e^{T A} u0 (up to the Krylov tolerance), whatever the start."""
    rhs = W.Rhs(W.RHS_ADR, 24, 20, 1 / 24, 1 / 20, nu=0.02, ax=0.7, ay=-0.4, gamma=0.0)
    u0 = np.random.default_rng(3).standard_normal(rhs.n)
    h, n = 0.05, 6
    u = I.integrate(rhs, u0, h, n, method, I.krylov_solver(tol=1e-13, m_max=40))
    op = W.Operator(kind=W.OP_ADR, nx=rhs.nx, ny=rhs.ny, nu=rhs.nu, ax=rhs.ax, ay=rhs.ay)
    ref = closed_form.adr_phi_combo(op, u0[:, None], h * n, 0)
    assert np.linalg.norm(u - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("method,q", [(I.EPI4, 4), (I.EPI5, 5), (I.SRERK3, 3)])
def test_allen_cahn_pde_converges_at_the_method_order(method, q):
    """The paper's Allen-Cahn problem on a coarse 8 x 8 grid (dense phi
    combinations): errors against a fine-step SRERK3 reference fall at the
    method's order (multistep starts from reference states)."""
    iv = W.ivp_allen_cahn(side=8)
    rhs, u0 = iv.rhs, iv.u0
    T = 0.4
    ref_steps = 1280
    fine = [u0]
    u = u0
    for k in range(ref_steps):
        u = I.srerk3_step(rhs, u, T / ref_steps, I.dense_solver)
        fine.append(u)
    errs = []
    for nsteps in (8, 16, 32):
        h = T / nsteps
        P = I.history_length(method)
        stride = ref_steps // nsteps
        start = [fine[(k + 1) * stride] for k in range(P)]
        y = I.integrate(rhs, u0, h, nsteps, method, I.dense_solver, start=start)
        errs.append(np.linalg.norm(y - fine[-1]))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    # the rate approaches q from below as h falls (pre-asymptotic at h = T/8)
    assert min(rates) >= q - 0.6 and rates[-1] >= q - 0.35, (errs, rates)


def test_srerk3_start_keeps_the_order():
    """EPI4 with its first two steps from SRERK3 substeps (the library's
    start) still converges at fourth order on the scalar problem."""
    rhs, u0, exact = _scalar_ac()
    errs = []
    for nsteps in (10, 20, 40):
        u = I.integrate(rhs, u0, 1.0 / nsteps, nsteps, I.EPI4, I.dense_solver, start_substeps=4)
        errs.append(abs(u[0] - exact(1.0)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(rates) >= 3.6, (errs, rates)


def test_jacobian_is_the_derivative_of_f():
    """Central differences of f along a random direction equal J v for both
    problem kinds."""
    rng = np.random.default_rng(5)
    for rhs in (W.ivp_allen_cahn(side=12).rhs, W.ivp_adr(side=12).rhs):
        u = rng.uniform(0.1, 0.9, rhs.n)
        v = rng.standard_normal(rhs.n)
        eps = 1e-6
        fd = (I.f(rhs, u + eps * v) - I.f(rhs, u - eps * v)) / (2 * eps)
        from oracle import operators
        jv = operators.apply(I.jacobian(rhs, u), v)
        assert np.linalg.norm(fd - jv) <= 1e-7 * np.linalg.norm(jv)
