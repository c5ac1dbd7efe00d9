"""Pins of the oracle's derivatives (oracle/adjoint.py, oracle/closed_form.py).

The directional derivative in the operator is checked against two things that
do not use the block (Van Loan) construction: central differences of the dense
phi combination, and the DFT closed form of the constant-coefficient ADR
operator differentiated by hand.  The B-gradient is checked by the
dot-product test <g, y_k(v)> = <G_k, v>.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, closed_form, krylov, operators, phi


def _adr(nx, ny, nu=0.05, ax=1.0, ay=0.5, react=-0.3):
    return W.Operator(kind=W.OP_ADR, nx=nx, ny=ny, nu=nu, ax=ax, ay=ay, react=react)


def _dnu():
    # the direction dA = d/dnu A = the 5-point Laplacian (an ADR operator with nu = 1)
    return dict(nu=1.0, ax=0.0, ay=0.0, react=0.0)


def _dir(op, **kw):
    return dataclasses.replace(op, kind=W.OP_ADR, field0=None, field1=None, **kw)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _dense_tangent(op, dop, B, h, p):
    """[I 0] of the first half of expm(h [[At, Et], [0, At]]) [0; z] (dense)."""
    A = operators.dense(op)
    dA = operators.dense(dop)
    n, n1 = op.n, op.n + p
    At = phi.augmented_matrix(A, B, p)
    M = np.zeros((2 * n1, 2 * n1))
    M[:n1, :n1] = At
    M[n1:, n1:] = At
    M[:n, n1:n1 + n] = dA
    z = np.zeros(2 * n1)
    z[n1:n1 + n] = B[:, 0]
    if p > 0:
        z[n1 + n1 - 1] = 1.0
    r = phi.expm_taylor(h * M) @ z
    return r[n1:n1 + n], r[:n]


def test_dense_van_loan_equals_central_difference():
    op = _adr(5, 4)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((op.n, 3))
    h, p, eps = 0.3, 2, 1e-5
    y, dy = _dense_tangent(op, _dir(op, **_dnu()), B, h, p)
    yp = phi.phi_combo_dense(operators.dense(dataclasses.replace(op, nu=op.nu + eps)), B, h, p)
    ym = phi.phi_combo_dense(operators.dense(dataclasses.replace(op, nu=op.nu - eps)), B, h, p)
    assert _rel(y, phi.phi_combo_dense(operators.dense(op), B, h, p)) <= 1e-13
    assert _rel(dy, (yp - ym) / (2 * eps)) <= 1e-7


@pytest.mark.parametrize("orth,tform", [("mgs", "gsmgs"), ("hybrid", "gsmgs"), ("hybrid", "cwy")])
def test_tangent_krylov_exact_at_full_dimension(orth, tform):
    op = _adr(4, 3, react=0.2)
    rng = np.random.default_rng(6)
    B = rng.standard_normal((op.n, 3))
    h, p = 0.4, 2
    dop = _dir(op, nu=0.7, ax=0.3, ay=-0.2, react=1.1)   # a general direction
    y0, dy0 = _dense_tangent(op, dop, B, h, p)
    m = 2 * (op.n + p)
    y, dy, info = adjoint.phi_combo_tangent(op, dop, B, h, p, fixed_m=m, fixed_substeps=1,
                                            m_max=m, orth=orth, tform=tform)
    assert _rel(y, y0) <= 1e-11 and _rel(dy, dy0) <= 1e-10


def test_closed_form_dnu_equals_central_difference():
    op = _adr(32, 24, nu=0.02)
    rng = np.random.default_rng(7)
    B = rng.standard_normal((op.n, 4))
    h, p, eps = 0.05, 3, 1e-6
    d = closed_form.adr_phi_combo_dnu(op, B, h, p)
    yp = closed_form.adr_phi_combo(dataclasses.replace(op, nu=op.nu + eps), B, h, p)
    ym = closed_form.adr_phi_combo(dataclasses.replace(op, nu=op.nu - eps), B, h, p)
    assert _rel(d, (yp - ym) / (2 * eps)) <= 1e-6


def test_tangent_adaptive_matches_closed_form():
    op = _adr(40, 32, nu=0.01)
    rng = np.random.default_rng(8)
    B = rng.standard_normal((op.n, 3))
    h, p, tol = 0.05, 2, 1e-10
    y, dy, info = adjoint.phi_combo_tangent(op, _dir(op, **_dnu()), B, h, p, tol=tol, m_max=48,
                                            orth="hybrid")
    assert info.status == 0
    assert _rel(y, closed_form.adr_phi_combo(op, B, h, p)) <= 10 * tol
    assert _rel(dy, closed_form.adr_phi_combo_dnu(op, B, h, p)) <= 1e-7


@pytest.mark.parametrize("tr", [False, True])
def test_grad_B_dot_product_test_and_closed_form(tr):
    op = dataclasses.replace(_adr(24, 20, nu=0.02), transpose=tr)
    rng = np.random.default_rng(9)
    g = rng.standard_normal(op.n)
    h, p = 0.05, 2
    G = adjoint.grad_B(op, g, h, p, krylov.phi_combo, tol=1e-12, m_max=48, orth="hybrid")
    Gc = adjoint.grad_B(op, g, h, p, closed_form.adr_phi_combo)
    assert _rel(G, Gc) <= 1e-10
    for k in range(p + 1):                     # <g, h^k phi_k(hA) v> = <G_k, v>
        v = rng.standard_normal(op.n)
        Bk = np.zeros((op.n, k + 1))
        Bk[:, k] = v
        yk = closed_form.adr_phi_combo(op, Bk, h, k)
        assert abs(g @ yk - Gc[:, k] @ v) <= 1e-11 * abs(g) @ abs(yk)


@pytest.mark.parametrize("coef", ["nu", "ax", "ay", "react"])
def test_closed_form_coefficient_derivatives_equal_central_differences(coef):
    op = _adr(32, 24, nu=0.02, ax=1.0, ay=-0.5, react=0.3)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((op.n, 4))
    h, p, eps = 0.05, 3, 1e-6
    unit = {"nu": 0.0, "ax": 0.0, "ay": 0.0, "react": 0.0}
    unit[coef] = 1.0
    d = closed_form.adr_phi_combo_deriv(op, _dir(op, **unit), B, h, p)
    v = getattr(op, coef)
    yp = closed_form.adr_phi_combo(dataclasses.replace(op, **{coef: v + eps}), B, h, p)
    ym = closed_form.adr_phi_combo(dataclasses.replace(op, **{coef: v - eps}), B, h, p)
    assert _rel(d, (yp - ym) / (2 * eps)) <= 1e-6
    for tr in (False, True):             # and the tangent Krylov solve, both orientations
        opt = dataclasses.replace(op, transpose=tr)
        _, dy, _ = adjoint.phi_combo_tangent(opt, _dir(opt, **unit), B, h, p, tol=1e-11,
                                             m_max=48, orth="hybrid")
        assert _rel(dy, closed_form.adr_phi_combo_deriv(opt, _dir(opt, **unit), B, h, p)) <= 1e-8
