"""Pins of oracle/operators.py and oracle/closed_form.py (no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form, operators


def _loop_adr(op, x):
    """Brute-force 5-point finite differences, one grid point at a time."""
    nx, ny = op.nx, op.ny
    y = np.zeros(nx * ny)
    for iy in range(ny):
        for ix in range(nx):
            c = x[iy * nx + ix]
            e = x[iy * nx + (ix + 1) % nx]
            w = x[iy * nx + (ix - 1) % nx]
            n = x[((iy + 1) % ny) * nx + ix]
            s = x[((iy - 1) % ny) * nx + ix]
            lap = (e + w - 2 * c) / op.dx ** 2 + (n + s - 2 * c) / op.dy ** 2
            adv = op.ax * (e - w) / (2 * op.dx) + op.ay * (n - s) / (2 * op.dy)
            v = op.nu * lap - adv + op.react * c
            if op.field0 is not None:
                v += op.field0[iy * nx + ix] * c
            y[iy * nx + ix] = v
    return y


def test_adr_matches_pointwise_loops():
    pr = W.random_problem(21, nx=7, ny=5, with_diag=True, react=0.3)
    x = np.random.default_rng(0).standard_normal(pr.op.n)
    assert np.allclose(operators.apply(pr.op, x), _loop_adr(pr.op, x), rtol=1e-14, atol=1e-9)


def _rhs_allen_cahn(op, u):
    return op.nu * operators.diffusion_part(op, u) + u - u ** 3


def _rhs_brusselator(op, x):
    npt = op.nx * op.ny
    u, v = x[:npt], x[npt:]
    su = W.Operator(kind=0, nx=op.nx, ny=op.ny)
    lu = operators.diffusion_part(su, u)
    lv = operators.diffusion_part(su, v)
    fu = op.nu * lu + op.brus_a - (op.brus_b + 1.0) * u + u * u * v
    fv = op.nu2 * lv + op.brus_b * u - u * u * v
    return np.concatenate([fu, fv])


def _fd_jacobian(f, x0, eps=1e-6):
    n = len(x0)
    J = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = eps
        J[:, i] = (f(x0 + e) - f(x0 - e)) / (2 * eps)
    return J


def test_allen_cahn_is_jacobian_of_rhs():
    pr = W.random_problem(22, kind=W.OP_ALLEN_CAHN, nx=6, ny=5, nu=0.01)
    op = pr.op
    J = _fd_jacobian(lambda u: _rhs_allen_cahn(op, u), op.field0)
    A = operators.dense(op)
    assert np.allclose(A, J, rtol=1e-7, atol=1e-6 * np.max(np.abs(A)))


def test_brusselator_is_jacobian_of_rhs():
    pr = W.random_problem(23, kind=W.OP_BRUSSELATOR, nx=5, ny=4, nu=0.02)
    op = pr.op
    x0 = np.concatenate([op.field0, op.field1])
    J = _fd_jacobian(lambda x: _rhs_brusselator(op, x), x0)
    A = operators.dense(op)
    assert np.allclose(A, J, rtol=1e-7, atol=1e-6 * np.max(np.abs(A)))


@pytest.mark.parametrize("kind", [W.OP_ADR, W.OP_ALLEN_CAHN, W.OP_BRUSSELATOR])
def test_transpose_is_matrix_transpose(kind):
    pr = W.random_problem(24, kind=kind, nx=5, ny=6, with_diag=True, react=-0.2)
    A = operators.dense(pr.op)
    At = operators.dense(pr.op.with_transpose())
    assert np.allclose(At, A.T, rtol=1e-14, atol=1e-10)


@pytest.mark.parametrize("transpose", [False, True])
def test_dft_eigenvalues_match_stencil(transpose):
    op = W.Operator(kind=W.OP_ADR, nx=8, ny=6, nu=0.03, ax=1.3, ay=-0.4,
                    react=0.25, transpose=transpose, dx=0.11, dy=0.07)
    x = np.random.default_rng(1).standard_normal(op.n)
    assert np.allclose(closed_form.adr_apply_spectral(op, x),
                       operators.apply(op, x), rtol=1e-12, atol=1e-10)


def test_dft_closed_form_matches_dense_exponential():
    from oracle import phi
    op = W.Operator(kind=W.OP_ADR, nx=6, ny=5, nu=0.02, ax=1.0, ay=0.5, react=-0.3)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((op.n, 4))
    A = operators.dense(op)
    for h in (0.01, 0.2):
        ref = phi.phi_combo_dense(A, B, h, 3)
        got = closed_form.adr_phi_combo(op, B, h, 3)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
