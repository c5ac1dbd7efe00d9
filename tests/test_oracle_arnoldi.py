"""Pins of oracle/arnoldi.py (no GPU): the Arnoldi relation, orthogonality,
QR of the Krylov matrix, the correction-matrix identities of Section 3.2 and
the worked T_3 example."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import arnoldi, krylov, operators, phi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _problem(seed=31, nx=9, ny=7, p=2, kind=W.OP_ADR):
    pr = W.random_problem(seed, kind=kind, nx=nx, ny=ny, p=p, with_diag=True)
    mu = krylov.balance_scale(pr.B, p)
    apply = lambda x: krylov.aug_apply(pr.op, pr.B, p, mu, x)
    z = krylov.start_vector(pr.B, p, mu)
    return pr, apply, z


def _aug_dense(apply, n):
    A = np.zeros((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        A[:, i] = apply(e)
        e[i] = 0.0
    return A


def test_mgs_arnoldi_relation_and_orthogonality():
    pr, apply, z = _problem()
    m = 20
    arn = arnoldi.MGSArnoldi(apply, z, m)
    assert arn.extend(m) == m
    V, H = arn.V[:, :m + 1], arn.H[:m + 1, :m]
    A = _aug_dense(apply, len(z))
    assert np.linalg.norm(A @ V[:, :m] - V @ H) <= 1e-13 * np.linalg.norm(A, 2)
    assert np.linalg.norm(np.eye(m + 1) - V.T @ V, 2) <= 1e-13
    assert np.allclose(np.tril(H, -2), 0.0)
    assert np.all(np.diag(H, -1) > 0)
    assert np.allclose(V[:, 0] * arn.beta, z, rtol=0, atol=1e-14 * arn.beta)


def test_mgs_basis_equals_qr_of_krylov_matrix():
    pr, apply, z = _problem(seed=32, nx=5, ny=4)
    m = 6
    K = np.zeros((len(z), m))
    v = z.copy()
    for i in range(m):
        K[:, i] = v
        v = apply(v)
    Q, R = np.linalg.qr(K)
    Q = Q * np.sign(np.diag(R))           # positive diagonal convention
    arn = arnoldi.MGSArnoldi(apply, z, m)
    arn.extend(m)
    assert np.allclose(arn.V[:, :m], Q, atol=1e-9)


@pytest.mark.parametrize("tform", ["cwy", "ncwy", "gsmgs"])
def test_hybrid_matches_mgs_hessenberg(tform):
    pr, apply, z = _problem(seed=33)
    m = 25
    a = arnoldi.MGSArnoldi(apply, z, m)
    a.extend(m)
    b = arnoldi.HybridArnoldi(apply, z, m, tform=tform)
    b.extend(m)
    assert b.beta == pytest.approx(a.beta, rel=1e-14)
    Ha, Hb = a.H[:m + 1, :m], b.H[:m + 1, :m]
    assert np.linalg.norm(Ha - Hb) <= 1e-12 * np.linalg.norm(Ha)
    Vb = b.basis()
    assert np.linalg.norm(np.eye(m + 1) - Vb.T @ Vb, 2) <= 1e-12
    assert np.linalg.norm(Vb - a.V[:, :m + 1]) <= 1e-11


@pytest.mark.parametrize("tform", ["cwy", "ncwy", "gsmgs"])
def test_hybrid_extension_reuses_basis(tform):
    """Extending 10 -> 20 equals running 20 steps at once."""
    pr, apply, z = _problem(seed=34)
    a = arnoldi.HybridArnoldi(apply, z, 20, tform=tform)
    a.extend(10)
    a.extend(20)
    b = arnoldi.HybridArnoldi(apply, z, 20, tform=tform)
    b.extend(20)
    assert np.allclose(a.H[:21, :20], b.H[:21, :20], rtol=1e-13, atol=1e-13)


def test_cwy_recursion_is_product_of_rank_one_projectors():
    """(I - v_j v_j^T)...(I - v_1 v_1^T) = I - V_j T_j V_j^T for unit vectors,
    T_j built row by row by eq. recursionForT (Section 3.2.1)."""
    rng = np.random.default_rng(7)
    n, j = 30, 8
    V = rng.standard_normal((n, j))
    V /= np.linalg.norm(V, axis=0)
    T = np.eye(j)
    for r in range(1, j):
        T[r, :r] = arnoldi.cwy_row(V[:, :r].T @ V[:, r], T[:r, :r])
    P = np.eye(n)
    for r in range(j):
        P = (np.eye(n) - np.outer(V[:, r], V[:, r])) @ P
    assert np.linalg.norm(P - (np.eye(n) - V @ T @ V.T)) <= 1e-13
    L = np.tril(V.T @ V, -1)
    assert np.allclose(T, np.linalg.inv(np.eye(j) + L), atol=1e-13)


def test_gsmgs_is_two_gauss_seidel_sweeps():
    """gsmgs_apply == M^{-1}(I + N M^{-1}) b == two Gauss-Seidel sweeps on the
    normal equations V^T V x = V^T w from x0 = 0 (Section 3.2.3)."""
    rng = np.random.default_rng(8)
    n, j = 40, 7
    V = rng.standard_normal((n, j))
    V /= np.linalg.norm(V, axis=0)
    w = rng.standard_normal(n)
    G = V.T @ V
    L = np.tril(G, -1)
    M = np.eye(j) + L
    N = -L.T
    Minv = np.linalg.inv(M)
    b = V.T @ w
    got = arnoldi.gsmgs_apply(M, Minv, N, b)
    x1 = np.linalg.solve(M, b)
    x2 = np.linalg.solve(M, b + N @ x1)
    assert np.allclose(got, x2, rtol=1e-13, atol=1e-13)
    assert np.allclose(M - N, G, atol=1e-15)
    # a single sweep is the CWY projection, (I + L)^{-1} b
    assert not np.allclose(got, x1, atol=1e-6)


def test_golden_t3_example():
    with open(os.path.join(GOLDEN, "t3_example.json")) as f:
        g = json.load(f)
    rng = np.random.default_rng(9)
    vals = dict(zip(g["symbols"], rng.uniform(-0.3, 0.3, 3)))

    def ev(mat):
        return np.array([[eval(e, {"__builtins__": {}}, vals) for e in row] for row in mat])

    a21, a31, a32 = vals["a21"], vals["a31"], vals["a32"]
    L = np.array([[0, 0, 0], [a21, 0, 0], [a31, a32, 0]])
    T = np.eye(3)
    for r in range(1, 3):
        T[r, :r] = arnoldi.cwy_row(L[r, :r], T[:r, :r])
    assert np.allclose(T, ev(g["cwy"]), atol=1e-15)
    Tn = np.eye(3)
    for r in range(1, 3):
        Tn[r, :r] = arnoldi.ncwy_row(L[r, :r])
    assert np.allclose(Tn, ev(g["ncwy"]), atol=1e-15)
    assert np.allclose(T - Tn, ev(g["dropped_term"]), atol=1e-15)


@pytest.mark.parametrize("orth", ["mgs", "cwy", "gsmgs"])
def test_lucky_breakdown_on_diagonal_operator(orth):
    """A diagonal operator with d distinct values: the augmented Krylov space
    has dimension d + p, so the process stops there and is exact."""
    d_vals = np.array([-3.0, -1.0, -0.5, 0.2, 1.1])
    nx, ny = 10, 4
    idx = np.random.default_rng(12).integers(0, len(d_vals), nx * ny)
    diag = d_vals[idx]
    op = W.Operator(kind=W.OP_ADR, nx=nx, ny=ny, nu=0.0, ax=0.0, ay=0.0, field0=diag)
    p = 2
    B = np.random.default_rng(13).standard_normal((op.n, p + 1))
    mu = krylov.balance_scale(B, p)
    apply = lambda x: krylov.aug_apply(op, B, p, mu, x)
    z = krylov.start_vector(B, p, mu)
    m_cap = 15
    if orth == "mgs":
        arn = arnoldi.MGSArnoldi(apply, z, m_cap)
    else:
        arn = arnoldi.HybridArnoldi(apply, z, m_cap, tform=orth)
    j = arn.extend(m_cap)
    assert arn.breakdown and j == len(d_vals) + p
    if orth != "mgs":
        assert arn.n_fallback >= 1       # the estimate cancels at the breakdown step


def test_orthogonality_loss_ordering_on_stiff_problem():
    """The two-sweep correction keeps V^T V closest to I (Section 3.2.3)."""
    pr = W.config2(side=64)
    mu = krylov.balance_scale(pr.B, pr.p)
    apply = lambda x: krylov.aug_apply(pr.op, pr.B, pr.p, mu, 200.0 * x)
    z = krylov.start_vector(pr.B, pr.p, mu)
    loss = {}
    for tf in ("cwy", "gsmgs"):
        a = arnoldi.HybridArnoldi(apply, z, 40, tform=tf)
        a.extend(40)
        Vb = a.basis()[:, :40]
        loss[tf] = np.linalg.norm(np.eye(40) - Vb.T @ Vb, 2)
    m = arnoldi.MGSArnoldi(apply, z, 40)
    m.extend(40)
    loss["mgs"] = np.linalg.norm(np.eye(40) - m.V[:, :40].T @ m.V[:, :40], 2)
    assert loss["gsmgs"] <= loss["cwy"]
    assert max(loss.values()) < 1e-8


# ---- incomplete orthogonalisation (ioCGS, Section 2.3.1) --------------------

def _symmetric_problem(seed=51, nx=11, ny=9):
    """Diffusion + reaction + a diagonal field, p = 0: A is symmetric."""
    rng = np.random.default_rng(seed)
    op = W.Operator(kind=W.OP_ADR, nx=nx, ny=ny, nu=0.02, react=-0.4,
                    field0=rng.uniform(-1.0, 1.0, nx * ny))
    b = rng.standard_normal(op.n)
    return op, (lambda x: operators.apply(op, x)), b


def test_iop_on_symmetric_operator_is_lanczos():
    """For symmetric A the full Arnoldi process has a tridiagonal H (the
    Lanczos recurrence), so orthogonalising against the previous two vectors
    gives the same H and V as MGS (until orthogonality is lost)."""
    op, apply, b = _symmetric_problem()
    A = operators.dense(op)
    assert np.allclose(A, A.T)
    m = 12
    a = arnoldi.MGSArnoldi(apply, b, m)
    a.extend(m)
    c = arnoldi.IOPArnoldi(apply, b, m, window=2)
    c.extend(m)
    assert np.allclose(np.triu(a.H[:m + 1, :m], 2), 0.0, atol=1e-12 * np.abs(a.H).max())
    assert np.linalg.norm(c.H[:m + 1, :m] - a.H[:m + 1, :m]) <= 1e-10 * np.linalg.norm(a.H)
    assert np.linalg.norm(c.V[:, :m + 1] - a.V[:, :m + 1]) <= 1e-9


def test_iop_with_full_window_is_classical_gram_schmidt():
    """A window of at least m is classical Gram-Schmidt against the whole
    basis: the same Hessenberg matrix as MGS in exact arithmetic; a window of
    one leaves the entries above the diagonal zero."""
    pr, apply, z = _problem(seed=52, nx=8, ny=6)
    m = 8
    a = arnoldi.MGSArnoldi(apply, z, m)
    a.extend(m)
    c = arnoldi.IOPArnoldi(apply, z, m, window=m)
    c.extend(m)
    assert np.linalg.norm(c.H[:m + 1, :m] - a.H[:m + 1, :m]) <= 1e-10 * np.linalg.norm(a.H)
    d = arnoldi.IOPArnoldi(apply, z, m, window=1)
    d.extend(m)
    assert np.allclose(np.triu(d.H[:m + 1, :m], 1), 0.0)


def test_iop_arnoldi_relation_without_orthogonality():
    """On a non-normal operator the two-vector window still satisfies
    A V_m = V_{m+1} Hbar (each column is built that way), each new vector is
    orthogonal to its window, but V^T V is far from I."""
    pr, apply, z = _problem(seed=53, nx=10, ny=8)
    m = 20
    c = arnoldi.IOPArnoldi(apply, z, m, window=2)
    assert c.extend(m) == m
    V, H = c.V[:, :m + 1], c.H[:m + 1, :m]
    A = _aug_dense(apply, len(z))
    assert np.linalg.norm(A @ V[:, :m] - V @ H) <= 1e-12 * np.linalg.norm(A, 2)
    assert np.allclose(np.triu(H, 2), 0.0) and np.allclose(np.tril(H, -2), 0.0)
    for j in range(1, m + 1):
        lo = max(0, j - 2)
        assert np.all(np.abs(V[:, lo:j].T @ V[:, j]) <= 1e-12)
    assert np.linalg.norm(np.eye(m + 1) - V.T @ V, 2) > 1e-3


def test_iop_exact_at_invariant_subspace():
    """A diagonal operator with d distinct values and p = 0 (a symmetric
    matrix, so the two-vector window is the Lanczos recurrence): the Krylov
    space is invariant after d steps (lucky breakdown), where A V = V H makes
    V exp(tau H) e_1 exact."""
    d_vals = np.array([-2.0, -0.7, 0.3, 0.9])
    nx, ny = 8, 5
    diag = d_vals[np.random.default_rng(54).integers(0, len(d_vals), nx * ny)]
    op = W.Operator(kind=W.OP_ADR, nx=nx, ny=ny, field0=diag)
    p = 0
    B = np.random.default_rng(55).standard_normal((op.n, p + 1))
    y, info = krylov.phi_combo(op, B, 0.4, p, fixed_m=12, fixed_substeps=1, m_max=12,
                               orth="iop")
    assert info.breakdowns == 1 and info.m_last == len(d_vals)
    ref = np.zeros(op.n)
    for k in range(p + 1):
        ref += 0.4 ** k * np.array([phi.phi_scalar(k, 0.4 * d) for d in diag]) * B[:, k]
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
