"""Pins of oracle/phi.py against quadrature, eigen-decompositions and library
routines (no GPU)."""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy.integrate import quad

from oracle import phi


def _phi_quad(k, z):
    """phi_k(z) from its integral definition (eq. phi_int_def) by quadrature."""
    if k == 0:
        return complex(np.exp(z))
    def f_re(th):
        return (np.exp((1 - th) * z) * th ** (k - 1) / math.factorial(k - 1)).real
    def f_im(th):
        return (np.exp((1 - th) * z) * th ** (k - 1) / math.factorial(k - 1)).imag
    re = quad(f_re, 0.0, 1.0, epsabs=0.0, epsrel=2e-14, limit=200)[0]
    im = quad(f_im, 0.0, 1.0, epsabs=0.0, epsrel=2e-14, limit=200)[0]
    return complex(re, im)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("z", [-250.0, -30.0, -3.0, -1.0, -0.7, 0.0, 1e-9, 0.3,
                               1.0, 2.5, 6.0, -2 + 3j, 0.4 - 0.5j, -40 + 10j])
def test_phi_scalar_matches_integral_definition(k, z):
    got = complex(phi.phi_scalar(k, z))
    ref = _phi_quad(k, z)
    assert abs(got - ref) <= 2e-14 * abs(ref) + 1e-300


def test_phi_at_zero_is_inverse_factorial():
    for k in range(8):
        assert phi.phi_scalar(k, 0.0) == pytest.approx(1.0 / math.factorial(k), rel=1e-15)


def test_phi_vectorised_matches_scalar():
    z = np.linspace(-20, 5, 41)
    v = phi.phi_scalar(2, z)
    for zi, vi in zip(z, v):
        assert vi == pytest.approx(complex(_phi_quad(2, zi)).real, rel=1e-13, abs=1e-300)


def test_expm_symmetric_against_eigendecomposition():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((12, 12))
    S = 3.0 * (X + X.T)
    lam, Q = np.linalg.eigh(S)
    ref = (Q * np.exp(lam)) @ Q.T
    got = phi.expm_taylor(S)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_expm_nonnormal_against_similarity():
    rng = np.random.default_rng(4)
    n = 9
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    U = np.triu(rng.standard_normal((n, n)) * 0.3, 1) + np.eye(n)
    Vs = Q @ U                               # well conditioned, non-orthogonal
    lam = rng.uniform(-8, 1, n)
    X = Vs @ np.diag(lam) @ np.linalg.inv(Vs)
    ref = Vs @ np.diag(np.exp(lam)) @ np.linalg.inv(Vs)
    got = phi.expm_taylor(X)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_expm_nilpotent_finite_series():
    # N = c * (upper shift): exp(N) has entries c^k / k! on the k-th superdiagonal
    n, c = 7, 5.0
    N = c * np.eye(n, k=1)
    got = phi.expm_taylor(N)
    for k in range(n):
        assert np.allclose(np.diag(got, k), c ** k / math.factorial(k), rtol=1e-14, atol=0)
    assert np.allclose(np.tril(got, -1), 0.0)


@pytest.mark.parametrize("scale", [0.01, 1.0, 30.0, 300.0])
def test_expm_against_library_pade(scale):
    rng = np.random.default_rng(5)
    X = scale * rng.standard_normal((15, 15)) / 15.0 - scale * np.eye(15)
    ref = scipy.linalg.expm(X)
    got = phi.expm_taylor(X)
    assert np.linalg.norm(got - ref) <= 1e-11 * max(np.linalg.norm(ref), 1e-300)


def test_expm_semigroup():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((10, 10))
    E1 = phi.expm_taylor(X)
    E2 = phi.expm_taylor(2.0 * X)
    assert np.linalg.norm(E1 @ E1 - E2) <= 1e-12 * np.linalg.norm(E2)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 5])
def test_augmented_identity_diagonal(p):
    """Top block of exp(h Atilde)[b_0; e_p] == sum_k h^k phi_k(h d) b_k."""
    rng = np.random.default_rng(10 + p)
    n = 7
    d = rng.uniform(-20, 2, n)
    B = rng.standard_normal((n, p + 1))
    h = 0.37
    got = phi.phi_combo_dense(np.diag(d), B, h, p)
    ref = np.zeros(n)
    for k in range(p + 1):
        ref += h ** k * np.array([complex(_phi_quad(k, h * di)).real for di in d]) * B[:, k]
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    assert np.linalg.norm(phi.phi_combo_diag(d, B, h, p) - ref) <= 1e-13 * np.linalg.norm(ref)


def test_augmented_identity_discriminates_step_placement():
    """Dropping the h^k weights (the ansatz without a step) gives a different
    vector, so the identity fixes where h goes."""
    rng = np.random.default_rng(11)
    n, p, h = 6, 3, 0.3
    d = rng.uniform(-5, 1, n)
    B = rng.standard_normal((n, p + 1))
    got = phi.phi_combo_dense(np.diag(d), B, h, p)
    wrong = sum(phi.phi_scalar(k, h * d) * B[:, k] for k in range(p + 1))
    assert np.linalg.norm(got - wrong) > 0.1 * np.linalg.norm(got)
    # reversing the order of the b_k inside B is also caught
    Brev = np.concatenate([B[:, :1], B[:, :0:-1]], axis=1)
    assert np.linalg.norm(phi.phi_combo_dense(np.diag(d), Brev, h, p) - got) > 1e-3
