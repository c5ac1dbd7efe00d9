"""The scaling threshold of the device's small exponential (degree-19 Taylor
polynomial): theta_19 is the largest 1-norm x for which the backward-error
bound of the truncated series, sum_{k>19} |c_k| x^(k-1) <= 2^-53 with c_k the
coefficients of h(x) = log(e^{-x} T_19(x)) (Al-Mohy and Higham, SIAM J.
Matrix Anal. Appl. 31 (2009), Section 3), holds.  Recomputed here with exact
rational series arithmetic and compared with the constant in the kernel
source.  Host only."""
import math
import os
import re
from fractions import Fraction

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2410_14917_amd", "csrc", "kp_expm.h")
K = 100     # series length: the terms past it are below 1e-70 at theta


def _mul(a, b):
    c = [Fraction(0)] * (K + 1)
    for i, x in enumerate(a):
        if x:
            for j in range(K + 1 - i):
                if b[j]:
                    c[i + j] += x * b[j]
    return c


def theta(m: int) -> float:
    fact = [math.factorial(k) for k in range(K + 1)]
    emx = [Fraction((-1) ** k, fact[k]) for k in range(K + 1)]
    tail = [Fraction(0)] * (m + 1) + [Fraction(1, fact[j]) for j in range(m + 1, K + 1)]
    r = _mul(emx, tail)                       # 1 - e^{-x} T_m(x)
    h = [Fraction(0)] * (K + 1)               # log(1 - r) = -sum r^n / n
    p, n = r[:], 1
    while any(p):
        for k in range(K + 1):
            h[k] -= p[k] / n
        p, n = _mul(p, r), n + 1
    c = [abs(float(x)) for x in h]
    assert all(c[k] == 0.0 for k in range(m + 1))   # h starts at x^(m+1)
    bound = lambda x: sum(c[k] * x ** (k - 1) for k in range(m + 1, K + 1))
    lo, hi = 0.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if bound(mid) <= 2.0 ** -53 else (lo, mid)
    return lo


def test_theta19_matches_the_kernel_constant():
    text = open(SRC).read()
    got = float(re.search(r"kTheta19\s*=\s*([0-9.eE+-]+)", text).group(1))
    assert abs(theta(19) - got) <= 1e-13 * got


def test_theta_grows_with_the_degree():
    # a longer series allows a larger scaled norm; degree 18 lies below 19
    assert theta(18) < theta(19) < theta(20)
