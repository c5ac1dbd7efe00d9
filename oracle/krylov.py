"""Krylov evaluation of the phi combination (oracle, test infrastructure).

y = sum_{k=0}^p h^k phi_k(hA) b_k is computed as the top block of
exp(h Atilde) z, z = [b_0; mu e_p], Atilde = [[A, Bhat/mu], [0, K]]
(Section 2.1, eq. philincomb).  Bhat = [b_p, ..., b_1] and K is the p x p
upper shift.  mu is a power of two (the largest one not above
max_{k>=1} ||b_k||_inf), a balancing of the two blocks that is exact in
floating point and leaves the result unchanged; the paper does not fix one.

The exponential is applied by substepping (Section 2.2, eq. substep):
w_{i+1} = exp(tau_i Atilde) w_i, each factor by the Krylov projection
beta V_m exp(tau_i H_m) e_1 (eq. kryexp) built by Algorithm 1 (default) or
Algorithm 4.  The error of a substep is estimated from the (m+1)-st entry of
exp(tau_i Hbar) e_1, Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]].

Schedules
---------
fixed     fixed_m > 0, fixed_substeps = n: n equal substeps tau = h/n with
          exactly fixed_m Arnoldi steps each (fewer on lucky breakdown).
adaptive  the substep controller below.  The paper delegates it to KIOPS and
          does not print its formulas, so this controller is this project's
          own (stated identically in the HIP library):
            start tau = h, m = min(16, m_max) (or the given m_init, tau_init);
            omega = err * h / (tol * beta * tau)        (beta = ||w_i||);
            accept iff omega <= 1;
            on reject: if m < m_max, double m (capped) and continue the same
              Arnoldi process (basis reuse); else shrink tau (same basis, only
              the small exponential is recomputed);
            tau update: tau *= clamp(0.9 * omega^(-1/(q+1)), 0.2, 4),
              q = ceil(m/4), omega = 0 -> factor 4;
            controller="pi" (the PI step-size control that Section 5 names as
              future work) replaces the factor after an accepted substep by
              clamp(0.9 * omega^(-0.7/(q+1)) * omega_prev^(0.4/(q+1)), 0.2, 4),
              omega_prev that of the previous accepted substep (the
              Gustafsson PI gains of Hairer and Wanner, Solving ODEs II,
              Section IV.2); the first accepted substep and every rejection
              use the power law above;
            lucky breakdown: the space is invariant, tau = h - t, accept;
            the last substep is clipped to end exactly at h.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

from . import operators
from .arnoldi import HybridArnoldi, IOPArnoldi, MGSArnoldi
from .phi import expm_taylor

STATUS_OK, STATUS_NOT_CONVERGED, STATUS_NONFINITE = 0, 1, 2

F_SAFE, F_MIN, F_MAX = 0.9, 0.2, 4.0
PI_KI, PI_KP = 0.7, 0.4


def step_factor(omega: float, m: int, omega_prev: float = 0.0, controller: str = "power"):
    """Step-size factor after a substep of dimension m with normalised error
    omega (accept iff omega <= 1).  omega_prev > 0 with controller "pi":
    the proportional-integral law; otherwise the power law."""
    if omega == 0.0:
        return F_MAX
    q = (m + 3) // 4
    if controller == "pi" and omega_prev > 0.0:
        f = F_SAFE * omega ** (-PI_KI / (q + 1)) * omega_prev ** (PI_KP / (q + 1))
    else:
        f = F_SAFE * omega ** (-1.0 / (q + 1))
    return min(F_MAX, max(F_MIN, f))


def balance_scale(B: np.ndarray, p: int) -> float:
    """Largest power of two not above max_{k>=1} ||b_k||_inf (1 if that is 0)."""
    if p == 0:
        return 1.0
    mx = float(np.max(np.abs(B[:, 1:p + 1])))
    if not (mx > 0.0) or not math.isfinite(mx):
        return 1.0
    return math.ldexp(1.0, math.frexp(mx)[1] - 1)


def aug_apply(op, B: np.ndarray, p: int, mu: float, x: np.ndarray) -> np.ndarray:
    """[A x_top + (Bhat/mu) x_tail;  K x_tail]."""
    n = op.n
    y = np.empty(n + p)
    top = operators.apply(op, x[:n])
    for c in range(p):                   # column c of Bhat is b_{p-c}
        top = top + (x[n + c] / mu) * B[:, p - c]
    y[:n] = top
    if p > 0:
        y[n:n + p - 1] = x[n + 1:n + p]
        y[n + p - 1] = 0.0
    return y


def start_vector(B: np.ndarray, p: int, mu: float) -> np.ndarray:
    n = B.shape[0]
    z = np.zeros(n + p)
    z[:n] = B[:, 0]
    if p > 0:
        z[n + p - 1] = mu
    return z


def hbar(H: np.ndarray, m: int) -> np.ndarray:
    """(m+1) x (m+1) matrix [[H_m, 0], [h_{m+1,m} e_m^T, 0]]."""
    Hb = np.zeros((m + 1, m + 1))
    Hb[:m + 1, :m] = H[:m + 1, :m]
    return Hb


@dataclasses.dataclass
class Info:
    status: int = STATUS_OK
    substeps: int = 0
    rejected: int = 0
    arnoldi_steps: int = 0
    expm_evals: int = 0
    m_last: int = 0
    err_max: float = 0.0
    n_fallback: int = 0
    breakdowns: int = 0
    schedule: List[Tuple[float, int]] = dataclasses.field(default_factory=list)
    orth_loss: float = 0.0


def _make_arnoldi(orth, apply, w, m_cap, tform, delta, eps_bd):
    if orth == "mgs":
        return MGSArnoldi(apply, w, m_cap, eps_bd=eps_bd)
    if orth == "iop":
        return IOPArnoldi(apply, w, m_cap, window=2, eps_bd=eps_bd)
    if orth != "hybrid":
        raise ValueError(orth)
    return HybridArnoldi(apply, w, m_cap, tform=tform, delta=delta, eps_bd=eps_bd)


def _basis(arn, m):
    if isinstance(arn, (MGSArnoldi, IOPArnoldi)):
        return arn.V[:, :m]
    return arn.basis()[:, :m]


def expmv(apply, w: np.ndarray, h: float, tol: float = 1e-8, m_max: int = 64,
          fixed_m: int = 0, fixed_substeps: int = 0, orth: str = "mgs",
          tform: str = "gsmgs", max_substeps: int = 2000, delta: float = 1e-10,
          eps_bd: float = 1e-12, want_orth_loss=False, m_init: int = 16,
          tau_init: float = 0.0, schedule=None, controller: str = "power"):
    """exp(h M) w for the operator M given by apply(x) = M x, by substepped
    Krylov projections with the schedules above.  Returns (vector, Info).

    schedule: the replay schedule, a list of accepted substeps (tau_i, m_i):
    each is one Krylov projection of dimension m_i (fewer at a lucky
    breakdown) advanced by tau_i, in order; tol, m_max and the controller are
    not used.  This replays a schedule another implementation logged, so the
    two results can be compared at rounding level (Section 3's substepping,
    eq. substep)."""
    n = len(w)
    info = Info()
    if schedule is not None:
        return _replay(apply, w, schedule, orth, tform, delta, eps_bd, info)
    fixed = fixed_m > 0
    if fixed:
        nsub = max(1, fixed_substeps)
        m = fixed_m
        tau = h / nsub
    else:
        m = min(m_init, m_max)
        tau = min(tau_init, h) if tau_init > 0.0 else h
    if controller not in ("power", "pi"):
        raise ValueError(controller)
    omega_prev = 0.0                               # of the last accepted substep
    t = 0.0
    while t < h:
        if info.substeps >= (nsub if fixed else max_substeps):
            if not fixed:
                info.status = STATUS_NOT_CONVERGED
            break
        if not fixed:
            tau = min(tau, h - t)
        arn = _make_arnoldi(orth, apply, w, m_max if not fixed else m, tform,
                            delta, eps_bd)
        if orth in ("mgs", "iop") and arn.beta == 0.0:
            break                                  # zero stays zero
        mb = arn.extend(m)
        beta = arn.beta
        if not beta:
            break
        info.arnoldi_steps += mb
        while True:
            if arn.breakdown:
                if not fixed:
                    tau = h - t
                Hb = hbar(arn.H, mb)
                Hb[mb, mb - 1] = 0.0
                F = expm_taylor(tau * Hb)[:, 0]
                info.expm_evals += 1
                err = 0.0
                omega = 0.0
                info.breakdowns += 1
                break
            Hb = hbar(arn.H, mb)
            F = expm_taylor(tau * Hb)[:, 0]
            info.expm_evals += 1
            err = beta * abs(F[mb])
            if fixed:
                omega = 0.0
                break
            omega = err * h / (tol * beta * tau)
            if not math.isfinite(omega):
                info.status = STATUS_NONFINITE
                return np.full(n, np.nan), info
            if omega <= 1.0:
                break
            info.rejected += 1
            if mb < m_max:
                m = min(2 * m, m_max)
                before = arn.j
                mb = arn.extend(m)
                info.arnoldi_steps += mb - before
                continue
            tau = tau * step_factor(omega, mb)
            if tau <= 1e-14 * h:
                info.status = STATUS_NOT_CONVERGED
                return w.copy(), info
        if want_orth_loss:
            Vb = _basis(arn, mb)
            info.orth_loss = max(info.orth_loss,
                                 float(np.linalg.norm(np.eye(mb) - Vb.T @ Vb, 2)))
        Vm = _basis(arn, mb)
        w = beta * (Vm @ F[:mb])
        info.err_max = max(info.err_max, err)
        info.schedule.append((tau, mb))
        info.substeps += 1
        info.m_last = mb
        if isinstance(arn, HybridArnoldi):
            info.n_fallback += arn.n_fallback
        if fixed:
            t = h if info.substeps == nsub else t + tau
        else:
            t = h if tau >= h - t else t + tau
            tau = tau * step_factor(omega, mb, omega_prev, controller)
            omega_prev = omega
    return w.copy(), info


def _replay(apply, w, schedule, orth, tform, delta, eps_bd, info):
    """The substeps of a given schedule; see expmv."""
    for tau, m_i in schedule:
        arn = _make_arnoldi(orth, apply, w, int(m_i), tform, delta, eps_bd)
        if orth in ("mgs", "iop") and arn.beta == 0.0:
            break
        mb = arn.extend(int(m_i))
        beta = arn.beta
        if not beta:
            break
        info.arnoldi_steps += mb
        Hb = hbar(arn.H, mb)
        if arn.breakdown:
            Hb[mb, mb - 1] = 0.0
            info.breakdowns += 1
        F = expm_taylor(tau * Hb)[:, 0]
        info.expm_evals += 1
        info.err_max = max(info.err_max, 0.0 if arn.breakdown else beta * abs(F[mb]))
        w = beta * (_basis(arn, mb) @ F[:mb])
        info.schedule.append((tau, mb))
        info.substeps += 1
        info.m_last = mb
        if isinstance(arn, HybridArnoldi):
            info.n_fallback += arn.n_fallback
    return w.copy(), info


def phi_combo(op, B: np.ndarray, h: float, p: int, tol: float = 1e-8,
              m_max: int = 64, fixed_m: int = 0, fixed_substeps: int = 0,
              orth: str = "mgs", tform: str = "gsmgs", max_substeps: int = 2000,
              delta: float = 1e-10, eps_bd: float = 1e-12, want_orth_loss=False,
              mu: float = None, m_init: int = 16, tau_init: float = 0.0, schedule=None,
              controller: str = "power"):
    """Returns (y, Info).  orth: 'mgs' (Algorithm 1), 'hybrid' (Algorithm 4)
    or 'iop' (ioCGS, Section 2.3.1); schedule: replay the given accepted
    substeps (see expmv); controller: 'power' or 'pi' (see the module
    docstring)."""
    n = op.n
    B = np.asarray(B, dtype=np.float64)
    if not np.all(np.isfinite(B[:, :p + 1])):
        info = Info()
        info.status = STATUS_NONFINITE
        return np.full(n, np.nan), info
    if mu is None:
        mu = balance_scale(B, p)
    w = start_vector(B, p, mu)
    if h == 0.0:
        return B[:, 0].copy(), Info()

    def apply(x):
        return aug_apply(op, B, p, mu, x)

    r, info = expmv(apply, w, h, tol=tol, m_max=m_max, fixed_m=fixed_m,
                    fixed_substeps=fixed_substeps, orth=orth, tform=tform,
                    max_substeps=max_substeps, delta=delta, eps_bd=eps_bd,
                    want_orth_loss=want_orth_loss, m_init=m_init, tau_init=tau_init,
                    schedule=schedule, controller=controller)
    return r[:n].copy(), info
