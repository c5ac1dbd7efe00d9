"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and fixes problem parameters; it holds
none of the phi-function / Krylov arithmetic.  Both the CPU oracle and the HIP
path receive the arrays produced here, so neither side generates inputs for the
other.

Workloads follow the shapes of the paper's test problems (second-order finite
differences on 2D grids, Section 4.3) at the sizes of the five benchmark
configurations:

  cfg1  advection-diffusion, 64x64 periodic, p=3, fixed m=40
  cfg2  Allen-Cahn Jacobian 0.01*Lap + diag(1-3u^2), 1024x1024, p=2, m<=64
  cfg3  2-species Brusselator Jacobian, 2048x2048 (N=8,388,608), p=2, m<=64
  cfg4  512 advection-diffusion-reaction problems, sides U{32..512}, p=3, m<=48
  cfg5  advection-diffusion 1024x1024 with a least-squares loss, p=2

All grids are unit periodic squares, dx = 1/nx, dy = 1/ny.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 20241017

# Operator kinds (same numbering as the C header's KP_OP_* constants).
OP_ADR = 0          # nu*Lap + centred advection + r (+ optional diagonal field)
OP_ALLEN_CAHN = 1   # nu*Lap + diag(1 - 3 u^2), u = field0
OP_BRUSSELATOR = 2  # 2-species Brusselator Jacobian at (u, v) = (field0, field1)


@dataclasses.dataclass
class Operator:
    """Matrix-free 2D periodic operator description (host side)."""
    kind: int
    nx: int
    ny: int
    nu: float = 0.0          # diffusion (species u for the Brusselator)
    nu2: float = 0.0         # diffusion of species v (Brusselator only)
    ax: float = 0.0          # advection velocity, x
    ay: float = 0.0          # advection velocity, y
    react: float = 0.0       # constant reaction coefficient (ADR)
    brus_a: float = 1.0      # Brusselator constant A
    brus_b: float = 3.0      # Brusselator constant B
    field0: Optional[np.ndarray] = None   # ADR diag / AC state u / Brusselator u
    field1: Optional[np.ndarray] = None   # Brusselator v
    transpose: bool = False
    dx: float = 0.0
    dy: float = 0.0

    def __post_init__(self):
        if self.dx == 0.0:
            self.dx = 1.0 / self.nx
        if self.dy == 0.0:
            self.dy = 1.0 / self.ny

    @property
    def npoints(self) -> int:
        return self.nx * self.ny

    @property
    def n(self) -> int:
        """Length of the state vector the operator acts on."""
        return self.npoints * (2 if self.kind == OP_BRUSSELATOR else 1)

    def with_transpose(self, flag: bool = True) -> "Operator":
        return dataclasses.replace(self, transpose=flag)


@dataclasses.dataclass
class Problem:
    op: Operator
    B: np.ndarray            # N x (p+1), columns b_0..b_p (float64, Fortran order)
    h: float
    p: int
    m_max: int
    tol: float
    fixed_m: int = 0         # >0: fixed Krylov dimension
    fixed_substeps: int = 0  # >0 with fixed_m: equal substeps tau = h / fixed_substeps
    seed: int = 0
    name: str = ""
    y: Optional[np.ndarray] = None   # target for the adjoint loss (cfg5)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_columns(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k i.i.d. N(0,1), column-major."""
    return np.asfortranarray(rng.standard_normal((k, n)).T)


def smooth_field(rng: np.random.Generator, nx: int, ny: int, modes: int = 16,
                 kmax: int = 8, amplitude: float = 0.9) -> np.ndarray:
    """Sum of `modes` random Fourier cosines on the unit periodic square,
    rescaled to max |u| = amplitude.  Integer wavenumbers in [-kmax, kmax]
    (not both zero), phases U[0, 2pi).  Returned flattened, x fastest."""
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)          # shape (ny, nx), X varies along axis 1
    s = np.zeros((ny, nx))
    q = 0
    while q < modes:
        kx, ky = rng.integers(-kmax, kmax + 1, size=2)
        if kx == 0 and ky == 0:
            continue
        ph = rng.uniform(0.0, 2.0 * math.pi)
        s += np.cos(2.0 * math.pi * (kx * X + ky * Y) + ph)
        q += 1
    s *= amplitude / np.max(np.abs(s))
    return np.ascontiguousarray(s.reshape(-1))


def adr(nx, ny, nu=0.01, ax=1.0, ay=0.5, react=0.0, diag=None) -> Operator:
    return Operator(kind=OP_ADR, nx=nx, ny=ny, nu=nu, ax=ax, ay=ay, react=react,
                    field0=diag)


def config1(seed: Optional[int] = None) -> Problem:
    """64x64 periodic advection-diffusion, nu=0.01, a=(1,0.5), h=0.05, p=3,
    b_k ~ N(0,1), one substep of fixed m=40."""
    seed = SEED_BASE + 1 if seed is None else seed
    rng = rng_for(seed)
    op = adr(64, 64)
    B = gaussian_columns(rng, op.n, 4)
    return Problem(op=op, B=B, h=0.05, p=3, m_max=40, tol=1e-10, fixed_m=40,
                   fixed_substeps=1, seed=seed, name="cfg1-adr64")


def config2(seed: Optional[int] = None, side: int = 1024) -> Problem:
    """Allen-Cahn Jacobian 0.01*Lap + diag(1-3u^2), u a smooth random field
    (16 Fourier modes, amplitude 0.9), h=0.1, p=2, m<=64, tol 1e-8."""
    seed = SEED_BASE + 2 if seed is None else seed
    rng = rng_for(seed)
    u = smooth_field(rng, side, side)
    op = Operator(kind=OP_ALLEN_CAHN, nx=side, ny=side, nu=0.01, field0=u)
    B = gaussian_columns(rng, op.n, 3)
    return Problem(op=op, B=B, h=0.1, p=2, m_max=64, tol=1e-8, seed=seed,
                   name=f"cfg2-allen-cahn{side}")


def config3(seed: Optional[int] = None, side: int = 2048) -> Problem:
    """Brusselator Jacobian (A=1, B=3, D_u=0.02, D_v=0.01) at u = 1*(1+U[-.1,.1]),
    v = 3*(1+U[-.1,.1]); N = 2*side^2; h=0.01, p=2, m<=64, tol 1e-6."""
    seed = SEED_BASE + 3 if seed is None else seed
    rng = rng_for(seed)
    npt = side * side
    u = 1.0 * (1.0 + rng.uniform(-0.1, 0.1, npt))
    v = 3.0 * (1.0 + rng.uniform(-0.1, 0.1, npt))
    op = Operator(kind=OP_BRUSSELATOR, nx=side, ny=side, nu=0.02, nu2=0.01,
                  brus_a=1.0, brus_b=3.0, field0=u, field1=v)
    B = gaussian_columns(rng, op.n, 3)
    return Problem(op=op, B=B, h=0.01, p=2, m_max=64, tol=1e-6, seed=seed,
                   name=f"cfg3-brusselator{side}")


def config4(seed: Optional[int] = None, nprob: int = 512, side_lo: int = 32,
            side_hi: int = 512) -> list:
    """Batched uneven advection-diffusion-reaction problems: side ~ U{lo..hi},
    nu ~ logU[1e-3, 1e-1], r ~ U[-1, 1], a=(1, 0.5), h=0.05, p=3, m<=48,
    tol 1e-8."""
    seed = SEED_BASE + 4 if seed is None else seed
    rng = rng_for(seed)
    probs = []
    for k in range(nprob):
        side = int(rng.integers(side_lo, side_hi + 1))
        nu = float(math.exp(rng.uniform(math.log(1e-3), math.log(1e-1))))
        r = float(rng.uniform(-1.0, 1.0))
        op = adr(side, side, nu=nu, react=r)
        B = gaussian_columns(rng, op.n, 4)
        probs.append(Problem(op=op, B=B, h=0.05, p=3, m_max=48, tol=1e-8,
                             seed=seed, name=f"cfg4-{k}"))
    return probs


def config5(seed: Optional[int] = None, side: int = 1024) -> Problem:
    """Adjoint workload: advection-diffusion (nu=0.01, a=(1,0.5)), h=0.05, p=2,
    b_k and target y ~ N(0,1)."""
    seed = SEED_BASE + 5 if seed is None else seed
    rng = rng_for(seed)
    op = adr(side, side)
    B = gaussian_columns(rng, op.n, 3)
    y = rng.standard_normal(op.n)
    return Problem(op=op, B=B, h=0.05, p=2, m_max=64, tol=1e-10, seed=seed,
                   name=f"cfg5-adr{side}", y=y)


def random_problem(seed: int, kind: int = OP_ADR, nx: int = 16, ny: int = 12,
                   p: int = 2, h: float = 0.05, m_max: int = 24, tol: float = 1e-10,
                   nu: float = 0.01, ax: float = 1.0, ay: float = 0.5,
                   react: float = 0.0, with_diag: bool = False) -> Problem:
    """Small seeded problem of any operator kind, for parity and edge tests."""
    rng = rng_for(seed)
    npt = nx * ny
    f0 = f1 = None
    if kind == OP_ADR and with_diag:
        f0 = rng.uniform(-1.0, 1.0, npt)
    elif kind == OP_ALLEN_CAHN:
        f0 = smooth_field(rng, nx, ny, modes=4, kmax=2)
    elif kind == OP_BRUSSELATOR:
        f0 = 1.0 * (1.0 + rng.uniform(-0.1, 0.1, npt))
        f1 = 3.0 * (1.0 + rng.uniform(-0.1, 0.1, npt))
    op = Operator(kind=kind, nx=nx, ny=ny, nu=nu, nu2=0.5 * nu, ax=ax, ay=ay,
                  react=react, field0=f0, field1=f1)
    B = gaussian_columns(rng, op.n, p + 1)
    return Problem(op=op, B=B, h=h, p=p, m_max=m_max, tol=tol, seed=seed,
                   name=f"rand-{kind}-{nx}x{ny}")


# ---- nonlinear problems of the exponential integrators (Section 4.3) ---------
#
# u' = f(u) on a periodic grid (point (ix, iy) at index iy*nx + ix):
#   RHS_ALLEN_CAHN  f(u) = nu Lap u + u - u^3
#   RHS_ADR         f(u) = nu Lap u - ax Dx u - ay Dy u + gamma u (u - 1/2) (1 - u)
# (same numbering as the C header's KP_RHS_* constants).  The paper's
# problems have no-flow / Neumann boundaries; these are their periodic
# stand-ins, with the paper's coefficients and initial states.
RHS_ALLEN_CAHN = 0
RHS_ADR = 1


@dataclasses.dataclass
class Rhs:
    kind: int
    nx: int
    ny: int
    dx: float
    dy: float
    nu: float = 0.0
    ax: float = 0.0
    ay: float = 0.0
    gamma: float = 0.0

    @property
    def n(self) -> int:
        return self.nx * self.ny


@dataclasses.dataclass
class Ivp:
    rhs: Rhs
    u0: np.ndarray
    dt: float
    nsteps: int
    tol: float
    m_max: int = 64
    name: str = ""


def ivp_allen_cahn(side: int = 2000, dt: float = 1e-2, nsteps: int = 2,
                   tol: float = 1e-12) -> Ivp:
    """Allen-Cahn on [-1, 1]^2 (Section 4.3): epsilon = 0.1, initial state
    0.1 + 0.1 cos(2 pi x) cos(2 pi y), dt = 1e-2 (t_f = 0.02: two steps)."""
    dx = 2.0 / side
    x = -1.0 + dx * np.arange(side)
    X, Y = np.meshgrid(x, x)
    u0 = 0.1 + 0.1 * np.cos(2.0 * math.pi * X) * np.cos(2.0 * math.pi * Y)
    return Ivp(Rhs(RHS_ALLEN_CAHN, side, side, dx, dx, nu=0.1), np.ascontiguousarray(u0.reshape(-1)),
               dt, nsteps, tol, name=f"allen-cahn{side}")


def ivp_adr(side: int = 2000, dt: float = 1e-2, nsteps: int = 10, tol: float = 1e-12,
            gamma: float = 100.0) -> Ivp:
    """Advection-diffusion-reaction on [0, 1]^2 (Section 4.3): epsilon = 1e-2,
    alpha = -6 (f = eps Lap u - alpha (u_x + u_y) + gamma u (u - 1/2)(1 - u)),
    initial state 0.3 + 256 (x y (1 - x)(1 - y))^2, dt = 1e-2 (t_f = 0.1);
    gamma is not printed, 100 is taken."""
    dx = 1.0 / side
    x = dx * np.arange(side)
    X, Y = np.meshgrid(x, x)
    u0 = 0.3 + 256.0 * (X * Y * (1.0 - X) * (1.0 - Y)) ** 2
    return Ivp(Rhs(RHS_ADR, side, side, dx, dx, nu=1e-2, ax=-6.0, ay=-6.0, gamma=gamma),
               np.ascontiguousarray(u0.reshape(-1)), dt, nsteps, tol, name=f"adr{side}")

