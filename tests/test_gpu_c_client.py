"""The library driven by a C++ program through its C ABI alone (no Python, no
torch in that process): tests/c_abi_client.cpp runs the forward, batched and
backward entry points and the host planner on an advection-diffusion-reaction
problem; its outputs are checked against the oracle's closed forms (the
operator is diagonalised by the discrete Fourier basis) and its fixed-schedule
Krylov process."""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, closed_form, krylov

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "c_abi_client")
FP64_TOL = 1e-10
UNITS = [(1.0, 0, 0, 0), (0, 1.0, 0, 0), (0, 0, 1.0, 0), (0, 0, 0, 1.0)]   # nu, ax, ay, react


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("m,nsub", [(32, 2), (0, 0)], ids=["fixed-m32x2", "adaptive"])
def test_c_client_against_oracle(tmp_path, m, nsub):
    if not os.path.exists(CLIENT):
        pytest.fail("tests/c_abi_client is not built (run the package build)")
    op = W.Operator(kind=W.OP_ADR, nx=64, ny=48, nu=0.02, ax=1.0, ay=-0.5, react=-0.2)
    rng = np.random.default_rng(77)
    p, h, tol = 2, 0.05, 1e-12
    B = rng.standard_normal((op.n, p + 1))
    g = rng.standard_normal(op.n)
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.array([op.nx, op.ny, p, m, nsub], dtype=np.int32).tobytes())
        f.write(np.array([op.nu, op.ax, op.ay, op.react, h, tol], dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(B.T).tobytes())
        f.write(g.tobytes())
    print(f"c_abi_client {op.nx}x{op.ny} p={p} m={m} nsub={nsub}", flush=True)
    res = subprocess.run([CLIENT, str(src), str(dst)], capture_output=True, text=True,
                         timeout=120)
    sys.stdout.write(res.stdout + res.stderr)
    assert res.returncode == 0
    raw = np.fromfile(dst, dtype=np.uint8)
    st = np.frombuffer(raw[:16].tobytes(), dtype=np.int32)
    vals = np.frombuffer(raw[16:].tobytes(), dtype=np.float64)
    n = op.n
    y, yb0, yb1 = vals[:n], vals[n:2 * n], vals[2 * n:3 * n]
    gB = vals[3 * n:3 * n + (p + 1) * n].reshape(p + 1, n).T
    gc = vals[3 * n + (p + 1) * n:]
    assert list(st) == [0, 0, 0, 0] and gc.size == 4

    exact = closed_form.adr_phi_combo(op, B, h, p)
    print(f"  y rel closed form {rel(y, exact):.2e}")
    assert rel(y, exact) <= FP64_TOL
    if m:
        ref, _ = krylov.phi_combo(op, B, h, p, fixed_m=m, fixed_substeps=nsub, m_max=m)
        assert rel(y, ref) <= FP64_TOL
    assert rel(yb0, y) <= 1e-12 and rel(yb1, y) <= 1e-12
    gB_ref = adjoint.grad_B(op, g, h, p, closed_form.adr_phi_combo)
    print(f"  grad_B rel {rel(gB, gB_ref):.2e}")
    assert rel(gB, gB_ref) <= 1e-9
    for c, unit in enumerate(UNITS):
        d = W.Operator(kind=W.OP_ADR, nx=op.nx, ny=op.ny, nu=unit[0], ax=unit[1], ay=unit[2],
                       react=unit[3])
        ref = float(g @ closed_form.adr_phi_combo_deriv(op, d, B, h, p))
        print(f"  grad_coef[{c}] {gc[c]:.12e} ref {ref:.12e}")
        assert abs(gc[c] - ref) <= 1e-8 * abs(ref)
