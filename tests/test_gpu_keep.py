"""The on-chip path of the one-reduction kernel: where each workgroup's rows of
a one-plane grid fit one sub-tile (4096 elements, rows of at most 2048), the
matvec pass leaves x_j and w in LDS for the basis update, which leaves the new
vector there for the next matvec pass (w is never stored).  Checked against
the DFT closed form, against the same call on a row partition where the path
is off (the configured rows_per_wg), against the oracle replaying the same
fixed schedule, and the library's count of the vector
passes it kept on chip (per Arnoldi process of m steps: 1 for the first step,
which stores no w, 4 for each later one, 2 for the close: 4 m - 1)."""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import closed_form, krylov
import paper_2410_14917_amd as kp

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


# (nx, ny, rows of a partition with the path off, path on by default)
CASES = [
    (300, 257, 14, True),     # 13 rows x 300 = 3900 per workgroup, 20 workgroups
    (333, 129, 14, True),     # odd rows: 12 rows (even, pair alignment), 11 workgroups
    (2047, 40, 4, True),      # 2 rows of 2047, the widest rows the halo copy takes
    (96, 70, 43, True),       # 42 rows, two workgroups, a ragged second one
    (2050, 30, 2, False),     # rows wider than 2048: off
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}")
@pytest.mark.parametrize("orth", ["h-gsmgs", "h-cwy"])
def test_onchip_path_against_closed_form_and_off_partition(case, orth):
    nx, ny, rows_off, on = case
    print(f"keep: {nx}x{ny} {orth}", flush=True)
    sys.stdout.flush()
    op_h = W.Operator(kind=W.OP_ADR, nx=nx, ny=ny, nu=0.05, ax=1.0, ay=0.5, react=-0.5)
    p, h, m, s = 2, 1e-4, 24, 2
    Bh = np.random.default_rng(nx + ny).standard_normal((op_h.n, p + 1))
    op = kp.Operator.from_host(op_h)
    B = torch.as_tensor(np.ascontiguousarray(Bh.T), device="cuda")
    ys, counts = [], []
    for rows in (0, rows_off):
        with kp.Context(orth=orth, fixed_m=m, fixed_substeps=s, rows_per_wg=rows) as ctx:
            y, info = ctx.phi_combo(op, B, h, m_max=m, info=True)
        assert info["status"] == 0 and info["arnoldi_steps"] == s * m
        ys.append(y.cpu().numpy())
        counts.append(info["onchip_passes"])
    assert counts == [s * (4 * m - 1) if on else 0, 0]
    ref, _ = krylov.phi_combo(op_h, Bh, h, p, fixed_m=m, fixed_substeps=s, m_max=m)
    assert rel(ys[0], ref) <= 1e-10
    assert rel(ys[0], ys[1]) <= 1e-13
    # the adaptive call on the default partition, against the DFT closed form
    with kp.Context(orth=orth) as ctx:
        y, info = ctx.phi_combo(op, B, h, tol=1e-10, m_max=64, info=True)
    assert info["status"] == 0
    assert (info["onchip_passes"] > 0) == on
    assert rel(y.cpu().numpy(), closed_form.adr_phi_combo(op_h, Bh, h, p)) <= 1e-9
