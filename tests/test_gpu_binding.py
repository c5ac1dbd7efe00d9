"""The binding on the GPU: wrong outputs are refused before any launch, the
differentiable call raises when a solve does not succeed, and the library
reports the runtime it is bound to."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2410_14917_amd as kp
from paper_2410_14917_amd import autograd as kpa

pytestmark = pytest.mark.gpu


def _problem():
    pr = W.random_problem(5, kind=W.OP_ADR, nx=40, ny=32, p=2, h=0.05)
    op = kp.Operator.from_host(pr.op, device="cuda")
    B = torch.as_tensor(np.ascontiguousarray(pr.B.T), device="cuda")
    return pr, op, B


def test_wrong_outputs_are_refused():
    pr, op, B = _problem()
    n = pr.op.n
    bad = [torch.empty(n, dtype=torch.float32, device="cuda"),
           torch.empty(n - 1, dtype=torch.float64, device="cuda"),
           torch.empty(2 * n, dtype=torch.float64, device="cuda")[::2],
           torch.empty(n, dtype=torch.float64)]
    with kp.Context() as ctx:
        for out in bad:
            with pytest.raises(ValueError):
                ctx.phi_combo(op, B, pr.h, tol=1e-8, m_max=16, out=out)
        good = torch.empty(n, dtype=torch.float64, device="cuda")
        dop = kp.Operator(op.kind, op.nx, op.ny, nu=1.0)
        for out in bad:
            with pytest.raises(ValueError):
                ctx.phi_combo_tangent(op, dop, B, pr.h, out=good, dout=out)
        with pytest.raises(ValueError):
            ctx.phi_combo_tangent(op, dop, B, pr.h, out=good, dout=good)
        # the context still works afterwards
        y, info = ctx.phi_combo(op, B, pr.h, tol=1e-8, m_max=16, out=good, info=True)
        assert info["status"] == 0


def test_autograd_raises_when_a_solve_does_not_converge():
    pr, op, B = _problem()
    Bg = B.clone().requires_grad_(True)
    nu = torch.tensor(pr.op.nu, dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(kp.SolveError) as e:
        kpa.phi_combo(Bg, nu, op, pr.h, tol=1e-12, m_max=2, max_substeps=2)
    assert e.value.info["status"] == 1
    y = kpa.phi_combo(Bg, nu, op, pr.h, tol=1e-8, m_max=24)     # a good call still works
    y.sum().backward()
    assert torch.isfinite(Bg.grad).all() and torch.isfinite(nu.grad)
    kpa.release_contexts()


def test_runtime_info():
    r = kp.runtime_info()
    assert r["hip_runtime_version"] > 0 and r["hip_driver_version"] > 0
    assert any("libamdhip64" in pth for pth in r["mapped_runtimes"])
    print(r)
