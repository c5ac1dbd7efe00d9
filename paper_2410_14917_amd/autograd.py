"""Gradients of the phi combination (torch.autograd), computed by the library.

    y = sum_{k=0}^{p} h^k phi_k(h A(nu)) b_k,    A(nu) = nu Lap + (the rest of A)

For an upstream gradient g = dL/dy:

  * dL/db_k = h^k phi_k(h A^T) g: one Krylov solve with the transposed
    operator per k (kp_phi_combo with transpose set, B = [0, ..., 0, g]); this
    is the adjoint of the map b_k -> y (the phi functions of A^T are the
    transposes of those of A).
  * dL/dnu = <g, dy/dnu>, with dy/dnu from one solve of the block operator
    [[Atilde, Etilde], [0, Atilde]], Etilde = [[Lap, 0], [0, 0]]
    (kp_phi_combo_tangent: the Frechet derivative of the exponential of the
    augmented matrix of Section 2.1 in the direction of the operator change).

Every solve runs in the HIP library; torch only holds the tensors and forms
the chain-rule inner product.
"""
from __future__ import annotations


from . import Context, Operator


def _with(op: Operator, **kw) -> Operator:
    o = Operator(op.kind, op.nx, op.ny, nu=op.nu, nu2=op.nu2, ax=op.ax, ay=op.ay,
                 react=op.react, brus_a=op.brus_a, brus_b=op.brus_b, field0=op.field0,
                 field1=op.field1, transpose=op.transpose, dx=op.dx, dy=op.dy)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


_CTX = {}


def _context(ctx_kw) -> Context:
    """One Context per (device, stream, configuration), kept for the process:
    the workspace is allocated once and reused by the forward and backward
    solves (calls on one stream are ordered, so sharing it is safe)."""
    import torch
    s = torch.cuda.current_stream()
    key = (torch.cuda.current_device(), s.cuda_stream, tuple(sorted(ctx_kw.items())))
    c = _CTX.get(key)
    if c is None:
        c = _CTX[key] = Context(stream=s, **ctx_kw)
    return c


def _fn():
    import torch

    class PhiComboFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, B, nu, op, h, tol, m_max, ctx_kw):
            opn = _with(op, nu=float(nu))
            y = _context(ctx_kw).phi_combo(opn, B.contiguous(), h, tol=tol, m_max=m_max)
            ctx.save_for_backward(B)
            ctx.op, ctx.h, ctx.tol, ctx.m_max, ctx.ctx_kw = opn, h, tol, m_max, ctx_kw
            return y

        @staticmethod
        def backward(ctx, g):
            (B,) = ctx.saved_tensors
            op, h, tol, m_max = ctx.op, ctx.h, ctx.tol, ctx.m_max
            g = g.contiguous()
            grad_B = grad_nu = None
            c = _context(ctx.ctx_kw)
            if ctx.needs_input_grad[0]:
                opt = _with(op, transpose=not op.transpose)
                p = B.shape[0] - 1
                grad_B = torch.empty_like(B)
                for k in range(p + 1):
                    Bk = torch.zeros((k + 1, B.shape[1]), dtype=B.dtype, device=B.device)
                    Bk[k] = g
                    c.phi_combo(opt, Bk, h, tol=tol, m_max=m_max, out=grad_B[k])
            if ctx.needs_input_grad[1]:
                dop = _with(op, nu=1.0, ax=0.0, ay=0.0, react=0.0, field0=None,
                            field1=None)
                _, dy = c.phi_combo_tangent(op, dop, B.contiguous(), h, tol=tol,
                                            m_max=m_max)
                grad_nu = torch.dot(g, dy).reshape(())
            return grad_B, grad_nu, None, None, None, None, None

    return PhiComboFn


_FN = None


def release_contexts() -> None:
    """Free the workspaces of the cached Contexts."""
    for c in _CTX.values():
        c.close()
    _CTX.clear()


def phi_combo(B, nu, op: Operator, h: float, tol: float = 1e-8, m_max: int = 64, **ctx_kw):
    """Differentiable phi combination: B (p+1, N) and nu (0-dim tensor) may
    require gradients; op supplies the grid and the other coefficients.
    ctx_kw are Context options (orth, basis, fixed_m, fixed_substeps, ...);
    the solves run on torch's current stream."""
    if "stream" in ctx_kw:
        raise ValueError("phi_combo runs on torch's current stream; do not pass stream")
    global _FN
    if _FN is None:
        _FN = _fn()
    return _FN.apply(B, nu, op, h, tol, m_max, ctx_kw)
