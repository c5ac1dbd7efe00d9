"""Gradients of the phi combination (torch.autograd), computed by the library.

    y = sum_{k=0}^{p} h^k phi_k(h A(theta)) b_k,
    A(theta) = nu Lap - ax Dx - ay Dy + react I (+ the operator's fields)

For an upstream gradient g = dL/dy, kp_phi_combo_backward returns

  * dL/db_k = h^k phi_k(h A^T) g: one Krylov solve with the transposed
    operator per k (B = [0, ..., 0, g]); the adjoint of the map b_k -> y, as
    the phi functions of A^T are the transposes of those of A;
  * dL/dtheta_c = <g, dy/dtheta_c> for every coefficient that requires a
    gradient: one solve of the block operator [[Atilde, Etilde], [0, Atilde]],
    Etilde = [[dA/dtheta_c, 0], [0, 0]] (the Frechet derivative of the
    exponential of Section 2.1's augmented matrix in the direction of the
    coefficient), and a fixed-order device inner product.

Every solve and the inner products run in the HIP library; torch only holds
the tensors.
"""
from __future__ import annotations

from . import Context, Operator, raise_on_status

COEFS = ("nu", "ax", "ay", "react")


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
        def forward(ctx, B, nu, ax, ay, react, op, h, tol, m_max, ctx_kw):
            vals = {name: float(t) for name, t in zip(COEFS, (nu, ax, ay, react))
                    if t is not None}
            opn = _with(op, **vals)
            # the solve's status is checked (a call that did not converge,
            # met non-finite data or was aborted raises SolveError rather
            # than returning a wrong or unwritten y)
            y, info = _context(ctx_kw).phi_combo(opn, B.contiguous(), h, tol=tol, m_max=m_max,
                                                 info=True)
            raise_on_status(info)
            ctx.save_for_backward(B)
            ctx.op, ctx.h, ctx.tol, ctx.m_max, ctx.ctx_kw = opn, h, tol, m_max, ctx_kw
            return y

        @staticmethod
        def backward(ctx, g):
            (B,) = ctx.saved_tensors
            want_B = ctx.needs_input_grad[0]
            coefs = [name for name, need in zip(COEFS, ctx.needs_input_grad[1:5]) if need]
            gB, gc, info = _context(ctx.ctx_kw).phi_combo_backward(
                ctx.op, B.contiguous(), ctx.h, g.contiguous(), tol=ctx.tol, m_max=ctx.m_max,
                want_B=want_B, coefs=coefs, info=True)
            raise_on_status(info)   # the worst status of the backward's solves
            grads = [gc[COEFS.index(name)].reshape(()) if name in coefs else None
                     for name in COEFS]
            return (gB, *grads, None, None, None, None, None)

    return PhiComboFn


_FN = None


def release_contexts() -> None:
    """Free the workspaces of the cached Contexts."""
    for c in _CTX.values():
        c.close()
    _CTX.clear()


def phi_combo(B, nu, op: Operator, h: float, tol: float = 1e-8, m_max: int = 64, ax=None,
              ay=None, react=None, **ctx_kw):
    """Differentiable phi combination: B (p+1, N) and the coefficient tensors
    nu, ax, ay, react (0-dim; None keeps op's value) may require gradients;
    op supplies the grid, the fields and the other coefficients.  ctx_kw are
    Context options (orth, basis, fixed_m, fixed_substeps, ...); the solves
    run on torch's current stream."""
    if "stream" in ctx_kw:
        raise ValueError("phi_combo runs on torch's current stream; do not pass stream")
    global _FN
    if _FN is None:
        _FN = _fn()
    return _FN.apply(B, nu, ax, ay, react, op, h, tol, m_max, ctx_kw)
