"""Krylov evaluation of sum_k h^k phi_k(hA) b_k on an MI355X (gfx950).

Thin PyTorch binding over libkrylov_phi (include/krylov_phi.h): torch supplies
device memory and the current stream; every step of the computation runs in
the library's HIP kernels.  See arXiv:2410.14917, Section 3.3 (Algorithm 4)
for the hybrid low-synchronisation Arnoldi process the library implements.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

from . import _lib
from ._lib import (KP_OP_ADR, KP_OP_ALLEN_CAHN, KP_OP_BRUSSELATOR, KpConfig, KpInfo,
                   KpOp)

__all__ = ["Context", "Operator", "phi_combo", "runtime_info", "batch_plan", "SolveError",
           "raise_on_status", "KP_OP_ADR", "KP_OP_ALLEN_CAHN", "KP_OP_BRUSSELATOR"]


def _torch():
    import torch
    return torch


class Operator:
    """Matrix-free 2D periodic operator on the GPU (fields are device tensors)."""

    def __init__(self, kind, nx, ny, nu=0.0, nu2=0.0, ax=0.0, ay=0.0, react=0.0,
                 brus_a=1.0, brus_b=3.0, field0=None, field1=None, transpose=False,
                 dx=None, dy=None):
        self.kind, self.nx, self.ny = int(kind), int(nx), int(ny)
        self.nu, self.nu2, self.ax, self.ay = float(nu), float(nu2), float(ax), float(ay)
        self.react, self.brus_a, self.brus_b = float(react), float(brus_a), float(brus_b)
        self.dx = float(dx) if dx else 1.0 / nx
        self.dy = float(dy) if dy else 1.0 / ny
        self.field0, self.field1 = field0, field1
        self.transpose = bool(transpose)

    @classmethod
    def from_host(cls, op, device="cuda"):
        """From a workloads.Operator (numpy fields) to device tensors."""
        torch = _torch()
        f0 = None if op.field0 is None else torch.as_tensor(op.field0, dtype=torch.float64,
                                                            device=device).contiguous()
        f1 = None if op.field1 is None else torch.as_tensor(op.field1, dtype=torch.float64,
                                                            device=device).contiguous()
        return cls(op.kind, op.nx, op.ny, nu=op.nu, nu2=op.nu2, ax=op.ax, ay=op.ay,
                   react=op.react, brus_a=op.brus_a, brus_b=op.brus_b, field0=f0,
                   field1=f1, transpose=op.transpose, dx=op.dx, dy=op.dy)

    @property
    def n(self):
        return self.nx * self.ny * (2 if self.kind == KP_OP_BRUSSELATOR else 1)

    def c_struct(self) -> KpOp:
        def ptr(t):
            if t is None:
                return None
            _check_vec("an operator field", t, self.nx * self.ny)
            return ctypes.c_void_p(t.data_ptr())
        return KpOp(self.kind, self.nx, self.ny, int(self.transpose), self.dx, self.dy,
                    self.nu, self.nu2, self.ax, self.ay, self.react, self.brus_a,
                    self.brus_b, ptr(self.field0), ptr(self.field1))


STATUS_NAMES = {0: "ok", 1: "not converged", 2: "non-finite data", 3: "aborted (wait limit)"}


class SolveError(RuntimeError):
    """A solve ended with kp_info.status != KP_STATUS_OK."""

    def __init__(self, info):
        self.info = info
        super().__init__(f"libkrylov_phi: solve ended with status {info['status']} "
                         f"({STATUS_NAMES.get(info['status'], '?')}): {info}")


def raise_on_status(info):
    """Raise SolveError unless the kp_info record (as a dict) reports OK."""
    if info["status"] != 0:
        raise SolveError(info)
    return info


def _check_vec(name, t, n, device=None):
    """A caller-supplied output must be a contiguous float64 device vector of
    n elements (on `device` when given); checked before any launch, since the
    kernels write n float64 through its pointer."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the inputs on {device}")
    return t


def _b_layout(B, n):
    """(p, ldb) of a (p+1, N) right-hand-side tensor with unit stride along N."""
    if B.dim() != 2 or B.shape[1] != n or (n > 1 and B.stride(1) != 1):
        raise ValueError(f"B must have shape (p+1, {n}) with unit stride along N")
    # the stride of a single row is arbitrary (torch and numpy may report 1)
    ldb = B.stride(0) if B.shape[0] > 1 else n
    if ldb < n:
        raise ValueError(f"rows of B overlap (row stride {ldb} < {n})")
    return B.shape[0] - 1, ldb


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Owns a kp_ctx (device workspace, configuration, stream)."""

    def __init__(self, orth="h-gsmgs", basis="f64", max_substeps=0, fixed_m=0,
                 fixed_substeps=0, fallback_delta=0.0, breakdown_eps=0.0, m_init=0,
                 tau_init=0.0, controller="power", rows_per_wg=0, stream=None):
        """orth: "h-gsmgs" (default), "h-cwy", "h-ncwy" (Algorithm 4 with the
        correction of Algorithm 7, 5, 6), "mgs" (Algorithm 1) or "iocgs"
        (incomplete classical Gram-Schmidt over the previous two vectors);
        controller: "power" or "pi"; rows_per_wg: grid rows per workgroup of
        a single call (0: automatic)."""
        self.lib = _lib.load()
        self._stream = stream
        self.cfg = KpConfig(_stream_handle(stream), _lib.ORTH[orth], _lib.BASIS[basis],
                            int(m_init), int(max_substeps), int(fixed_m),
                            int(fixed_substeps), float(fallback_delta), float(breakdown_eps),
                            float(tau_init), _lib.CTRL[controller], int(rows_per_wg))
        h = ctypes.c_void_p()
        _lib.check(self.lib.kp_create(ctypes.byref(h), ctypes.byref(self.cfg)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.kp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def _check_B(B, n):
        torch = _torch()
        if B.dtype != torch.float64 or not B.is_cuda:
            raise ValueError("B must be a float64 device tensor of shape (p+1, N)")
        return _b_layout(B, n)

    def phi_combo(self, op: Operator, B, h: float, tol: float = 1e-8, m_max: int = 64,
                  out=None, info: bool = False):
        """out = sum_k h^k phi_k(h A) b_k; B is (p+1, N), row k = b_k."""
        torch = _torch()
        n = op.n
        p, ldb = self._check_B(B, n)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=B.device)
        _check_vec("out", out, n, B.device)
        opc = op.c_struct()
        inf = KpInfo() if info else None
        rc = self.lib.kp_phi_combo(self.h, ctypes.byref(opc), ctypes.c_void_p(B.data_ptr()),
                                   p, ldb, float(h), float(tol), int(m_max),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.byref(inf) if inf is not None else None)
        _lib.check(rc, self.h)
        return (out, inf.as_dict()) if info else out

    def phi_combo_tangent(self, op: Operator, dop: Operator, B, h: float, tol: float = 1e-8,
                          m_max: int = 64, out=None, dout=None, info: bool = False):
        """(out, dout): the phi combination and its derivative along the
        operator direction dop (same kind and grid as op; its nu, ax, ay,
        react are the direction).  One Krylov solve of the block operator."""
        torch = _torch()
        n = op.n
        p, ldb = self._check_B(B, n)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=B.device)
        if dout is None:
            dout = torch.empty(n, dtype=torch.float64, device=B.device)
        _check_vec("out", out, n, B.device)
        _check_vec("dout", dout, n, B.device)
        if out.data_ptr() == dout.data_ptr():
            raise ValueError("out and dout must be different tensors")
        opc, dopc = op.c_struct(), dop.c_struct()
        inf = KpInfo() if info else None
        rc = self.lib.kp_phi_combo_tangent(
            self.h, ctypes.byref(opc), ctypes.byref(dopc), ctypes.c_void_p(B.data_ptr()), p, ldb,
            float(h), float(tol), int(m_max), ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(dout.data_ptr()), ctypes.byref(inf) if inf is not None else None)
        _lib.check(rc, self.h)
        return (out, dout, inf.as_dict()) if info else (out, dout)

    COEFS = ("nu", "ax", "ay", "react")

    def phi_combo_backward(self, op: Operator, B, h: float, g, tol: float = 1e-8,
                           m_max: int = 64, want_B: bool = True, coefs=("nu",),
                           info: bool = False):
        """Gradients of a loss of y = phi_combo(op, B, h) given g = dL/dy:
        (grad_B (p+1, N) or None, grad_coef (4,) device tensor with the entries
        of `coefs` among ("nu", "ax", "ay", "react") filled)."""
        torch = _torch()
        n = op.n
        p, ldb = self._check_B(B, n)
        _check_vec("g", g, n, B.device)
        mask = 0
        for c in coefs:
            mask |= 1 << self.COEFS.index(c)
        gB = torch.empty((p + 1, n), dtype=torch.float64, device=B.device) if want_B else None
        gc = torch.zeros(4, dtype=torch.float64, device=B.device)
        opc = op.c_struct()
        inf = KpInfo() if info else None
        rc = self.lib.kp_phi_combo_backward(
            self.h, ctypes.byref(opc), ctypes.c_void_p(B.data_ptr()), p, ldb, float(h),
            float(tol), int(m_max), ctypes.c_void_p(g.data_ptr()),
            ctypes.c_void_p(gB.data_ptr()) if gB is not None else None, n, mask,
            ctypes.c_void_p(gc.data_ptr()), ctypes.byref(inf) if inf is not None else None)
        _lib.check(rc, self.h)
        return (gB, gc, inf.as_dict()) if info else (gB, gc)

    def phi_combo_batched(self, ops, Bs, hs, tol: float = 1e-8, m_max: int = 64, outs=None,
                          info: bool = False):
        """Independent phi combinations in one call: outs[i] = sum_k hs[i]^k
        phi_k(hs[i] A_i) Bs[i][k] for the operators ops[i] (Bs[i] is (p_i+1, N_i)).
        One persistent launch (replayed from a HIP graph while the problem
        shapes repeat).  Returns the list of outputs (and of info dicts)."""
        torch = _torch()
        n = len(ops)
        if n < 1 or len(Bs) != n or len(hs) != n:
            raise ValueError("ops, Bs and hs must have the same positive length")
        opc = (KpOp * n)(*[o.c_struct() for o in ops])
        bp = (ctypes.c_void_p * n)()
        pp = (ctypes.c_int32 * n)()
        lb = (ctypes.c_int64 * n)()
        hh = (ctypes.c_double * n)(*[float(x) for x in hs])
        if outs is None:
            outs = [torch.empty(o.n, dtype=torch.float64, device=B.device) for o, B in zip(ops, Bs)]
        op_ = (ctypes.c_void_p * n)()
        for i, (o, B, y) in enumerate(zip(ops, Bs, outs)):
            p, ldb = self._check_B(B, o.n)
            _check_vec(f"outs[{i}]", y, o.n, B.device)
            bp[i], pp[i], lb[i], op_[i] = B.data_ptr(), p, ldb, y.data_ptr()
        inf = (KpInfo * n)() if info else None
        rc = self.lib.kp_phi_combo_batched(self.h, n, opc, bp, pp, lb, hh, float(tol), int(m_max),
                                           op_, inf)
        _lib.check(rc, self.h)
        return (outs, [r.as_dict() for r in inf]) if info else outs

    def calibrate(self, force: bool = False):
        """Measure (or read from KP_AUTOTUNE_CACHE) the batched planner's cost
        model on this device; later batched calls of this context plan with
        it.  Returns (source: "measured" | "cache", model dict)."""
        import numpy as np
        v = np.zeros(5)
        rc = _lib.check(self.lib.kp_calibrate(self.h, int(bool(force)),
                                              v.ctypes.data_as(ctypes.c_void_p)), self.h)
        keys = ("bw_wg_Bps", "t_step_s", "t_team_s", "t_log_s", "t_expm64_s")
        return ("cache" if rc == 1 else "measured"), dict(zip(keys, v.tolist()))

    def read_bandwidth(self, nbytes: int = 1 << 30, reps: int = 20) -> float:
        """Practical HBM read rate in GB/s (kp_read_bandwidth: a plain
        streaming read in the persistent kernels' launch shape)."""
        v = ctypes.c_double()
        _lib.check(self.lib.kp_read_bandwidth(self.h, int(nbytes), int(reps), ctypes.byref(v)),
                   self.h)
        return v.value

    def schedule(self, cap: int = 8192):
        import numpy as np
        tau = np.zeros(cap)
        m = np.zeros(cap, dtype=np.int32)
        n = _lib.check(self.lib.kp_get_schedule(self.h, tau.ctypes.data_as(ctypes.c_void_p),
                                                m.ctypes.data_as(ctypes.c_void_p), cap), self.h)
        return list(zip(tau[:n].tolist(), m[:n].tolist()))

    def batch_schedule(self, i: int, cap: int = 8192):
        """(tau, m) of the accepted substeps of problem i of the last batched call."""
        import numpy as np
        tau = np.zeros(cap)
        m = np.zeros(cap, dtype=np.int32)
        n = _lib.check(self.lib.kp_get_batch_schedule(self.h, int(i),
                                                      tau.ctypes.data_as(ctypes.c_void_p),
                                                      m.ctypes.data_as(ctypes.c_void_p), cap),
                       self.h)
        return list(zip(tau[:n].tolist(), m[:n].tolist()))

    def arnoldi_begin(self, op: Operator, B, m_max: int):
        p, ldb = self._check_B(B, op.n)
        self._arn = (op, B, m_max, p)
        opc = op.c_struct()
        _lib.check(self.lib.kp_arnoldi_begin(self.h, ctypes.byref(opc),
                                             ctypes.c_void_p(B.data_ptr()), p, ldb, m_max),
                   self.h)

    def arnoldi_step(self, nsteps: int = 1):
        _lib.check(self.lib.kp_arnoldi_step(self.h, int(nsteps)), self.h)

    def arnoldi_read(self, want_basis: bool = True):
        import numpy as np
        op, B, m_max, p = self._arn
        H = np.zeros((m_max + 1) * m_max)
        j = ctypes.c_int32()
        beta = ctypes.c_double()
        flags = (ctypes.c_int32 * 2)()
        _lib.check(self.lib.kp_arnoldi_read(self.h, H.ctypes.data_as(ctypes.c_void_p), None,
                                            ctypes.byref(j), ctypes.byref(beta), flags), self.h)
        V = None
        if want_basis:
            V = np.zeros((j.value + 1) * (op.n + p))
            _lib.check(self.lib.kp_arnoldi_read(self.h, None, V.ctypes.data_as(ctypes.c_void_p),
                                                None, None, None), self.h)
            V = V.reshape(j.value + 1, op.n + p).T
        return {"H": H.reshape(m_max, m_max + 1).T, "j": j.value, "beta": beta.value,
                "breakdown": flags[0], "n_fallback": flags[1], "V": V}

    def integrate(self, rhs, u, dt: float, nsteps: int, method: str = "epi4",
                  tol: float = 1e-12, m_max: int = 64, start_substeps: int = 4,
                  info: bool = False):
        """Advance u (a contiguous float64 device vector of nx*ny, updated in
        place) by nsteps steps of size dt of an exponential integrator of
        Section 4.1 ("epi4", "epi5", "srerk3") for u' = f(u); rhs has the
        fields kind (0 Allen-Cahn, 1 ADR), nx, ny, dx, dy, nu, ax, ay, gamma
        (e.g. a workloads.Rhs).  Every phi combination is a library call with
        this context's configuration."""
        n = int(rhs.nx) * int(rhs.ny)
        _check_vec("u", u, n)
        r = _lib.KpRhs(int(rhs.kind), int(rhs.nx), int(rhs.ny), 0, float(rhs.dx), float(rhs.dy),
                       float(rhs.nu), float(getattr(rhs, "ax", 0.0)),
                       float(getattr(rhs, "ay", 0.0)), float(getattr(rhs, "gamma", 0.0)))
        inf = KpInfo() if info else None
        rc = self.lib.kp_integrate(self.h, ctypes.byref(r), _lib.METHODS[method], float(dt),
                                   int(nsteps), int(start_substeps), ctypes.c_void_p(u.data_ptr()),
                                   float(tol), int(m_max),
                                   ctypes.byref(inf) if inf is not None else None)
        _lib.check(rc, self.h)
        return (u, inf.as_dict()) if info else u

    def expm_hbar(self, H, m: int, tau: float):
        """exp(tau Hbar) e_1 by the device's small-exponential routine; H is
        (m+1) x m."""
        import numpy as np
        Hf = np.asfortranarray(np.asarray(H, dtype=np.float64)[:m + 1, :m])
        F = np.zeros(m + 1)
        _lib.check(self.lib.kp_expm_hbar(self.h, Hf.ctypes.data_as(ctypes.c_void_p), m + 1, m,
                                         float(tau), F.ctypes.data_as(ctypes.c_void_p)), self.h)
        return F


def phi_combo(op: Operator, B, h: float, tol: float = 1e-8, m_max: int = 64,
              info: bool = False, **ctx_kw):
    """One-shot convenience wrapper (creates and frees a Context)."""
    with Context(**ctx_kw) as ctx:
        return ctx.phi_combo(op, B, h, tol=tol, m_max=m_max, info=info)


def runtime_info():
    """The HIP runtime the library is bound to in this process: its version
    and driver version (from the library), and the paths of every HIP runtime
    and HSA runtime mapped into the process."""
    lib = _lib.load()
    rv, dv = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(lib.kp_runtime_version(ctypes.byref(rv), ctypes.byref(dv)))
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1] if len(line.split()) >= 6 else ""
                base = path.rsplit("/", 1)[-1]
                if base.startswith(("libamdhip64", "libhsa-runtime64")):
                    paths.add(path)
    except OSError:
        pass
    return {"hip_runtime_version": rv.value, "hip_driver_version": dv.value,
            "mapped_runtimes": sorted(paths)}


def batch_plan(ops, ps, hs, m_max: int = 64, n_wg: int = 256):
    """The batched call's planner on the host (no device needed): returns
    (team_of_problem, teams [(first workgroup, size)], predicted makespan s,
    predicted one-workgroup time s).  ops may be host operators with numpy
    fields: only the presence of a field matters."""
    lib = _lib.load()
    n = len(ops)

    def cs(o):
        f0 = ctypes.c_void_p(1) if getattr(o, "field0", None) is not None else None
        f1 = ctypes.c_void_p(1) if getattr(o, "field1", None) is not None else None
        return KpOp(int(o.kind), int(o.nx), int(o.ny), int(bool(o.transpose)), float(o.dx),
                    float(o.dy), float(o.nu), float(o.nu2), float(o.ax), float(o.ay),
                    float(o.react), float(o.brus_a), float(o.brus_b), f0, f1)
    opc = (KpOp * n)(*[cs(o) for o in ops])
    pp = (ctypes.c_int32 * n)(*[int(x) for x in ps])
    hh = (ctypes.c_double * n)(*[float(x) for x in hs])
    top = (ctypes.c_int32 * n)()
    w0 = (ctypes.c_int32 * n_wg)()
    sz = (ctypes.c_int32 * n_wg)()
    nt = ctypes.c_int32()
    ms, wk = ctypes.c_double(), ctypes.c_double()
    _lib.check(lib.kp_batch_plan(n, opc, pp, hh, int(m_max), int(n_wg), top, w0, sz,
                                 ctypes.byref(nt), ctypes.byref(ms), ctypes.byref(wk)))
    teams = [(w0[t], sz[t]) for t in range(nt.value)]
    return list(top), teams, ms.value, wk.value
