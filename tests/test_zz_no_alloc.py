"""kp_phi_combo_noalloc (the workspace in the library's static device array)
against kp_phi_combo through the C ABI: two calls in a row, the second with a
smaller problem; a problem beyond the array's capacity is refused before any
device work.  Runs last (it shares the one static array per GPU)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from paper_2410_14917_amd import _lib

pytestmark = pytest.mark.gpu


def _ctx(lib, stream, **kw):
    cfg = _lib.KpConfig()
    cfg.stream = ctypes.c_void_p(stream.cuda_stream)
    for k, v in kw.items():
        setattr(cfg, k, v)
    h = ctypes.c_void_p()
    assert lib.kp_create(ctypes.byref(h), ctypes.byref(cfg)) == 0
    return h


def _call(lib, fn, h, pr, out):
    op = pr.op
    f0 = None if op.field0 is None else torch.as_tensor(op.field0, device="cuda")
    f1 = None if op.field1 is None else torch.as_tensor(op.field1, device="cuda")
    kop = _lib.KpOp(op.kind, op.nx, op.ny, 0, op.dx, op.dy, op.nu, op.nu2, op.ax, op.ay,
                    op.react, op.brus_a, op.brus_b,
                    None if f0 is None else ctypes.c_void_p(f0.data_ptr()),
                    None if f1 is None else ctypes.c_void_p(f1.data_ptr()))
    B = torch.as_tensor(np.asfortranarray(pr.B[:, :pr.p + 1]).ravel(order="F"), device="cuda")
    info = _lib.KpInfo()
    rc = fn(h, ctypes.byref(kop), ctypes.c_void_p(B.data_ptr()), pr.p, op.n, pr.h, pr.tol,
            pr.m_max, ctypes.c_void_p(out.data_ptr()), ctypes.byref(info))
    torch.cuda.synchronize()
    return rc, info.as_dict()


@pytest.mark.parametrize("orth", [0, 3])
def test_noalloc_matches_the_allocating_call(orth):
    lib = _lib.load()
    stream = torch.cuda.current_stream()
    h = _ctx(lib, stream, orth=orth)
    try:
        big = W.random_problem(201, kind=W.OP_ALLEN_CAHN, nx=160, ny=150, p=2, h=0.1,
                               m_max=48, tol=1e-8)
        small = W.random_problem(202, kind=W.OP_ADR, nx=61, ny=37, p=3, h=0.05, m_max=32,
                                 tol=1e-9, with_diag=True)
        for pr in (big, small):
            ya = torch.empty(pr.op.n, dtype=torch.float64, device="cuda")
            yb = torch.full((pr.op.n,), float("nan"), dtype=torch.float64, device="cuda")
            rc_a, ia = _call(lib, lib.kp_phi_combo, h, pr, ya)
            rc_b, ib = _call(lib, lib.kp_phi_combo_noalloc, h, pr, yb)
            assert rc_a == 0 and rc_b == 0
            assert ia["status"] == 0 and ib == ia
            a, b = ya.cpu().numpy(), yb.cpu().numpy()
            err = np.linalg.norm(a - b) / np.linalg.norm(a)
            print(f"N={pr.op.n} substeps={ib['substeps']} rel={err:.2e}")
            assert err <= 1e-10
            assert np.array_equal(a, b)            # the same kernels and geometry
            # the schedule log afterwards is this call's
            tau = (ctypes.c_double * 64)()
            m = (ctypes.c_int32 * 64)()
            assert lib.kp_get_schedule(h, tau, m, 64) == ib["substeps"]
    finally:
        lib.kp_destroy(h)


def test_noalloc_refuses_a_problem_beyond_the_array():
    lib = _lib.load()
    h = _ctx(lib, torch.cuda.current_stream())
    try:
        pr = W.random_problem(203, kind=W.OP_ADR, nx=512, ny=512, p=1, h=0.05, m_max=64)
        out = torch.empty(pr.op.n, dtype=torch.float64, device="cuda")
        rc, _ = _call(lib, lib.kp_phi_combo_noalloc, h, pr, out)
        assert rc == _lib.KP_ETOOLARGE
        assert b"exceeds the static scratch" in lib.kp_last_error(h)
    finally:
        lib.kp_destroy(h)
