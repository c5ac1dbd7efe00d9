"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments before touching the GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2410_14917_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "krylov_phi.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(kp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_expected_functions():
    decl = _declared_functions()
    assert set(decl) == set(_lib.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_constants_match_header():
    text = open(HEADER).read()
    for name in ("KP_OK", "KP_EINVAL", "KP_EUNSUPPORTED", "KP_ORTH_H_GSMGS", "KP_ORTH_H_NCWY",
                 "KP_ORTH_MGS", "KP_ORTH_IOCGS", "KP_CTRL_PI", "KP_RHS_ADR", "KP_SRERK3",
                 "KP_EPI5", "KP_OP_BRUSSELATOR", "KP_BASIS_F32", "KP_MMAX", "KP_PMAX",
                 "KP_STATUS_NONFINITE"):
        m = re.search(rf"#define\s+{name}\s+(-?\d+)", text)
        assert m and int(m.group(1)) == getattr(_lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals the C
    compiler's for the header."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"kp_op": _lib.KpOp, "kp_config": _lib.KpConfig, "kp_info": _lib.KpInfo,
               "kp_rhs": _lib.KpRhs}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "krylov_phi.h"',
             "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_version_and_strerror():
    lib = _lib.load()
    assert lib.kp_version() == 10300
    assert lib.kp_strerror(-1) == b"invalid argument"
    assert lib.kp_strerror(12345) == b"unknown error"


def _ctx(**kw):
    lib = _lib.load()
    cfg = _lib.KpConfig(None, 0, 0, 0, 0, 0, 0, 0.0, 0.0, 0.0, 0, 0)
    for k, v in kw.items():
        setattr(cfg, k, v)
    h = ctypes.c_void_p()
    rc = lib.kp_create(ctypes.byref(h), ctypes.byref(cfg))
    return lib, h, rc


@pytest.mark.parametrize("field,val", [("orth", 7), ("orth", 5), ("basis_dtype", 3), ("m_init", 65), ("controller", 2), ("rows_per_wg", -1),
                                       ("m_init", -1), ("tau_init", -1.0),
                                       ("tau_init", float("inf")), ("fixed_m", 65),
                                       ("max_substeps", -2)])
def test_create_rejects_bad_config(field, val):
    lib, h, rc = _ctx(**{field: val})
    assert rc == _lib.KP_EINVAL


def test_create_rejects_fixed_m_without_substeps():
    lib, h, rc = _ctx(fixed_m=10, fixed_substeps=0)
    assert rc == _lib.KP_EINVAL


FAKE = ctypes.c_void_p(0x10000)      # never dereferenced: validation comes first
FAKE2 = ctypes.c_void_p(0x90000000)


def _op(**kw):
    base = dict(kind=0, nx=8, ny=8, transpose=0, dx=0.125, dy=0.125, nu=0.01, nu2=0.0,
                ax=1.0, ay=0.5, react=0.0, brus_a=1.0, brus_b=3.0, field0=None, field1=None)
    base.update(kw)
    return _lib.KpOp(**base)


@pytest.mark.parametrize("opkw,args", [
    (dict(kind=5), {}),
    (dict(nx=0), {}),
    (dict(dx=0.0), {}),
    (dict(nu=float("nan")), {}),
    (dict(kind=1), {}),                      # Allen-Cahn needs field0
    (dict(kind=2, field0=0x20000), {}),      # Brusselator needs both fields
    ({}, dict(p=-1)),
    ({}, dict(p=9)),
    ({}, dict(ldb=63)),
    ({}, dict(m_max=0)),
    ({}, dict(m_max=65)),
    ({}, dict(tol=0.0)),
    ({}, dict(h=-1.0)),
    ({}, dict(h=float("inf"))),
    ({}, dict(out=None)),
    ({}, dict(out="overlap")),
])
def test_phi_combo_rejects_bad_arguments(opkw, args):
    lib, h, rc = _ctx()
    assert rc == 0
    try:
        op = _op(**opkw)
        a = dict(B=FAKE, p=2, ldb=64, h=0.1, tol=1e-8, m_max=10, out=FAKE2)
        a.update(args)
        if a["out"] == "overlap":
            a["out"] = ctypes.c_void_p(0x10000 + 8 * 10)
        rc = lib.kp_phi_combo(h, ctypes.byref(op), a["B"], a["p"], a["ldb"], a["h"], a["tol"],
                              a["m_max"], a["out"], None)
        assert rc == _lib.KP_EINVAL
    finally:
        lib.kp_destroy(h)


def test_step_before_begin_is_a_state_error():
    lib, h, rc = _ctx()
    try:
        assert lib.kp_arnoldi_step(h, 1) == _lib.KP_ESTATE
        assert lib.kp_arnoldi_read(h, None, None, None, None, None) == _lib.KP_ESTATE
    finally:
        lib.kp_destroy(h)


def test_null_context_is_invalid():
    lib = _lib.load()
    op = _op()
    assert lib.kp_phi_combo(None, ctypes.byref(op), FAKE, 2, 64, 0.1, 1e-8, 10, FAKE2, None) \
        == _lib.KP_EINVAL
    assert lib.kp_destroy(None) == _lib.KP_EINVAL
    assert lib.kp_create(None, None) == _lib.KP_EINVAL


def test_batched_rejects_empty_and_missing_arrays():
    """nprob < 1 and missing host arrays are refused before any device work."""
    lib, h, rc = _ctx()
    assert rc == 0
    try:
        op = _op()
        ops = (_lib.KpOp * 1)(op)
        Bp = (ctypes.c_void_p * 1)(FAKE.value)
        ps = (ctypes.c_int32 * 1)(2)
        lds = (ctypes.c_int64 * 1)(64)
        hs = (ctypes.c_double * 1)(0.1)
        outs = (ctypes.c_void_p * 1)(FAKE2.value)
        full = [ops, Bp, ps, lds, hs, outs]
        for nprob in (0, -3):
            assert lib.kp_phi_combo_batched(h, nprob, ops, Bp, ps, lds, hs, 1e-8, 10, outs,
                                            None) == _lib.KP_EINVAL
        for miss in range(len(full)):
            args = [None if i == miss else a for i, a in enumerate(full)]
            assert lib.kp_phi_combo_batched(h, 1, args[0], args[1], args[2], args[3], args[4],
                                            1e-8, 10, args[5], None) == _lib.KP_EINVAL
        assert lib.kp_phi_combo_batched(None, 1, ops, Bp, ps, lds, hs, 1e-8, 10, outs,
                                        None) == _lib.KP_EINVAL
    finally:
        lib.kp_destroy(h)


def test_integrate_rejects_bad_arguments():
    lib, h, rc = _ctx()
    assert rc == 0
    try:
        def rhs(**kw):
            base = dict(kind=0, nx=8, ny=8, reserved=0, dx=0.125, dy=0.125, nu=0.1, ax=0.0,
                        ay=0.0, gamma=0.0)
            base.update(kw)
            return _lib.KpRhs(**base)
        good = dict(method=0, dt=0.01, nsteps=2, start=4, u=FAKE, tol=1e-8, m_max=16)
        for r, kw in [(rhs(kind=2), {}), (rhs(nx=0), {}), (rhs(dx=0.0), {}),
                      (rhs(nu=float("nan")), {}), (rhs(), dict(method=3)),
                      (rhs(), dict(dt=0.0)), (rhs(), dict(nsteps=-1)), (rhs(), dict(start=0)),
                      (rhs(), dict(u=None)), (rhs(), dict(tol=0.0)), (rhs(), dict(m_max=65))]:
            a = dict(good)
            a.update(kw)
            assert lib.kp_integrate(h, ctypes.byref(r), a["method"], a["dt"], a["nsteps"],
                                    a["start"], a["u"], a["tol"], a["m_max"], None) \
                == _lib.KP_EINVAL, kw
    finally:
        lib.kp_destroy(h)



def test_default_build_records_no_timeline():
    """The timeline entry points exist in the default build: the layout is
    reported, recording is refused as unsupported, bad arguments are
    invalid (no GPU work)."""
    lib = _lib.load()
    slots, wgs = ctypes.c_int32(), ctypes.c_int32()
    assert lib.kp_timeline_layout(ctypes.byref(slots), ctypes.byref(wgs)) == 0
    assert (slots.value, wgs.value) == (8, 256)
    assert lib.kp_timeline_layout(None, ctypes.byref(wgs)) == _lib.KP_EINVAL
    h = ctypes.c_void_p()
    assert lib.kp_create(ctypes.byref(h), None) == 0
    try:
        assert lib.kp_set_timeline(h, FAKE, 16) == _lib.KP_EUNSUPPORTED
        assert lib.kp_set_timeline(h, None, 16) == _lib.KP_EINVAL
        assert lib.kp_set_timeline(h, FAKE, -1) == _lib.KP_EINVAL
    finally:
        lib.kp_destroy(h)
    assert lib.kp_set_timeline(None, FAKE, 16) == _lib.KP_EINVAL


def test_read_bandwidth_rejects_bad_arguments():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.kp_create(ctypes.byref(h), None) == 0
    out = ctypes.c_double()
    try:
        assert lib.kp_read_bandwidth(h, 1 << 30, 10, None) == _lib.KP_EINVAL
        assert lib.kp_read_bandwidth(h, 1 << 19, 10, ctypes.byref(out)) == _lib.KP_EINVAL
        assert lib.kp_read_bandwidth(h, 1 << 37, 10, ctypes.byref(out)) == _lib.KP_EINVAL
        assert lib.kp_read_bandwidth(h, 1 << 30, 0, ctypes.byref(out)) == _lib.KP_EINVAL
    finally:
        lib.kp_destroy(h)
    assert lib.kp_read_bandwidth(None, 1 << 30, 10, ctypes.byref(out)) == _lib.KP_EINVAL
