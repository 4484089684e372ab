"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/esmf.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "esmf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(esmf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2002_00322_amd import _native
    L = _native.lib()
    names = _declared_symbols()
    assert "esmf_fock_build" in names and "esmf_eri_prepare" in names
    for name in names:
        assert hasattr(L, name), name
        assert name in _native.SIGNATURES, name


def test_status_strings():
    from paper_2002_00322_amd import _native
    L = _native.lib()
    assert L.esmf_status_string(0) == b"ESMF_OK"
    assert L.esmf_status_string(-1) == b"ESMF_ERR_INVALID_ARG"
    assert L.esmf_status_string(-4) == b"ESMF_ERR_NOT_SUPPORTED"


def _prepare_raw(n, centers, alpha, tau, storage=0):
    from paper_2002_00322_amd import _native as nat
    h = ctypes.c_void_p()
    c = np.ascontiguousarray(centers, dtype=np.float64)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    st = nat.lib().esmf_eri_prepare(n, c.ctypes.data_as(nat._dp), a.ctypes.data_as(nat._dp),
                                    tau, storage, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("case", ["n0", "neg_exp", "zero_exp", "nan_exp", "nan_centre",
                                  "neg_tau", "inf_tau", "bad_storage"])
def test_prepare_rejects_invalid_arguments(case):
    from paper_2002_00322_amd import _native as nat
    c = np.zeros((4, 3))
    a = np.ones(4)
    n, tau, storage = 4, 1e-10, 0
    if case == "n0":
        n = 0
    elif case == "neg_exp":
        a[2] = -1.0
    elif case == "zero_exp":
        a[1] = 0.0
    elif case == "nan_exp":
        a[0] = np.nan
    elif case == "nan_centre":
        c[3, 1] = np.inf
    elif case == "neg_tau":
        tau = -1e-12
    elif case == "inf_tau":
        tau = np.inf
    elif case == "bad_storage":
        storage = 7
    st, h = _prepare_raw(n, c, a, tau, storage)
    assert st == nat.ESMF_ERR_INVALID_ARG
    assert not h.value
    assert nat.lib().esmf_last_error() != b""


def test_build_rejects_invalid_arguments():
    from paper_2002_00322_amd import _native as nat
    L = nat.lib()
    vp = ctypes.c_void_p
    assert L.esmf_fock_build(None, 1, vp(16), vp(4096), vp(8192), 0, None) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_eri_release(None) == nat.ESMF_OK
    info = nat.EriInfo()
    assert L.esmf_eri_info_get(None, ctypes.byref(info)) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_fock_build_batched(-1, None, None, None, None, None, 0, None) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_fock_build_batched(0, None, None, None, None, None, 0, None) == nat.ESMF_OK
    rep = nat.TuneReport()
    assert L.esmf_fock_tune(None, 8, 0, None, ctypes.byref(rep)) == nat.ESMF_ERR_INVALID_ARG
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert L.esmf_timing_collect(None, ctypes.byref(n)) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_timing_collect(ctypes.byref(ms), ctypes.byref(n)) == nat.ESMF_OK and n.value == 0
    assert L.esmf_eri_lookup(None, 0, None, None, None, None, None) == nat.ESMF_ERR_INVALID_ARG


def test_python_errors_are_exceptions():
    import paper_2002_00322_amd as pa
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore(np.zeros((3, 3)), np.array([1.0, -1.0, 1.0]), 1e-10)
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore(np.zeros((3, 2)), np.ones(3), 1e-10)


def test_server_rejects_invalid_arguments_before_device_work():
    from paper_2002_00322_amd import _native as nat
    L = nat.lib()
    assert ctypes.sizeof(nat.ServerConfig) == 40 and ctypes.sizeof(nat.ServerStats) == 56
    h = ctypes.c_void_p()

    def cfg(**kw):
        base = dict(nstreams=2, max_group=4, max_inflight=1, prec=nat.PREC_FP64,
                    storage=nat.STORE_FP64, reserved=0, hbm_budget_bytes=1 << 30,
                    workspace_limit_bytes=1 << 30)
        base.update(kw)
        return nat.ServerConfig(**base)

    bad = [cfg(nstreams=0), cfg(nstreams=17), cfg(max_group=0), cfg(max_inflight=0),
           cfg(prec=7), cfg(storage=5), cfg(prec=nat.PREC_FP64, storage=nat.STORE_FP32),
           cfg(prec=nat.PREC_STORE32, storage=nat.STORE_FP64), cfg(hbm_budget_bytes=-1),
           cfg(prec=nat.PREC_MIXED, storage=nat.STORE_DIRECT),
           cfg(prec=nat.PREC_STORE32, storage=nat.STORE_DIRECT)]
    for c in bad:
        assert L.esmf_server_create(ctypes.byref(c), ctypes.byref(h)) == nat.ESMF_ERR_INVALID_ARG
        assert not h.value
    assert L.esmf_server_create(None, ctypes.byref(h)) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_server_create(ctypes.byref(cfg()), None) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_server_destroy(None) == nat.ESMF_OK
    rid = ctypes.c_int64()
    sid = ctypes.c_int32()
    assert L.esmf_server_submit(None, 1, 1, None, None, None, None, ctypes.byref(rid)) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_server_wait(None, 1, None) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_server_open_session(None, 4, None, None, 0.0, ctypes.byref(sid), None) == \
        nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_server_close_session(None, 1) == nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_server_stats_get(None, None) == nat.ESMF_ERR_INVALID_ARG


def test_esmf_terms_reject_invalid_arguments_before_device_work():
    from paper_2002_00322_amd import _native as nat
    L = nat.lib()
    vp = ctypes.c_void_p
    # distinct fake device addresses, far apart: never dereferenced on the host
    p = [vp(0x100000 * (i + 1)) for i in range(7)]
    inv = nat.ESMF_ERR_INVALID_ARG
    for n, no, nv in [(0, 1, 1), (4, 0, 4), (4, 2, 0), (-3, 1, 1), (40000, 1, 1), (8, 40000, 1)]:
        assert L.esmf_nine_densities(n, no, nv, *p, None) == inv
    assert L.esmf_nine_densities(8, 4, 4, None, *p[1:], None) == inv
    assert L.esmf_nine_densities(8, 4, 4, *p[:6], None, None) == inv
    # d overlapping an input: d = theta + 8 bytes
    assert L.esmf_nine_densities(8, 4, 4, p[0], p[1], p[2], p[3], p[4], p[5], vp(0x100008), None) == inv
    assert L.esmf_energy_two_body(0, 1.0, 1.0, p[0], p[1], p[2], p[3], None) == inv
    assert L.esmf_energy_two_body(8, 1.0, 1.0, None, p[1], p[2], p[3], None) == inv
    assert L.esmf_energy_two_body(8, 1.0, 1.0, p[0], p[1], p[2], None, None) == inv
    assert L.esmf_energy_two_body(8, float("nan"), 1.0, p[0], p[1], p[2], p[3], None) == inv
    assert L.esmf_energy_two_body(8, 1.0, float("inf"), p[0], p[1], p[2], p[3], None) == inv
    # e2 inside d (third matrix), j or k
    for e2 in (vp(0x100000 + 2 * 64 * 8 + 8), vp(0x200000 + 64 * 8), vp(0x300000 + 2 * 64 * 8 - 8)):
        assert L.esmf_energy_two_body(8, 1.0, 1.0, p[0], p[1], p[2], e2, None) == inv


def test_energy_gradient_rejects_invalid_arguments_before_device_work():
    from paper_2002_00322_amd import _native as nat
    L = nat.lib()
    vp = ctypes.c_void_p
    p = [vp(0x1000000 * (i + 1)) for i in range(11)]
    inv = nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_energy_gradient(0, 1, 1, 1.0, 1.0, *p, None) == inv
    assert L.esmf_energy_gradient(8, 4, 0, 1.0, 1.0, *p, None) == inv
    assert L.esmf_energy_gradient(8, 4, 4, 1.0, 0.0, *p, None) == inv
    assert L.esmf_energy_gradient(8, 4, 4, float("nan"), 1.0, *p, None) == inv
    assert L.esmf_energy_gradient(8, 4, 4, 1.0, 1.0, None, *p[1:], None) == inv
    # d_theta (output 9) on top of theta (input 0)
    q = list(p)
    q[9] = p[0]
    assert L.esmf_energy_gradient(8, 4, 4, 1.0, 1.0, *q, None) == inv


def test_prepare_cart_rejects_invalid_arguments_before_device_work():
    import paper_2002_00322_amd as pa
    A = np.zeros((2, 3))
    A[1, 0] = 1.0
    al = np.ones(2)
    for bad in ([[1, 1, 1], [0, 0, 0]], [[3, 0, 0], [0, 0, 0]], [[-1, 0, 0], [0, 0, 0]]):
        with pytest.raises(pa.InvalidArgument):
            pa.EriStore(A, al, 1e-10, lmn=np.array(bad))
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore(A, al, 1e-10, lmn=np.zeros((3, 3)))
    with pytest.raises(pa.NotSupported):
        pa.EriStore(A, al, 1e-10, storage=pa.STORE_DIRECT, lmn=np.array([[1, 0, 0], [0, 0, 0]]))


def test_prepare_contracted_rejects_invalid_arguments_before_device_work():
    import paper_2002_00322_amd as pa
    import workloads as wl
    cen, L, off, pe, pc = wl.contracted_basis(np.zeros((1, 3)))
    bad = off.copy()
    bad[2] = bad[1]
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore.contracted(cen, L, bad, pe, pc, 0.0)
    many = np.arange(cen.shape[0] + 1, dtype=np.int32) * 17  # 17 primitives per function
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore.contracted(cen, L, many, np.ones(int(many[-1])), np.ones(int(many[-1])), 0.0)
    with pytest.raises(pa.InvalidArgument):
        pa.EriStore.contracted(cen, L, off, pe, np.full_like(pc, np.nan), 0.0)
    with pytest.raises(pa.NotSupported):
        pa.EriStore.contracted(cen, L, off, pe, pc, 0.0, storage=pa.STORE_DIRECT)


def test_peak_probe_rejects_invalid_arguments_before_device_work():
    from paper_2002_00322_amd import _native as nat
    L = nat.lib()
    out = nat.Peaks()
    inv = nat.ESMF_ERR_INVALID_ARG
    assert L.esmf_probe_peaks(1 << 30, None, None) == inv
    assert L.esmf_probe_peaks((1 << 20) - 1, None, ctypes.byref(out)) == inv
    assert L.esmf_probe_peaks((64 << 30) + 1, None, ctypes.byref(out)) == inv


_STRUCTS = {"esmf_eri_info": "EriInfo", "esmf_tune_report": "TuneReport", "esmf_batch_report": "BatchReport",
            "esmf_server_config": "ServerConfig", "esmf_server_stats": "ServerStats", "esmf_peaks": "Peaks"}


def test_struct_layouts_match_the_header(tmp_path):
    # a C program compiled against include/esmf.h prints every struct's size
    # and its fields' offsets; the ctypes mirrors must agree field by field
    import shutil
    import subprocess
    from paper_2002_00322_amd import _native as nat
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = ["#include <stddef.h>", "#include <stdio.h>", '#include "esmf.h"', "int main(void) {"]
    for cname, pname in _STRUCTS.items():
        cls = getattr(nat, pname)
        src.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            src.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    src += ["    return 0;", "}"]
    (tmp_path / "layout.c").write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(tmp_path / "layout.c"),
                           "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, pname in _STRUCTS.items():
        cls = getattr(nat, pname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)
