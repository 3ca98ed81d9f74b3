"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point include/fastcpd.h declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2006_06281_amd as fc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastcpd.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpd(?:net)?_[a-z_0-9]+)\s*\(", src)))


def test_header_declarations_are_exported():
    lib = fc.load_library()
    names = _declared()
    assert "cpd_init" in names and "cpd_register" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", fc.LIB_PATH], capture_output=True,
                         text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_binding_names_match_header():
    assert sorted(fc.EXPORTED) == _declared()


def test_params_struct_layout():
    # 4 int32, 4 double, 6 int32, uint64, double, 2 int32
    assert ctypes.sizeof(fc.cpd_params) == 4 * 4 + 4 * 8 + 6 * 4 + 8 + 8 + 2 * 4
    assert fc.cpd_params.seed.offset % 8 == 0


def test_abi_version_and_build_info():
    lib = fc.load_library()
    assert lib.cpd_abi_version() == fc.CPD_ABI_VERSION
    assert b"gfx950" in lib.cpd_build_info()


def _ws(**kw):
    a = dict(M=100, N=120)
    a.update(kw)
    return fc.cpd_workspace_size(fc.make_params(**a))


def test_workspace_size_grows_with_problem():
    assert _ws() > 0
    assert _ws(M=2000, N=2000) > _ws()
    assert _ws(precision="fp64") > _ws(precision="fp32")


@pytest.mark.parametrize("bad", [
    dict(M=0), dict(N=0), dict(D=4), dict(D=0), dict(beta=0.0), dict(beta=-1.0),
    dict(lam=0.0), dict(w=1.0), dict(w=-0.1), dict(method=7), dict(precision=9),
    dict(eig_mode=5), dict(eig_mode="topk", K=0), dict(eig_mode="topk", K=101),
    dict(eig_mode="import", K=0), dict(tol=-1.0), dict(max_iter=0),
    dict(sigma2_init=float("nan")), dict(beta=float("inf")),
])
def test_bad_params_are_rejected(bad):
    with pytest.raises(fc.FastCPDError) as e:
        _ws(**bad)
    assert e.value.status == fc.CPD_E_ARG


def test_flags_and_version_fields():
    p = fc.make_params(10, 10)
    p.flags = 4  # not a CPD_FLAG_* bit
    with pytest.raises(fc.FastCPDError):
        fc.cpd_workspace_size(p)
    # the sorted layout carries the permutation, key and tile-box buffers
    sizes = [fc.cpd_workspace_size(fc.make_params(5000, 3000, sort=s, cull=c))
             for s, c in ((False, False), (True, False), (True, True))]
    assert sizes[0] < sizes[1] < sizes[2]
    p = fc.make_params(10, 10)
    p.abi_version = 99
    with pytest.raises(fc.FastCPDError):
        fc.cpd_workspace_size(p)


def test_null_arguments():
    lib = fc.load_library()
    p = fc.make_params(10, 10)
    assert lib.cpd_workspace_size(ctypes.byref(p), None) == fc.CPD_E_ARG
    assert lib.cpd_workspace_size(None, ctypes.byref(ctypes.c_size_t())) == fc.CPD_E_ARG
    h = ctypes.c_void_p()
    # NULL X/Y are rejected before any device call
    assert lib.cpd_init(ctypes.byref(h), ctypes.byref(p), None, None, None, 0, None) == fc.CPD_E_ARG
    assert h.value is None
    assert lib.cpd_step(None, None) == fc.CPD_E_ARG
    assert lib.cpd_eig_prepare(None, None, None, None) == fc.CPD_E_ARG
    assert lib.cpd_register(None, None, None, None, None) == fc.CPD_E_ARG
    assert lib.cpd_estep(None, None, None, None, None) == fc.CPD_E_ARG
    assert lib.cpd_destroy(None) == fc.CPD_OK


def test_workspace_checks_precede_device_checks():
    lib = fc.load_library()
    p = fc.make_params(10, 10)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert lib.cpd_init(ctypes.byref(h), ctypes.byref(p), fake, fake, None, 0, None) == fc.CPD_E_WORKSPACE
    mis = ctypes.c_void_p(0x1008)
    assert lib.cpd_init(ctypes.byref(h), ctypes.byref(p), fake, fake, mis, 1 << 30, None) == fc.CPD_E_WORKSPACE
    assert lib.cpd_init(ctypes.byref(h), ctypes.byref(p), fake, fake, fake, 16, None) == fc.CPD_E_WORKSPACE


def test_no_device_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib = fc.load_library()
    p = fc.make_params(10, 10)
    n = fc.cpd_workspace_size(p)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x100000)
    assert lib.cpd_init(ctypes.byref(h), ctypes.byref(p), fake, fake, fake, n, None) == fc.CPD_E_DEVICE
    assert b"device" in lib.cpd_last_error(None)


def test_status_strings():
    for s in (fc.CPD_OK, fc.CPD_E_ARG, fc.CPD_E_NUMERIC, fc.CPD_E_UNSUPPORTED):
        assert fc.status_name(s).startswith("CPD_")


def test_network_workspace_depends_on_precision_and_rejects_unknown_ones():
    lib = fc.load_library()
    n16, n32 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.cpdnet_workspace_size(2, 300, 200, fc.CPDNET_BF16, ctypes.byref(n16)) == fc.CPD_OK
    assert lib.cpdnet_workspace_size(2, 300, 200, fc.CPDNET_FP32, ctypes.byref(n32)) == fc.CPD_OK
    assert n32.value > n16.value > 0
    assert lib.cpdnet_workspace_size(2, 300, 200, 7, ctypes.byref(n16)) == fc.CPD_E_ARG
    assert lib.cpdnet_forward(None, None, None, 1, 10, 10, 7, None, None, 0, None) == fc.CPD_E_ARG
