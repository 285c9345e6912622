"""CPU checks of the C ABI: the library loads, exports every symbol declared in
include/mgl.h, and its host-only entry points (parameter count, workspace
sizing with CSR validation) behave as documented.  No GPU work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from mginputs import configs as Cf, hierarchy as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2608_29082_amd import binding as Bd
    if not os.path.exists(Bd.LIB_PATH):
        pytest.skip("libmgl.so not built")
    return Bd, Bd.load_library()


def test_header_symbols_exported():
    Bd, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "mgl.h")).read()
    declared = set(re.findall(r"\b(mg_[a-z_]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", Bd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mg_[a-z_]+)", out))
    assert declared and declared <= exported, declared - exported
    assert declared == set(Bd.EXPORTED)


def test_num_params_layout():
    Bd, lib = _lib()
    assert lib.mg_num_params(7, 3, 3, 3) == 84
    assert lib.mg_num_params(4, 2, 2, 2) == 3 * 11
    assert lib.mg_num_params(1, 2, 2, 2) == -1
    assert lib.mg_num_params(4, 2, 2, 2) == Cf.n_params(4, 2, 2, 2)


def _sizes(Bd, lib, hier, K=2, B=1, prec="fp64", flags=0, A=None, P=None):
    hh = Bd._HostHierarchy(A or hier.A, P or hier.P)
    flat = np.ascontiguousarray(Cf.identity_params(hier.nlevels, K, K, K))
    p = Bd._Params(K, K, K, 2, 2, flat.ctypes.data_as(C.POINTER(C.c_double)))
    o = Bd._Options(Bd.PRECISIONS[prec], B, 100, 10, 1e-8, 1e6, flags)
    ws, ck = C.c_size_t(), C.c_size_t()
    st = lib.mg_workspace_bytes(C.byref(hh.h), C.byref(p), C.byref(o), C.byref(ws), C.byref(ck))
    return st, ws.value, ck.value


def test_workspace_bytes_scale_with_batch_and_precision():
    Bd, lib = _lib()
    hier = H.square_hierarchy(33)
    st, ws1, ck1 = _sizes(Bd, lib, hier, B=1)
    assert st == 0 and ws1 > 0 and ck1 > 0
    st, ws64, ck64 = _sizes(Bd, lib, hier, B=64)
    assert st == 0 and ws64 > 20 * ws1 // 2
    n_tot = sum(hier.sizes)
    assert ck64 >= 2 * n_tot * 64 * 8            # f and u per level in FP64
    st, ws32, ck32 = _sizes(Bd, lib, hier, B=64, prec="fp32")
    assert st == 0 and ck32 < ck64
    st, wsb, _ = _sizes(Bd, lib, hier, B=64, flags=Bd.FLAG_BACKWARD)
    assert wsb > ws64


def test_malformed_inputs_rejected_on_host():
    Bd, lib = _lib()
    hier = H.square_hierarchy(17)
    # P with the wrong shape
    badP = [sp.csr_matrix(hier.P[0][:, :-1])] + hier.P[1:]
    st, _, _ = _sizes(Bd, lib, hier, P=badP)
    assert st == 2 and b"P[0]" in lib.mg_last_error()
    # unsorted columns in A
    A0 = hier.A[0].copy()
    A0.indices[[0, 1]] = A0.indices[[1, 0]]
    st, _, _ = _sizes(Bd, lib, hier, A=[A0] + hier.A[1:])
    assert st == 2 and b"sorted" in lib.mg_last_error()
    # batch width out of range
    st, _, _ = _sizes(Bd, lib, hier, B=0)
    assert st == 1
    st, _, _ = _sizes(Bd, lib, hier, B=257)
    assert st == 1


def test_helmholtz_header_symbols_exported():
    """Every entry point of include/mgh.h is exported and bound."""
    Bd, lib = _lib()
    from paper_2608_29082_amd import helmholtz as HB
    hdr = open(os.path.join(ROOT, "include", "mgh.h")).read()
    declared = set(re.findall(r"\b(mgh_[a-z_]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", Bd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mgh_[a-z_]+)", out))
    assert declared and declared <= exported, declared - exported
    assert declared == set(HB.EXPORTED)
    HB.load_library()
    assert lib.mgh_num_params(5, 1, 1, 1) == Cf.hz_n_params(5, 1, 1, 1) == 4 * 10 + 8 + 8
    assert lib.mgh_num_params(1, 1, 1, 1) == -1


def test_helmholtz_setup_rejects_bad_input_before_any_device_work():
    """mgh_setup validates its arguments on the host (no GPU needed for the
    rejected cases)."""
    Bd, lib = _lib()
    from paper_2608_29082_amd import helmholtz as HB
    from mginputs import helmholtz as HZ
    HB.load_library()
    h = HZ.hierarchy(9, 3.0, 2)
    host = HB._Host(h.A, h.P)
    vals = np.ascontiguousarray(Cf.hz_identity_params(2, 1, 1, 1, [("jacobi", 1, 1)]))
    ip = C.POINTER(C.c_int32)
    sm, pre, post = (np.array([0], dtype=np.int32), np.array([1], dtype=np.int32), np.array([1], dtype=np.int32))

    def call(KB=1, v=4, prec=0, B=1, smk=0, hier=None):
        sm[0] = smk
        p = HB._HParams(KB, 1, 1, sm.ctypes.data_as(ip), pre.ctypes.data_as(ip), post.ctypes.data_as(ip), v,
                        vals.ctypes.data_as(C.POINTER(C.c_double)))
        o = HB._HOptions(prec, B)
        out = C.c_void_p()
        return lib.mgh_setup(C.byref(hier or host.h), C.byref(p), C.byref(o), None, C.byref(out))
    assert call(KB=9) == 1
    assert call(v=0) == 1 and call(v=9) == 1
    assert call(prec=2) == 1
    assert call(B=0) == 1 and call(B=257) == 1
    assert call(smk=2) == 1
    bad = HB._Host([h.A[0], h.A[0]], h.P)           # P has the wrong column count
    assert call(hier=bad.h) == 2
    assert b"P_0" in lib.mgh_last_error()
