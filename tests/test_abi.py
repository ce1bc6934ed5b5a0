"""Host-side checks of the C-ABI library (no GPU needed): it is built for
gfx950, it loads, and it exports every entry point the header declares with
C linkage."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2211_14828_amd as rb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbkitk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbki_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert declared_functions() == sorted(rb.SYMBOLS)


def test_library_loads_and_exports_every_symbol():
    lib = rb.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rb.library_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rbki_\w+)", out))
    assert set(declared_functions()) <= exported
    assert lib.rbki_version().decode().startswith("rbkitk")


def test_library_holds_gfx950_code_objects():
    data = open(rb.library_path(), "rb").read()
    assert b"gfx950" in data


def test_oracle_is_not_linked_into_the_product():
    # the product package never imports the oracle
    pkg = os.path.join(ROOT, "paper_2211_14828_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def _params(dims, ranks, p=5, q=2, precision=0):
    n = len(dims)
    d = (ctypes.c_int64 * n)(*dims)
    r = (ctypes.c_int64 * n)(*ranks)
    prm = rb._Params(n, ctypes.cast(d, ctypes.POINTER(ctypes.c_int64)), ctypes.cast(r, ctypes.POINTER(ctypes.c_int64)),
                     p, q, 0, precision)
    prm._keep = (d, r)
    return prm


@pytest.mark.parametrize("dims,ranks,p,q,prec,why", [
    ((10, 10, 10), (11, 3, 3), 5, 2, 0, "rank above dim"),
    ((10, 10, 10), (0, 3, 3), 5, 2, 0, "zero rank"),
    ((10,), (3,), 5, 2, 0, "order 1"),
    ((10, 10, 10), (3, 3, 3), -1, 2, 0, "negative oversampling"),
    ((10, 10, 10), (3, 3, 3), 5, -2, 0, "negative q"),
    ((10, 10, 10), (3, 3, 3), 5, 2, 7, "unknown precision"),
    ((10, 0, 10), (3, 1, 3), 5, 2, 0, "empty mode"),
])
def test_invalid_arguments_are_rejected_before_any_launch(dims, ranks, p, q, prec, why):
    lib = rb.load_library()
    prm = _params(dims, ranks, p, q, prec)
    st = lib.rbki_tucker(ctypes.c_void_p(16), 1, ctypes.byref(prm), None, None, 1, None, 0, None, None)
    assert st == 1, why
    assert lib.rbki_last_error().decode()
    assert lib.rbki_tucker_workspace(ctypes.byref(prm), 1) == 0


def test_workspace_too_small_is_rejected():
    lib = rb.load_library()
    prm = _params((20, 20, 20), (3, 3, 3))
    need = lib.rbki_tucker_workspace(ctypes.byref(prm), 1)
    assert need > 0
    st = lib.rbki_tucker(ctypes.c_void_p(256), 1, ctypes.byref(prm), None, None, 1, ctypes.c_void_p(256), need - 1,
                         None, None)
    assert st == 1 and "workspace" in lib.rbki_last_error().decode()


def test_unknown_dtype_and_null_tensor_are_rejected():
    lib = rb.load_library()
    prm = _params((20, 20, 20), (3, 3, 3))
    assert lib.rbki_tucker(ctypes.c_void_p(256), 9, ctypes.byref(prm), None, None, 1, None, 0, None, None) == 1
    assert lib.rbki_tucker(None, 1, ctypes.byref(prm), None, None, 1, None, 0, None, None) == 1
    assert lib.rbki_tucker(ctypes.c_void_p(256), 1, ctypes.byref(prm), None, None, 2, None, 0, None, None) == 1


def test_server_rejects_bad_arguments_before_touching_the_device():
    lib = rb.load_library()
    out = ctypes.c_void_p(None)
    assert lib.rbki_server_create(1 << 30, 0, ctypes.byref(out)) == 1
    assert lib.rbki_server_create(1 << 30, 65, ctypes.byref(out)) == 1
    assert lib.rbki_server_create(1 << 10, 2, ctypes.byref(out)) == 1
    assert lib.rbki_server_create(1 << 30, 2, None) == 1
    assert out.value is None
    t = ctypes.c_uint64(0)
    prm = _params((20, 20, 20), (3, 3, 3))
    assert lib.rbki_server_submit(None, ctypes.c_void_p(256), 1, ctypes.byref(prm), None, None, 1, ctypes.byref(t)) == 1
    assert lib.rbki_server_destroy(None) == 0


def test_server_footprint_is_the_decomposition_workspace():
    lib = rb.load_library()
    for dims, ranks, q in [((20, 20, 20), (3, 3, 3), 2), ((256, 32, 100), (16, 16, 32), 3)]:
        prm = _params(dims, ranks, 5, q)
        for xt in (0, 1, 2):
            assert lib.rbki_server_request_bytes(ctypes.byref(prm), xt) == lib.rbki_tucker_workspace(ctypes.byref(prm), xt)
    bad = _params((10, 10, 10), (11, 3, 3))
    assert lib.rbki_server_request_bytes(ctypes.byref(bad), 1) == 0


def test_top_eigensolver_rejects_bad_sizes_before_any_launch():
    lib = rb.load_library()
    assert lib.rbki_sym_eig_top_workspace(0, 1) == 0
    assert lib.rbki_sym_eig_top_workspace(10, 11) == 0
    assert lib.rbki_sym_eig_top_workspace(513, 4) == 0
    need = lib.rbki_sym_eig_top_workspace(300, 50)
    assert need >= 300 * 300 * 8
    p = ctypes.c_void_p(256)
    assert lib.rbki_sym_eig_top(p, 300, 0, p, p, p, need, None) == 1
    assert lib.rbki_sym_eig_top(p, 600, 50, p, p, p, need, None) == 1
    assert lib.rbki_sym_eig_top(None, 300, 50, p, p, p, need, None) == 1
    assert lib.rbki_sym_eig_top(p, 300, 50, p, p, p, need - 1, None) == 1
    assert "workspace" in lib.rbki_last_error().decode()


def test_unknown_variant_is_rejected_and_the_power_basis_is_one_block_wide():
    lib = rb.load_library()
    prm = _params((40, 40, 40), (4, 4, 4), 4, 3, 0)
    krylov = lib.rbki_tucker_workspace(ctypes.byref(prm), 1)
    prm.variant = 1
    power = lib.rbki_tucker_workspace(ctypes.byref(prm), 1)
    # the power variant's basis is S wide instead of S (q + 1)
    assert 0 < power < krylov
    prm.variant = 7
    st = lib.rbki_tucker(ctypes.c_void_p(16), 1, ctypes.byref(prm), None, None, 1, None, 0, None, None)
    assert st == 1 and "variant" in lib.rbki_last_error().decode()
    assert lib.rbki_tucker_workspace(ctypes.byref(prm), 1) == 0


def test_sample_rate_is_validated_and_sizes_the_basis():
    lib = rb.load_library()
    prm = _params((40, 50, 30), (6, 6, 6), 5, 2, 0)
    full = lib.rbki_tucker_workspace(ctypes.byref(prm), 1)
    assert lib.rbki_basis_rows(ctypes.byref(prm), 1, 0) == 33      # S (q + 1) = 11 * 3 <= I
    prm.sample_rate = 1.0
    assert lib.rbki_tucker_workspace(ctypes.byref(prm), 1) == full
    prm.sample_rate = 0.01                                          # m = 15 columns of mode 0
    assert lib.rbki_tucker_workspace(ctypes.byref(prm), 1) > 0
    assert lib.rbki_basis_rows(ctypes.byref(prm), 1, 0) == 33
    prm.sample_rate = 0.005                                         # m = 8 < R + p in mode 0: S = 8
    assert lib.rbki_basis_rows(ctypes.byref(prm), 1, 0) == 24
    prm.sample_rate = 0.002                                         # m = 3 < R in mode 0: rejected
    assert lib.rbki_basis_rows(ctypes.byref(prm), 1, 0) == 0
    st = lib.rbki_tucker(ctypes.c_void_p(16), 1, ctypes.byref(prm), None, None, 1, None, 0, None, None)
    assert st == 1 and "fewer than its rank" in lib.rbki_last_error().decode()
    for bad in (-0.5, 1.5, float("nan")):
        prm.sample_rate = bad
        st = lib.rbki_tucker(ctypes.c_void_p(16), 1, ctypes.byref(prm), None, None, 1, None, 0, None, None)
        assert st == 1 and "sample_rate" in lib.rbki_last_error().decode()
        assert lib.rbki_tucker_workspace(ctypes.byref(prm), 1) == 0


def test_truncation_is_validated_and_sizes_its_workspace():
    lib = rb.load_library()
    prm = _params((40, 50, 30), (6, 6, 6), 5, 2, 0)
    indep = lib.rbki_tucker_workspace(ctypes.byref(prm), 1)
    prm.truncation = 1
    seq = lib.rbki_tucker_workspace(ctypes.byref(prm), 1)
    assert seq > indep > 0
    tr = (ctypes.c_int64 * 3)(2, 2, 2)
    assert lib.rbki_htr_workspace(ctypes.byref(prm), 1, tr) > seq
    prm.truncation = 5
    st = lib.rbki_tucker(ctypes.c_void_p(16), 1, ctypes.byref(prm), None, None, 1, None, 0, None, None)
    assert st == 1 and "truncation" in lib.rbki_last_error().decode()
    assert lib.rbki_tucker_workspace(ctypes.byref(prm), 1) == 0


def test_htr_als_arguments_are_checked():
    lib = rb.load_library()
    prm = _params((20, 20, 20), (6, 6, 6))
    tr = (ctypes.c_int64 * 3)(2, 2, 2)
    svd = lib.rbki_htr_workspace(ctypes.byref(prm), 1, tr)
    als = lib.rbki_htr_als_workspace(ctypes.byref(prm), 1, tr)
    assert als > svd > 0
    cores = (ctypes.c_void_p * 3)(16, 16, 16)
    for ms, tol in ((-1, 1e-3), (5000, 1e-3), (20, float("nan"))):
        st = lib.rbki_htr_als(ctypes.c_void_p(16), 1, ctypes.byref(prm), tr, ms, tol, cores, 1, ctypes.c_void_p(256),
                              als, None, None, None)
        assert st == 1
    big = (ctypes.c_int64 * 3)(65, 2, 2)
    st = lib.rbki_htr(ctypes.c_void_p(16), 1, ctypes.byref(prm), big, cores, 1, ctypes.c_void_p(256), 1 << 40, None,
                      None)
    assert st == 5


def test_enqueue_checks_its_result_buffer_and_arguments():
    lib = rb.load_library()
    prm = _params((20, 20, 20), (3, 3, 3))
    need = lib.rbki_tucker_workspace(ctypes.byref(prm), 1)
    nres = lib.rbki_tucker_result_bytes()
    assert nres > 0
    res = ctypes.create_string_buffer(nres)
    resp = ctypes.cast(res, ctypes.c_void_p)
    # no result buffer
    st = lib.rbki_tucker_enqueue(ctypes.c_void_p(256), 1, ctypes.byref(prm), None, None, 1, ctypes.c_void_p(256),
                                 need, None, None)
    assert st == 1 and "result" in lib.rbki_last_error().decode()
    # what rbki_tucker rejects (a workspace one byte short) is rejected before anything is enqueued
    st = lib.rbki_tucker_enqueue(ctypes.c_void_p(256), 1, ctypes.byref(prm), None, None, 1, ctypes.c_void_p(256),
                                 need - 1, resp, None)
    assert st == 1 and "workspace" in lib.rbki_last_error().decode()
    # a result with zero sums and no modes reads as error 0, status OK
    err = ctypes.c_double(-1.0)
    assert lib.rbki_tucker_result(ctypes.cast(ctypes.create_string_buffer(nres), ctypes.c_void_p),
                                  ctypes.byref(err)) == 0
    assert err.value == 0.0
    assert lib.rbki_tucker_result(None, ctypes.byref(err)) == 1
