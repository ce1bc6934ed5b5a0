"""rbki_tucker_noalloc (the workspace in the library's fixed device array)
against rbki_tucker (a caller workspace) through the C ABI: the same
kernels and launches, so the same results bit for bit, on two calls in a row
with the second smaller, and a problem beyond the array's size rejected."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2211_14828_amd as rb
    rb.load_library(build_if_missing=False)
    return torch, rb


def noalloc(torch, rb, X, ranks, p, q, seed, precision="plain"):
    lib = rb.load_library()
    prm = rb._params(X.shape, ranks, p, q, seed, precision)
    code = rb._dtype_code(torch, X.dtype)
    core = torch.empty(tuple(ranks), dtype=torch.float64, device=X.device)
    factors = [torch.empty((int(I), int(R)), dtype=torch.float64, device=X.device) for I, R in zip(X.shape, ranks)]
    fptr = (ctypes.c_void_p * len(factors))(*[f.data_ptr() for f in factors])
    err = ctypes.c_double(0.0)
    st = lib.rbki_tucker_noalloc(ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm),
                                 ctypes.c_void_p(core.data_ptr()), fptr, 0, ctypes.byref(err),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, core, factors, err.value


CASES = [
    # a larger problem, then a smaller one (the array keeps the first call's
    # contents when the second runs)
    [((130, 70, 150), (10, 8, 12), 5, 2, "float32", "plain"), ((37, 45, 29), (4, 5, 3), 5, 2, "float64", "plain")],
    [((300, 40, 270), (12, 6, 10), 5, 2, "float32", "mixed_fp8"), ((64, 50, 40), (6, 6, 6), 5, 1, "float32",
                                                                    "mixed_bf16")],
]


@pytest.mark.parametrize("pair", CASES)
def test_noalloc_equals_the_workspace_call(env, pair):
    torch, rb = env
    lib = rb.load_library()
    for dims, ranks, p, q, dtype, prec in pair:
        Xc, rng = synth.orthonormal_tucker(dims, ranks, 5 + sum(dims))
        X = synth.add_noise(Xc, 10.0, rng).astype(dtype)
        Xg = torch.from_numpy(X).cuda()
        prm = rb._params(dims, ranks, p, q, 9, prec)
        assert lib.rbki_tucker_workspace(ctypes.byref(prm), rb._dtype_code(torch, Xg.dtype)) <= \
            lib.rbki_tucker_noalloc_limit()
        st, core, factors, e = noalloc(torch, rb, Xg, ranks, p, q, 9, prec)
        assert st == 0, lib.rbki_last_error().decode()
        c2, f2, e2 = rb.tucker(Xg, ranks, p=p, q=q, seed=9, precision=prec, out_dtype=torch.float64)
        assert e == e2
        assert torch.equal(core, c2)
        for u, v in zip(factors, f2):
            assert torch.equal(u, v)


def test_noalloc_rejects_a_problem_beyond_its_array(env):
    torch, rb = env
    lib = rb.load_library()
    dims, ranks = (1000, 1000, 1000), (50, 50, 50)
    prm = rb._params(dims, ranks, 10, 4, 1, "plain")
    assert lib.rbki_tucker_workspace(ctypes.byref(prm), 1) > lib.rbki_tucker_noalloc_limit()
    core = (ctypes.c_void_p * 3)(16, 16, 16)
    st = lib.rbki_tucker_noalloc(ctypes.c_void_p(256), 1, ctypes.byref(prm), ctypes.c_void_p(256), core, 1, None,
                                 None)
    assert st == 1 and "fixed device scratch" in lib.rbki_last_error().decode()
