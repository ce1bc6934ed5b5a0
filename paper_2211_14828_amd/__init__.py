"""rBKI-TK / rBKI-TK-TR on MI355X: Python binding of the C-ABI library.

Argument marshalling only: every step of the decomposition runs in the HIP
kernels of ``librbkitk.so``.  PyTorch provides device memory (inputs, outputs
and the workspace) and the current HIP stream.  There is no CPU fallback: if
the library is missing or no GPU is visible, the calls raise.

    core, factors, rel_err = tucker(X, ranks, p=5, q=2, seed=0)
    cores, rel_err = htr(X, tucker_ranks, tr_ranks, p=6, q=2, seed=0)
    Qt, width = basis(X, mode, ranks, p, q, seed)          # Alg. 1, one mode
    with Server(hbm_bytes, slots) as sv:                    # many small solves
        t = sv.submit(X, ranks); core, factors, err, ms = sv.wait(t)
"""
import atexit
import ctypes
import os
import threading

__all__ = ["tucker", "tucker_adaptive", "htr", "basis", "sym_eig", "sym_eig_top", "omega", "philox", "workspace_bytes", "profile_enable",
           "profile_reset", "profile_read", "Server", "library_path", "load_library", "RbkiError",
           "PLAIN", "MIXED_BF16", "MIXED_FP8", "SYMBOLS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librbkitk.so")

PLAIN, MIXED_BF16, MIXED_FP8 = 0, 1, 2
_PRECISIONS = {"plain": PLAIN, "mixed_bf16": MIXED_BF16, "bf16": MIXED_BF16, "mixed_fp8": MIXED_FP8,
               "fp8": MIXED_FP8}
_F64, _F32, _BF16 = 0, 1, 2
_STATUS = {0: "RBKI_OK", 1: "RBKI_E_INVALID", 2: "RBKI_E_NOMEM", 3: "RBKI_E_HIP", 4: "RBKI_E_NOCONV",
           5: "RBKI_E_UNSUPPORTED"}

# Every symbol the header declares.
SYMBOLS = ("rbki_version", "rbki_last_error", "rbki_omega", "rbki_philox", "rbki_basis_workspace",
           "rbki_basis", "rbki_tucker_workspace", "rbki_tucker", "rbki_htr_workspace", "rbki_htr",
           "rbki_basis_rows", "rbki_release", "rbki_tucker_adaptive_workspace", "rbki_tucker_adaptive",
           "rbki_htr_als_workspace", "rbki_htr_als", "rbki_tucker_noalloc_limit", "rbki_tucker_noalloc",
           "rbki_sym_eig_workspace", "rbki_sym_eig", "rbki_sym_eig_top_workspace", "rbki_sym_eig_top",
           "rbki_profile_enable", "rbki_profile_reset", "rbki_profile_read", "rbki_server_request_bytes", "rbki_server_create", "rbki_server_submit",
           "rbki_server_poll", "rbki_server_wait", "rbki_server_destroy", "rbki_tucker_result_bytes",
           "rbki_tucker_enqueue", "rbki_tucker_result")


class RbkiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("dims", ctypes.POINTER(ctypes.c_int64)),
                ("ranks", ctypes.POINTER(ctypes.c_int64)), ("oversample", ctypes.c_int),
                ("power", ctypes.c_int), ("seed", ctypes.c_uint64), ("precision", ctypes.c_int),
                ("variant", ctypes.c_int), ("sample_rate", ctypes.c_double), ("truncation", ctypes.c_int)]


_lib = None
_lock = threading.Lock()


def library_path():
    return _LIB_PATH


def load_library(build_if_missing=True):
    """Load librbkitk.so (building it first only if it does not exist)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            if not build_if_missing:
                raise ImportError(f"{_LIB_PATH} is not built")
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        vp, i64, u64, ci, sz, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
        sig = {
            "rbki_version": (ctypes.c_char_p, []),
            "rbki_last_error": (ctypes.c_char_p, []),
            "rbki_omega": (ci, [u64, ci, i64, i64, ci, vp, vp]),
            "rbki_philox": (ci, [vp, i64, u64, vp, vp]),
            "rbki_basis_workspace": (sz, [P(_Params), ci, ci]),
            "rbki_basis": (ci, [vp, ci, P(_Params), ci, vp, P(i64), vp, sz, vp]),
            "rbki_basis_rows": (i64, [P(_Params), ci, ci]),
            "rbki_release": (None, []),
            "rbki_tucker_adaptive_workspace": (sz, [P(_Params), ci]),
            "rbki_tucker_adaptive": (ci, [vp, ci, P(_Params), dbl, vp, P(vp), ci, vp, sz, P(dbl), P(ci), vp]),
            "rbki_tucker_workspace": (sz, [P(_Params), ci]),
            "rbki_tucker": (ci, [vp, ci, P(_Params), vp, P(vp), ci, vp, sz, P(dbl), vp]),
            "rbki_tucker_result_bytes": (sz, []),
            "rbki_tucker_enqueue": (ci, [vp, ci, P(_Params), vp, P(vp), ci, vp, sz, vp, vp]),
            "rbki_tucker_result": (ci, [vp, P(dbl)]),
            "rbki_htr_workspace": (sz, [P(_Params), ci, P(i64)]),
            "rbki_htr": (ci, [vp, ci, P(_Params), P(i64), P(vp), ci, vp, sz, P(dbl), vp]),
            "rbki_htr_als_workspace": (sz, [P(_Params), ci, P(i64)]),
            "rbki_tucker_noalloc_limit": (sz, []),
            "rbki_tucker_noalloc": (ci, [vp, ci, P(_Params), vp, P(vp), ci, P(dbl), vp]),
            "rbki_htr_als": (ci, [vp, ci, P(_Params), P(i64), ci, dbl, P(vp), ci, vp, sz, P(dbl), P(ci), vp]),
            "rbki_sym_eig_workspace": (sz, [i64]),
            "rbki_sym_eig": (ci, [vp, i64, vp, vp, vp, sz, P(ci), vp]),
            "rbki_sym_eig_top_workspace": (sz, [i64, i64]),
            "rbki_sym_eig_top": (ci, [vp, i64, i64, vp, vp, vp, sz, vp]),
            "rbki_profile_enable": (None, [ci]),
            "rbki_profile_reset": (None, []),
            "rbki_profile_read": (ci, [ctypes.c_char_p, P(i64), P(dbl)]),
            "rbki_server_request_bytes": (sz, [P(_Params), ci]),
            "rbki_server_create": (ci, [sz, ci, P(vp)]),
            "rbki_server_submit": (ci, [vp, vp, ci, P(_Params), vp, P(vp), ci, P(u64)]),
            "rbki_server_poll": (ci, [vp, u64, P(ci), P(dbl), P(dbl)]),
            "rbki_server_wait": (ci, [vp, u64, P(dbl), P(dbl)]),
            "rbki_server_destroy": (ci, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        # release the library's own streams and events while the HIP runtime
        # is still up (atexit handlers run before the runtime's teardown)
        atexit.register(lib.rbki_release)
        return lib


def _check(status):
    if status != 0:
        raise RbkiError(status, load_library().rbki_last_error().decode())


# ------------------------------------------------------------------ helpers

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("rbkitk needs a GPU (HIP device); none is visible")
    return torch


def _dtype_code(torch, dt):
    if dt == torch.float64:
        return _F64
    if dt == torch.float32:
        return _F32
    if dt == torch.bfloat16:
        return _BF16
    raise TypeError(f"unsupported tensor dtype {dt}")


_VARIANTS = {"krylov": 0, "power": 1}


_TRUNCATIONS = {"independent": 0, "sequential": 1}


def _params(dims, ranks, p, q, seed, precision, variant="krylov", sample_rate=1.0, truncation="independent"):
    n = len(dims)
    if len(ranks) != n:
        raise ValueError("ranks must have one entry per mode")
    d = (ctypes.c_int64 * n)(*[int(v) for v in dims])
    r = (ctypes.c_int64 * n)(*[int(v) for v in ranks])
    prec = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prm = _Params(n, ctypes.cast(d, ctypes.POINTER(ctypes.c_int64)), ctypes.cast(r, ctypes.POINTER(ctypes.c_int64)),
                  int(p), int(q), int(seed) & 0xFFFFFFFFFFFFFFFF, prec,
                  _VARIANTS[variant] if isinstance(variant, str) else int(variant), float(sample_rate),
                  _TRUNCATIONS[truncation] if isinstance(truncation, str) else int(truncation))
    prm._keep = (d, r)
    return prm


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


_ws_cache = {}


def _workspace(torch, device, nbytes):
    """A device buffer of at least nbytes, reused across calls on the device."""
    key = str(device)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def _as_input(torch, X):
    if not X.is_cuda:
        raise ValueError("X must be a GPU tensor")
    return X.contiguous()


# ------------------------------------------------------------------ public API

def workspace_bytes(dims, ranks, p, q, dtype, precision="plain", tr_ranks=None, variant="krylov", sample_rate=1.0,
                    truncation="independent"):
    lib = load_library()
    import torch
    prm = _params(dims, ranks, p, q, 0, precision, variant, sample_rate, truncation)
    code = _dtype_code(torch, dtype)
    if tr_ranks is not None:
        tr = (ctypes.c_int64 * len(tr_ranks))(*tr_ranks)
        return lib.rbki_htr_workspace(ctypes.byref(prm), code, tr)
    return lib.rbki_tucker_workspace(ctypes.byref(prm), code)


def tucker(X, ranks, p=5, q=2, seed=0, precision="plain", out_dtype=None, rel_err=True, stream=None,
           workspace=None, variant="krylov", sample_rate=1.0, truncation="independent"):
    """rBKI-TK (Alg. 2).  Returns (core, [U^(1), ..., U^(N)], rel_err or None).
    variant "power": each factor from the power iterate (XX^T)^q W alone
    (the power-iteration comparison of Sec. 3.1).  sample_rate < 1: each
    mode's Krylov basis from that fraction of the unfolding's columns
    (Sec. 3.1).  truncation "sequential": each mode's factor from the tensor
    already projected on the earlier modes (ST-HOSVD form)."""
    torch = _torch()
    lib = load_library()
    X = _as_input(torch, X)
    code = _dtype_code(torch, X.dtype)
    if out_dtype is None:
        out_dtype = torch.float64 if X.dtype == torch.float64 else torch.float32
    ocode = _dtype_code(torch, out_dtype)
    prm = _params(X.shape, ranks, p, q, seed, precision, variant, sample_rate, truncation)
    need = lib.rbki_tucker_workspace(ctypes.byref(prm), code)
    if need == 0:
        _check(lib.rbki_tucker(None, code, ctypes.byref(prm), None, None, ocode, None, 0, None, None))
    ws = workspace if workspace is not None else _workspace(torch, X.device, need)
    core = torch.empty(tuple(int(r) for r in ranks), dtype=out_dtype, device=X.device)
    factors = [torch.empty((int(I), int(R)), dtype=out_dtype, device=X.device) for I, R in zip(X.shape, ranks)]
    fptr = (ctypes.c_void_p * len(factors))(*[f.data_ptr() for f in factors])
    err = ctypes.c_double(0.0)
    _check(lib.rbki_tucker(ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm), ctypes.c_void_p(core.data_ptr()),
                           fptr, ocode, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                           ctypes.byref(err) if rel_err else None, _stream(torch, stream)))
    return core, factors, (err.value if rel_err else None)


def tucker_result_buffer():
    """Page-locked host memory for one tucker_enqueue result."""
    torch = _torch()
    return torch.empty(int(load_library().rbki_tucker_result_bytes()), dtype=torch.uint8, pin_memory=True)


def tucker_enqueue(X, ranks, result, p=5, q=2, seed=0, precision="plain", out_dtype=None, stream=None,
                   workspace=None, variant="krylov", sample_rate=1.0, truncation="independent"):
    """tucker() without waiting for the stream: the same work, the explicit
    error included.  `result` (tucker_result_buffer()) receives the error sums
    when the stream gets there; tucker_result(result) then returns rel_err.
    Calls that share a workspace must be issued on one stream.  Returns
    (core, [U^(1), ..., U^(N)])."""
    torch = _torch()
    lib = load_library()
    X = _as_input(torch, X)
    code = _dtype_code(torch, X.dtype)
    if out_dtype is None:
        out_dtype = torch.float64 if X.dtype == torch.float64 else torch.float32
    ocode = _dtype_code(torch, out_dtype)
    prm = _params(X.shape, ranks, p, q, seed, precision, variant, sample_rate, truncation)
    need = lib.rbki_tucker_workspace(ctypes.byref(prm), code)
    if need == 0:
        _check(lib.rbki_tucker(None, code, ctypes.byref(prm), None, None, ocode, None, 0, None, None))
    if result.numel() < lib.rbki_tucker_result_bytes() or result.device.type != "cpu":
        raise ValueError("result must be a tucker_result_buffer()")
    ws = workspace if workspace is not None else _workspace(torch, X.device, need)
    core = torch.empty(tuple(int(r) for r in ranks), dtype=out_dtype, device=X.device)
    factors = [torch.empty((int(I), int(R)), dtype=out_dtype, device=X.device) for I, R in zip(X.shape, ranks)]
    fptr = (ctypes.c_void_p * len(factors))(*[f.data_ptr() for f in factors])
    _check(lib.rbki_tucker_enqueue(ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm),
                                   ctypes.c_void_p(core.data_ptr()), fptr, ocode, ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel(), ctypes.c_void_p(result.data_ptr()), _stream(torch, stream)))
    return core, factors


def tucker_result(result):
    """rel_err of a tucker_enqueue call whose work the stream has passed."""
    err = ctypes.c_double(0.0)
    _check(load_library().rbki_tucker_result(ctypes.c_void_p(result.data_ptr()), ctypes.byref(err)))
    return err.value


def tucker_adaptive(X, ranks, p=5, max_q=20, fit_tol=1e-3, seed=0, precision="plain", out_dtype=None,
                    stream=None, sample_rate=1.0):
    """rBKI-TK with q chosen by the stopping rule of Sec. 4 (stop once the
    Fit changes by at most fit_tol between Krylov steps).  Returns
    (core, [U^(1), ..., U^(N)], rel_err, q_used)."""
    torch = _torch()
    lib = load_library()
    X = _as_input(torch, X)
    code = _dtype_code(torch, X.dtype)
    if out_dtype is None:
        out_dtype = torch.float64 if X.dtype == torch.float64 else torch.float32
    ocode = _dtype_code(torch, out_dtype)
    prm = _params(X.shape, ranks, p, max_q, seed, precision, "krylov", sample_rate)
    need = lib.rbki_tucker_adaptive_workspace(ctypes.byref(prm), code)
    if need == 0:
        _check(lib.rbki_tucker_adaptive(None, code, ctypes.byref(prm), float(fit_tol), None, None, ocode, None, 0,
                                        None, None, None))
    ws = _workspace(torch, X.device, need)
    core = torch.empty(tuple(int(r) for r in ranks), dtype=out_dtype, device=X.device)
    factors = [torch.empty((int(I), int(R)), dtype=out_dtype, device=X.device) for I, R in zip(X.shape, ranks)]
    fptr = (ctypes.c_void_p * len(factors))(*[f.data_ptr() for f in factors])
    err = ctypes.c_double(0.0)
    qu = ctypes.c_int(0)
    _check(lib.rbki_tucker_adaptive(ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm), float(fit_tol),
                                    ctypes.c_void_p(core.data_ptr()), fptr, ocode, ctypes.c_void_p(ws.data_ptr()),
                                    ws.numel(), ctypes.byref(err), ctypes.byref(qu), _stream(torch, stream)))
    return core, factors, err.value, qu.value


def htr(X, tucker_ranks, tr_ranks, p=5, q=2, seed=0, precision="plain", out_dtype=None, rel_err=True,
        stream=None, variant="krylov", sample_rate=1.0, truncation="independent", method="svd", max_sweeps=20,
        fit_tol=1e-3, return_sweeps=False):
    """rBKI-TK-TR (Alg. 3).  method "svd": TR-SVD of the core; "als": TR-ALS
    sweeps from the TR-SVD cores (stopping rule of Sec. 4).  Returns
    ([X_1, ..., X_N], rel_err or None) (and the sweeps taken with
    return_sweeps)."""
    torch = _torch()
    lib = load_library()
    X = _as_input(torch, X)
    code = _dtype_code(torch, X.dtype)
    if out_dtype is None:
        out_dtype = torch.float64 if X.dtype == torch.float64 else torch.float32
    ocode = _dtype_code(torch, out_dtype)
    N = X.dim()
    prm = _params(X.shape, tucker_ranks, p, q, seed, precision, variant, sample_rate, truncation)
    tr = (ctypes.c_int64 * N)(*[int(v) for v in tr_ranks])
    als = method == "als"
    if method not in ("svd", "als"):
        raise ValueError("method must be 'svd' or 'als'")
    need = (lib.rbki_htr_als_workspace if als else lib.rbki_htr_workspace)(ctypes.byref(prm), code, tr)
    if need == 0:
        if als:
            _check(lib.rbki_htr_als(None, code, ctypes.byref(prm), tr, int(max_sweeps), float(fit_tol), None, ocode,
                                    None, 0, None, None, None))
        _check(lib.rbki_htr(None, code, ctypes.byref(prm), tr, None, ocode, None, 0, None, None))
    ws = _workspace(torch, X.device, need)
    r = [int(tr_ranks[-1])] + [int(v) for v in tr_ranks]
    cores = [torch.empty((r[n], int(X.shape[n]), r[n + 1]), dtype=out_dtype, device=X.device) for n in range(N)]
    cptr = (ctypes.c_void_p * N)(*[c.data_ptr() for c in cores])
    err = ctypes.c_double(0.0)
    sweeps = ctypes.c_int(0)
    if als:
        _check(lib.rbki_htr_als(ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm), tr, int(max_sweeps),
                                float(fit_tol), cptr, ocode, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.byref(err) if rel_err else None, ctypes.byref(sweeps), _stream(torch, stream)))
    else:
        _check(lib.rbki_htr(ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm), tr, cptr, ocode,
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(err) if rel_err else None,
                            _stream(torch, stream)))
    if return_sweeps:
        return cores, (err.value if rel_err else None), sweeps.value
    return cores, (err.value if rel_err else None)


def basis(X, mode, ranks, p=5, q=2, seed=0, precision="plain", stream=None, variant="krylov", sample_rate=1.0):
    """Alg. 1 for one mode.  Returns (Qt as a float64 (S' x I_n) tensor whose
    first `width` rows are the orthonormal basis, width)."""
    torch = _torch()
    lib = load_library()
    X = _as_input(torch, X)
    code = _dtype_code(torch, X.dtype)
    prm = _params(X.shape, ranks, p, q, seed, precision, variant, sample_rate)
    need = lib.rbki_basis_workspace(ctypes.byref(prm), code, int(mode))
    if need == 0:
        _check(lib.rbki_basis(None, code, ctypes.byref(prm), int(mode), None, None, None, 0, None))
    ws = _workspace(torch, X.device, need)
    I = int(X.shape[mode])
    rows = lib.rbki_basis_rows(ctypes.byref(prm), code, int(mode))
    Qt = torch.empty((rows, I), dtype=torch.float64, device=X.device)
    width = ctypes.c_int64(0)
    _check(lib.rbki_basis(ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm), int(mode),
                          ctypes.c_void_p(Qt.data_ptr()), ctypes.byref(width), ctypes.c_void_p(ws.data_ptr()),
                          ws.numel(), _stream(torch, stream)))
    return Qt, width.value


def sym_eig(Z, stream=None):
    """Eigenvalues (descending) and eigenvectors (rows) of a symmetric PSD
    float64 device matrix by the device Jacobi solver.  Returns (lam, Vt, sweeps)."""
    torch = _torch()
    lib = load_library()
    Z = Z.contiguous()
    if Z.dtype != torch.float64 or Z.dim() != 2 or Z.shape[0] != Z.shape[1]:
        raise ValueError("Z must be a square float64 tensor")
    n = int(Z.shape[0])
    ws = _workspace(torch, Z.device, lib.rbki_sym_eig_workspace(n))
    lam = torch.empty(n, dtype=torch.float64, device=Z.device)
    Vt = torch.empty((n, n), dtype=torch.float64, device=Z.device)
    sweeps = ctypes.c_int(0)
    _check(lib.rbki_sym_eig(ctypes.c_void_p(Z.data_ptr()), n, ctypes.c_void_p(lam.data_ptr()),
                            ctypes.c_void_p(Vt.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            ctypes.byref(sweeps), _stream(torch, stream)))
    return lam, Vt, sweeps.value


def sym_eig_top(Z, k, stream=None):
    """The k largest eigenvalues (descending) and their eigenvectors (rows) of
    a symmetric PSD float64 device matrix (tridiagonal reduction, bisection,
    inverse iteration).  Returns (lam, Vt)."""
    torch = _torch()
    lib = load_library()
    Z = Z.contiguous()
    if Z.dtype != torch.float64 or Z.dim() != 2 or Z.shape[0] != Z.shape[1]:
        raise ValueError("Z must be a square float64 tensor")
    n, k = int(Z.shape[0]), int(k)
    ws = _workspace(torch, Z.device, lib.rbki_sym_eig_top_workspace(n, k))
    lam = torch.empty(max(k, 0), dtype=torch.float64, device=Z.device)
    Vt = torch.empty((max(k, 0), n), dtype=torch.float64, device=Z.device)
    _check(lib.rbki_sym_eig_top(ctypes.c_void_p(Z.data_ptr()), n, k, ctypes.c_void_p(lam.data_ptr()),
                                ctypes.c_void_p(Vt.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                _stream(torch, stream)))
    return lam, Vt


def omega(seed, mode, J, S, dtype=None, device="cuda", stream=None):
    """Omega^(n)T (S x J) of the sketch stream, on the device."""
    torch = _torch()
    lib = load_library()
    dtype = dtype or torch.float64
    out = torch.empty((int(S), int(J)), dtype=dtype, device=device)
    _check(lib.rbki_omega(int(seed), int(mode), int(J), int(S), _dtype_code(torch, dtype),
                          ctypes.c_void_p(out.data_ptr()), _stream(torch, stream)))
    return out


def philox(counters, seed, stream=None):
    """Raw Philox4x32-10 blocks for counters (count x 4, int32 or uint32 bit
    patterns on the device); returns count x 4 int32 bit patterns."""
    torch = _torch()
    lib = load_library()
    c = counters.contiguous()
    if c.dtype not in (torch.int32, torch.uint32) or c.dim() != 2 or c.shape[1] != 4:
        raise ValueError("counters must be a (count, 4) 32-bit integer tensor")
    out = torch.empty_like(c)
    _check(lib.rbki_philox(ctypes.c_void_p(c.data_ptr()), int(c.shape[0]), int(seed), ctypes.c_void_p(out.data_ptr()),
                           _stream(torch, stream)))
    return out


def profile_enable(on=True):
    load_library().rbki_profile_enable(1 if on else 0)


def profile_reset():
    load_library().rbki_profile_reset()


def profile_read(kernel):
    lib = load_library()
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(lib.rbki_profile_read(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


class Server:
    """Request server for many small rBKI-TK solves (continuous batching).

    One device arena of ``hbm_bytes`` is allocated at construction; ``slots``
    worker threads, each with its own stream, admit queued requests in order as
    their workspace fits the free arena memory, so several solves run on the
    device at once.  ``submit`` returns a ticket at once; ``wait`` / ``poll``
    return (core, factors, rel_err, latency_ms).  The output tensors and the
    input are held until the ticket is collected."""

    def __init__(self, hbm_bytes, slots=4, device=None):
        torch = _torch()
        self._torch = torch
        self._lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        h = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(self._lib.rbki_server_create(int(hbm_bytes), int(slots), ctypes.byref(h)))
        self._h = h
        self._held = {}

    def request_bytes(self, dims, ranks, p=5, q=2, dtype=None, precision="plain"):
        dtype = dtype or self._torch.float32
        prm = _params(dims, ranks, p, q, 0, precision)
        return self._lib.rbki_server_request_bytes(ctypes.byref(prm), _dtype_code(self._torch, dtype))

    def submit(self, X, ranks, p=5, q=2, seed=0, precision="plain", out_dtype=None, variant="krylov",
               sample_rate=1.0, truncation="independent"):
        torch = self._torch
        if self._h is None:
            raise RuntimeError("server is closed")
        X = _as_input(torch, X)
        code = _dtype_code(torch, X.dtype)
        if out_dtype is None:
            out_dtype = torch.float64 if X.dtype == torch.float64 else torch.float32
        ocode = _dtype_code(torch, out_dtype)
        prm = _params(X.shape, ranks, p, q, seed, precision, variant, sample_rate, truncation)
        core = torch.empty(tuple(int(r) for r in ranks), dtype=out_dtype, device=X.device)
        factors = [torch.empty((int(I), int(R)), dtype=out_dtype, device=X.device) for I, R in zip(X.shape, ranks)]
        fptr = (ctypes.c_void_p * len(factors))(*[f.data_ptr() for f in factors])
        # the request reads X on the server's (non-blocking) streams: wait
        # for the work queued so far on the caller's stream, which produced X,
        # and only for that
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(X.device))
        ev.synchronize()
        ticket = ctypes.c_uint64(0)
        _check(self._lib.rbki_server_submit(self._h, ctypes.c_void_p(X.data_ptr()), code, ctypes.byref(prm),
                                            ctypes.c_void_p(core.data_ptr()), fptr, ocode, ctypes.byref(ticket)))
        self._held[ticket.value] = (X, core, factors)
        return ticket.value

    def _collect(self, ticket):
        _, core, factors = self._held.pop(ticket, (None, None, None))
        return core, factors

    def poll(self, ticket):
        """None while running, else (core, factors, rel_err, latency_ms)."""
        done = ctypes.c_int(0)
        err = ctypes.c_double(0.0)
        ms = ctypes.c_double(0.0)
        st = self._lib.rbki_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(err),
                                        ctypes.byref(ms))
        if st == 0 and not done.value:
            return None
        core, factors = self._collect(ticket)
        _check(st)
        return core, factors, err.value, ms.value

    def wait(self, ticket):
        err = ctypes.c_double(0.0)
        ms = ctypes.c_double(0.0)
        st = self._lib.rbki_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(err), ctypes.byref(ms))
        core, factors = self._collect(ticket)
        _check(st)
        return core, factors, err.value, ms.value

    def close(self):
        if self._h is not None:
            _check(self._lib.rbki_server_destroy(self._h))
            self._h = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
