"""Seeded synthetic inputs, shared by the oracle's tests and by the GPU path.

This module only *makes data*: it holds none of the decomposition method's
arithmetic.  The generators follow the paper's own data recipes:

* noise: X = X_c + lambda N with N i.i.d. N(0, 1) and lambda chosen from the
  realised norms so that SNR(dB) = 20 log10(||X_c||_F / ||lambda N||_F) holds
  exactly (Sec. 4.1.1, eq. (16));
* Gaussian random Tucker tensors: core and factors i.i.d. N(0, 1)
  (Sec. 4.1.1, first bullet);
* power-functional tensors x_{i,j,k} = (i^p + j^p + k^p)^(-1/p) with 1-based
  indices and p = 10 (Sec. 4.1.1, eq. (17));
* tensor-ring tensors (Def. 2, eq. (3)) with Gaussian cores;

and the fixed workloads used for parity and measurement (orthonormal factors
from the QR of a Gaussian matrix with the signs fixed so that diag(R) > 0).

Host generation uses NumPy's PCG64 stream; the multi-GB workloads can also be
generated on the GPU with a seeded torch generator (a different stream, so a
given test uses one source for both the GPU run and the oracle).
"""
import math

import numpy as np

# -------------------------------------------------------------------- helpers


def _rng(seed):
    return np.random.default_rng(int(seed))


def orthonormal_columns(rng, n, r):
    """Q of the QR of an n x r standard Gaussian matrix, with diag(R) > 0."""
    Q, R = np.linalg.qr(rng.standard_normal((n, r)))
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn


def tucker_full(G, factors):
    """G x_1 U1 x_2 U2 ... x_N UN for row-major arrays (data assembly)."""
    X = np.asarray(G, np.float64)
    for n, U in enumerate(factors):
        X = np.moveaxis(np.tensordot(U, X, axes=([1], [n])), 0, n)
    return np.ascontiguousarray(X)


def tr_full(cores):
    """Full tensor of a tensor ring (eq. (3)) for row-major cores (r, I, r'),
    one slab X[i_1] at a time: the chain G_1[:, i_1, :] G_2 ... G_{N-1} keeps
    the closing index a as a free index, and the slab is one product with
    G_N arranged as [(a, r_{N-1}), i_N], which closes the ring (sums over a).
    No intermediate holds the two-ended chain of the whole tensor (64 times
    the tensor for a 64^5 ring of rank 8)."""
    dims = [int(C.shape[1]) for C in cores]
    r0, rl = int(cores[0].shape[0]), int(cores[-1].shape[0])
    L = np.ascontiguousarray(np.transpose(cores[-1], (2, 0, 1)).reshape(r0 * rl, dims[-1]))
    X = np.empty(dims, dtype=np.float64)
    for i in range(dims[0]):
        T = np.asarray(cores[0][:, i, :], np.float64)              # (a, r_1)
        for C in cores[1:-1]:
            T = np.tensordot(T, C, axes=([T.ndim - 1], [0]))       # (a, I_2..I_k, r_k)
        T = np.moveaxis(T, 0, -2)                                  # (I_2..I_{N-1}, a, r_{N-1})
        X[i] = (T.reshape(-1, r0 * rl) @ L).reshape(dims[1:])
    return X


def noise_scale(clean_norm, noise_norm, snr_db):
    """lambda with 20 log10(||X_c|| / ||lambda N||) = snr_db (eq. (16))."""
    return clean_norm / (noise_norm * 10.0 ** (snr_db / 20.0))


def add_noise(Xc, snr_db, rng, dtype=np.float64):
    """Xc + lambda N rounded to dtype, N ~ N(0, 1) drawn in one call (row-major
    order), lambda from the realised norms (eq. (16)).  The sum is formed in
    float64 and rounded once, slab by slab, so that a multi-GB tensor needs
    no full-size temporary beyond N and the result."""
    N = rng.standard_normal(Xc.shape)
    lam = noise_scale(np.linalg.norm(Xc.ravel()), np.linalg.norm(N.ravel()), snr_db)
    out = np.empty(Xc.shape, dtype=dtype)
    xf, nf, of = Xc.reshape(-1), N.reshape(-1), out.reshape(-1)
    step = 1 << 24
    for s in range(0, xf.size, step):
        of[s:s + step] = xf[s:s + step] + lam * nf[s:s + step]
    return out


# ------------------------------------------------------ the paper's generators


def gaussian_tucker(dims, ranks, seed):
    """Tucker tensor with N(0,1) core and N(0,1) factors (Sec. 4.1.1)."""
    rng = _rng(seed)
    G = rng.standard_normal(tuple(ranks))
    factors = [rng.standard_normal((I, R)) for I, R in zip(dims, ranks)]
    return tucker_full(G, factors)


def power_functional(dims, p=10):
    """x_{i1..iN} = (sum_k i_k^p)^(-1/p), 1-based (eq. (17))."""
    grids = np.meshgrid(*[np.arange(1, I + 1, dtype=np.float64) for I in dims], indexing="ij")
    s = sum(g ** p for g in grids)
    return s ** (-1.0 / p)


def noisy(Xc, snr_db, seed):
    return add_noise(np.asarray(Xc, np.float64), snr_db, _rng(seed))


# ------------------------------------------------------------- fixed workloads


def orthonormal_tucker(dims, ranks, seed, factor_decay=None, core_decay=None):
    """Clean Tucker tensor with an N(0,1) core and orthonormal factors.
    factor_decay = "inverse" scales column k (1-based) of every factor by 1/k;
    core_decay = rho multiplies the core by diag(rho^k), k = 0.., in every mode."""
    rng = _rng(seed)
    G = rng.standard_normal(tuple(ranks))
    if core_decay is not None:
        for n, R in enumerate(ranks):
            shape = [1] * len(ranks)
            shape[n] = R
            G = G * (core_decay ** np.arange(R, dtype=np.float64)).reshape(shape)
    factors = []
    for I, R in zip(dims, ranks):
        U = orthonormal_columns(rng, I, R)
        if factor_decay == "inverse":
            U = U / np.arange(1, R + 1, dtype=np.float64)
        factors.append(U)
    return tucker_full(G, factors), rng


def tensor_ring_data(dims, tr_rank, seed, var):
    rng = _rng(seed)
    cores = [rng.standard_normal((tr_rank, I, tr_rank)) * math.sqrt(var) for I in dims]
    return tr_full(cores), rng


# Workloads.  "seeds" are (data seed, sketch seed).
WORKLOADS = {
    # Plain rBKI-TK, FP64, 64^3, Tucker ranks 8, 20 dB, p=5, q=2.
    "tucker64_f64": dict(dims=(64, 64, 64), ranks=(8, 8, 8), p=5, q=2, snr=20.0,
                         dtype="float64", kind="tucker", seeds=(101, 201)),
    # Plain vs mixed, 400^3 FP32, ranks 20, factor columns scaled 1/k, 10 dB,
    # p=10, q=3.
    "tucker400_f32": dict(dims=(400, 400, 400), ranks=(20, 20, 20), p=10, q=3, snr=10.0,
                          dtype="float32", kind="tucker", factor_decay="inverse",
                          seeds=(102, 202)),
    # Hierarchical TR, 64^5 FP32 from a ring of ranks 8 with N(0, 1/8) cores,
    # 15 dB, Tucker ranks 16, p=6, q=2, TR ranks 8.
    "ring64x5_f32": dict(dims=(64,) * 5, ranks=(16,) * 5, p=6, q=2, snr=15.0,
                         dtype="float32", kind="ring", tr_rank=8, tr_var=1.0 / 8,
                         tr_ranks=(8,) * 5, seeds=(103, 203)),
    # Large rBKI-TK, 1000^3 FP32, ranks 50, core x_n diag(0.95^k), 10 dB,
    # p=10, q=4.
    "tucker1000_f32": dict(dims=(1000, 1000, 1000), ranks=(50, 50, 50), p=10, q=4,
                           snr=10.0, dtype="float32", kind="tucker", core_decay=0.95,
                           seeds=(105, 205)),
}


def scaled_workload(name, dims=None, ranks=None, **over):
    """A copy of a workload recipe with other sizes (same structure)."""
    w = dict(WORKLOADS[name])
    if dims is not None:
        w["dims"] = tuple(dims)
    if ranks is not None:
        w["ranks"] = tuple(ranks)
    w.update(over)
    return w


def make_host(w):
    """Generate a workload on the host: returns (X in w's dtype, X_clean fp64)."""
    seed = w["seeds"][0]
    if w["kind"] == "tucker":
        Xc, rng = orthonormal_tucker(w["dims"], w["ranks"], seed,
                                     factor_decay=w.get("factor_decay"),
                                     core_decay=w.get("core_decay"))
    elif w["kind"] == "ring":
        Xc, rng = tensor_ring_data(w["dims"], w["tr_rank"], seed, w["tr_var"])
    else:
        raise ValueError(w["kind"])
    if w.get("snr") is not None:
        X = add_noise(Xc, w["snr"], rng, dtype=np.dtype(w["dtype"]))
    else:
        X = Xc.astype(w["dtype"])
    return np.ascontiguousarray(X), Xc


def make_device(w, device="cuda"):
    """Generate a workload directly in GPU memory with a seeded torch
    generator (for the multi-GB sizes).  Returns X as a torch tensor of w's
    dtype.  Assembly runs in float64 and is rounded once at the end."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(w["seeds"][0]))
    f64 = dict(dtype=torch.float64, device=device, generator=gen)
    dims = tuple(w["dims"])
    if w["kind"] == "tucker":
        ranks = tuple(w["ranks"])
        G = torch.randn(ranks, **f64)
        if w.get("core_decay") is not None:
            for n, R in enumerate(ranks):
                shape = [1] * len(ranks)
                shape[n] = R
                dec = w["core_decay"] ** torch.arange(R, dtype=torch.float64, device=device)
                G = G * dec.reshape(shape)
        X = G
        for n, (I, R) in enumerate(zip(dims, ranks)):
            Q, Rm = torch.linalg.qr(torch.randn((I, R), **f64))
            sgn = torch.sign(torch.diagonal(Rm))
            sgn[sgn == 0] = 1.0
            U = Q * sgn
            if w.get("factor_decay") == "inverse":
                U = U / torch.arange(1, R + 1, dtype=torch.float64, device=device)
            X = torch.movedim(torch.tensordot(U, X, dims=([1], [n])), 0, n).contiguous()
    elif w["kind"] == "ring":
        r = int(w["tr_rank"])
        cores = [torch.randn((r, I, r), **f64) * math.sqrt(w["tr_var"]) for I in dims]
        # one slab X[i_1] at a time, the closing index kept free (as tr_full)
        L = cores[-1].permute(2, 0, 1).reshape(r * r, dims[-1]).contiguous()
        X = torch.empty(dims, dtype=torch.float64, device=device)
        for i in range(dims[0]):
            T = cores[0][:, i, :]
            for C in cores[1:-1]:
                T = torch.tensordot(T, C, dims=([T.ndim - 1], [0]))
            T = torch.movedim(T, 0, -2).reshape(-1, r * r)
            X[i] = (T @ L).reshape(dims[1:])
            del T
    else:
        raise ValueError(w["kind"])
    if w.get("snr") is not None:
        cn = torch.linalg.vector_norm(X).item()
        N = torch.randn(X.shape, **f64)
        lam = noise_scale(cn, torch.linalg.vector_norm(N).item(), w["snr"])
        X.add_(N, alpha=lam)
        del N
    dt = {"float64": torch.float64, "float32": torch.float32, "bfloat16": torch.bfloat16}[w["dtype"]]
    return X.to(dt).contiguous()


def fingerprint(X):
    """Float64 sums over the stored values of X (slab by slab) and 32 stored
    values at fixed linear indices: identifies a generated tensor, so that a
    stored result computed on it elsewhere can be matched to it."""
    flat = np.asarray(X).reshape(-1)
    n2 = 0.0
    a1 = 0.0
    step = 1 << 24
    for s in range(0, flat.size, step):
        c = flat[s:s + step].astype(np.float64)
        n2 += float(np.dot(c, c))
        a1 += float(np.sum(np.abs(c)))
    idx = np.random.default_rng(12345).integers(0, flat.size, size=32)
    return {"norm2": n2, "abs_sum": a1, "index": [int(i) for i in idx],
            "values": [float(flat[i]) for i in idx]}


def same_fingerprint(a, b):
    """The two fingerprints describe the same tensor: equal sampled values,
    and sums that agree to 1e-10 (float64 sums of the same values taken in
    another order, on another machine, differ by about 1e-13)."""
    return (a["index"] == b["index"] and a["values"] == b["values"]
            and abs(a["norm2"] - b["norm2"]) <= 1e-10 * abs(b["norm2"])
            and abs(a["abs_sum"] - b["abs_sum"]) <= 1e-10 * abs(b["abs_sum"]))


# ------------------------------------------------------------ served request mix


def served_requests(count=2000, seed=7, lo=32, hi=256):
    """Request recipes of the served mix: third-order tensors with dims
    U{lo..hi}, ranks r ~ U{4..32} capped at dim//2, Gaussian core,
    orthonormal factors, SNR ~ U[5, 30] dB, stored as bf16, p = 5,
    q ~ U{1, 2, 3}, Poisson arrivals (unit-rate inter-arrival gaps; the
    caller scales them).  Request i uses data seed 10^6 + i and sketch seed
    2 * 10^6 + i."""
    rng = _rng(seed)
    reqs = []
    t = 0.0
    for i in range(count):
        dims = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        ranks = tuple(int(min(r, d // 2)) for r, d in zip(rng.integers(4, 33, size=3), dims))
        snr = float(rng.uniform(5.0, 30.0))
        q = int(rng.integers(1, 4))
        t += float(rng.exponential(1.0))
        reqs.append(dict(dims=dims, ranks=ranks, p=5, q=q, snr=snr, dtype="bfloat16",
                         kind="tucker", seeds=(10 ** 6 + i, 2 * 10 ** 6 + i), arrival=t))
    return reqs
