"""Tensor-ring model (Def. 2, eq. (3)), TR-SVD, and Alg. 3 (rBKI-TK-TR).

Alg. 3 cites TR-SVD (Zhao et al. 2016, "Tensor ring decomposition") for the
decomposition of the small core but does not restate it.  Written here from
that method's published description, with fixed ranks instead of an accuracy
threshold:

  with TR ranks (r_1, ..., r_N) and closing rank r_0 = r_N,
  1. unfold the tensor as S_1 x (S_2 ... S_N) and take its SVD; keep
     k = min(r_0 r_1, rank) triplets, zero-padded to r_0 r_1 columns;
  2. core 1 is the left factor reshaped to (S_1, r_0, r_1) with column
     c = a0 * r_1 + a1, permuted to (r_0, S_1, r_1);
  3. the remainder Sigma V^T is reshaped to (r_0, r_1, S_2, ..., S_N) and its
     r_0 axis moved last, giving (r_1, S_2, ..., S_N, r_0);
  4. for k = 2 .. N-1, unfold the remainder as (r_{k-1} S_k) x rest, SVD,
     keep r_k triplets (zero-padded), core k is the left factor reshaped to
     (r_{k-1}, S_k, r_k), the remainder is Sigma V^T;
  5. the last core is the remainder reshaped to (r_{N-1}, S_N, r_0).

Readings: Alg. 3 wraps "TR-ALS(G, R_n)" in a loop over n, but a TR-SVD yields
all cores at once, so it is run once; the contraction of step 4 attaches the
Tucker factor to the middle (dimension) mode of each core,
X_n = G_n x_2 U^(n) in R^{R_{n-1} x I_n x R_n}.

Because each step's left factor has orthonormal columns, the squared error
||G - TR(cores)||_F^2 equals the sum of the squared discarded singular values
over all steps when r_0 r_1 does not exceed the rank of the first unfolding
(with zero padding it is at most that sum); and because the Tucker factors
are orthonormal, ||X - TR(X_1..X_N)||^2 = ||X - [[G; U]]||^2 +
||G - TR(G_1..G_N)||^2.

Sign reading.  With r_0 > 1 the first step files singular vector c under the
index pair (a0, a1); negating one singular vector negates one (a1, a0) block
of the next unfolding, which is not an orthogonal change of that matrix and
alters the truncation.  TR-SVD is therefore fixed here by giving every left
singular vector the sign that makes its largest-magnitude entry positive
(the same rule as the Tucker factors).
"""
import numpy as np

from .rbki import rbki_tucker, canonical_signs
from .tensor import fro


def _truncated_svd_padded(M, r):
    """Leading min(r, rank) singular triplets of M, zero-padded to r, with
    canonical signs (largest-magnitude entry of each left vector positive)."""
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    Uc = canonical_signs(U)
    flip = np.where(np.sum(Uc * U, axis=0) < 0, -1.0, 1.0)
    U, Vt = Uc, Vt * flip[:, None]
    k = min(r, s.size)
    Ul = np.zeros((M.shape[0], r))
    Rl = np.zeros((r, M.shape[1]))
    Ul[:, :k] = U[:, :k]
    Rl[:k] = s[:k, None] * Vt[:k]
    discarded = float(np.sum(s[k:] ** 2))
    return Ul, Rl, discarded


def tr_svd(G, tr_ranks):
    """TR-SVD of G (S_1 x ... x S_N) with TR ranks (r_1, ..., r_N), r_0 = r_N.
    Returns the cores [(r_{k-1}, S_k, r_k)] and the sum of the squared
    discarded singular values."""
    G = np.asarray(G, np.float64)
    N = G.ndim
    S = G.shape
    r = [int(tr_ranks[-1])] + [int(v) for v in tr_ranks]     # r[0] = r_N
    discarded = 0.0
    Ul, C, d = _truncated_svd_padded(G.reshape(S[0], -1), r[0] * r[1])
    discarded += d
    cores = [Ul.reshape(S[0], r[0], r[1]).transpose(1, 0, 2).copy()]
    C = C.reshape((r[0], r[1]) + S[1:])
    C = np.moveaxis(C, 0, -1)                                  # (r1, S2..SN, r0)
    for k in range(1, N - 1):
        M = C.reshape(r[k] * S[k], -1)
        Ul, C, d = _truncated_svd_padded(M, r[k + 1])
        discarded += d
        cores.append(Ul.reshape(r[k], S[k], r[k + 1]))
        C = C.reshape((r[k + 1],) + S[k + 1:] + (r[0],))
    cores.append(C.reshape(r[N - 1], S[N - 1], r[0]).copy())
    return cores, discarded


def tr_to_full(cores):
    """X(i_1..i_N) = trace(X_1(:, i_1, :) X_2(:, i_2, :) ... X_N(:, i_N, :))
    (eq. (3))."""
    T = cores[0]                                     # (r0, S1, r1)
    for Ck in cores[1:]:
        T = np.tensordot(T, Ck, axes=([T.ndim - 1], [0]))
    # T has shape (r0, S1, ..., SN, r0): close the ring
    return np.trace(T, axis1=0, axis2=T.ndim - 1)


def attach_factors(cores, factors):
    """Alg. 3, step 4: X_n = G_n x_2 U^(n)."""
    return [np.einsum("asb,is->aib", Gn, U) for Gn, U in zip(cores, factors)]


def rbki_htr(X, tucker_ranks, p, q, seed, tr_ranks, explicit_error=True):
    """Alg. 3 (rBKI-TK-TR) with the TR-SVD branch.  Returns the TR cores of
    X, the relative error and a dict of intermediate results.

    explicit_error: True   -- ||X - TR(X_1..X_N)|| from the full ring (small
                              tensors only: the ring is contracted whole);
                    "core" -- sqrt(||X - [[G; U]]||^2 + ||G - TR(G_1..G_N)||^2),
                              both terms explicit (the second on the small
                              core), equal to the above because the Tucker
                              factors are orthonormal;
                    False  -- the Tucker error plus the discarded energy of
                              the TR-SVD steps."""
    X = np.asarray(X, np.float64)
    G, factors, e_tk, tk_infos = rbki_tucker(X, tucker_ranks, p, q, seed, return_info=True)
    core_cores, discarded = tr_svd(G, tr_ranks)
    cores = attach_factors(core_cores, factors)
    nx = fro(X)
    gap2 = None
    if explicit_error == "core":
        gap2 = fro(G - tr_to_full(core_cores)) ** 2
        err = float(np.sqrt((e_tk * nx) ** 2 + gap2)) / nx
    elif explicit_error:
        err = fro(X - tr_to_full(cores)) / nx
    else:
        err = float(np.sqrt((e_tk * nx) ** 2 + discarded)) / nx
    info = {"G": G, "factors": factors, "core_cores": core_cores,
            "tucker_error": e_tk, "discarded": discarded, "core_gap2": gap2,
            "tucker_infos": tk_infos}
    return cores, err, info


# ----------------------------------------------------------------------- TR-ALS
#
# Alg. 3, step 3 names TR-ALS (Zhao et al. 2016) as the way to decompose the
# compressed core, TR-SVD as the alternative.  TR-ALS, written here from that
# method's published description: with the cores Z_1..Z_N of a tensor ring,
# the tensor's entries are T(i_1..i_N) = Tr(Z_k(i_k) Z_{k+1}(i_{k+1}) ...
# Z_{k-1}(i_{k-1})) for every k (the trace is cyclic), so with the other cores
# fixed the entries are linear in Z_k:
#   T_<k>[i_k, p] = sum_{a, b} Z_k[a, i_k, b] M[b, p, a],
# where M (r_k x P x r_{k-1}) is the product Z_{k+1} ... Z_N Z_1 ... Z_{k-1}
# of the other cores and p runs over (i_{k+1}, ..., i_N, i_1, ..., i_{k-1}) in
# that order.  One ALS update of core k is the least-squares fit of G's
# unfolding G_<k> in that column order by this linear model; a sweep updates
# k = 1, ..., N in turn.
#
# Readings: the cores start from Gaussian values of the sketch stream
# (philox, tag 2: core k's entry at linear index (a S_k + i) r_k + b of
# stream (seed, k)), scaled by 1/sqrt(S_k r_{k-1} r_k).  (A TR-SVD start is
# zero-padded whenever r_{k-1} r_k exceeds the rank of a core's unfolding,
# which makes the least-squares updates rank-deficient and their solution a
# matter of thresholds; a random start gives full-rank updates.)  The
# iteration follows the rule of Sec. 4 for all methods: at most 20 sweeps,
# stopping when the Fit 1 - ||G - TR||/||G|| (a fraction) changes by at most
# 1e-3 between sweeps (the start counts as sweep 0); each least-squares
# problem takes its minimum-norm solution.


def subchain(cores, k):
    """M = Z_{k+1} ... Z_N Z_1 ... Z_{k-1} as an (r_k, P, r_{k-1}) array, p
    running over the other modes in cyclic order from k+1."""
    N = len(cores)
    order = [(k + j) % N for j in range(1, N)]
    M = cores[order[0]]
    for j in order[1:]:
        M = np.tensordot(M, cores[j], axes=([M.ndim - 1], [0]))
    rk, rk1 = cores[k].shape[2], cores[k].shape[0]
    return M.reshape(rk, -1, rk1)


def cyclic_unfolding(G, k):
    """G_<k>: mode k as rows, the other modes as columns in the cyclic order
    k+1, ..., N, 1, ..., k-1."""
    N = G.ndim
    order = [k] + [(k + j) % N for j in range(1, N)]
    return np.transpose(G, order).reshape(G.shape[k], -1)


def als_design(cores, k):
    """The design matrix D (P x r_{k-1} r_k) of the update of core k:
    D[p, a r_k + b] = M[b, p, a]."""
    M = subchain(cores, k)
    return np.ascontiguousarray(M.transpose(1, 2, 0).reshape(M.shape[1], -1))


def als_update(G, cores, k):
    """The least-squares core k (minimum-norm solution) given the others."""
    D = als_design(cores, k)
    Gk = cyclic_unfolding(G, k)
    rk1, Sk, rk = cores[k].shape
    Zt, *_ = np.linalg.lstsq(D, Gk.T, rcond=None)      # (r_{k-1} r_k) x S_k
    return Zt.reshape(rk1, rk, Sk).transpose(0, 2, 1).copy()


TAG_TR_START = 2


def tr_als_start(shape, tr_ranks, seed):
    """The TR-ALS start: core k (r_{k-1} x S_k x r_k) holds the Gaussian values
    of stream (seed, k, tag 2) at linear indices 0 .. r_{k-1} S_k r_k - 1,
    divided by sqrt(S_k r_{k-1} r_k)."""
    from . import philox
    r = [int(tr_ranks[-1])] + [int(v) for v in tr_ranks]
    cores = []
    for k, S in enumerate(shape):
        n = r[k] * S * r[k + 1]
        z = philox.gaussian_at(seed, k, np.arange(n, dtype=np.uint64), tag=TAG_TR_START)
        cores.append(z.reshape(r[k], S, r[k + 1]) / np.sqrt(S * r[k] * r[k + 1]))
    return cores


def tr_als(G, tr_ranks, max_sweeps=20, fit_tol=1e-3, history=False, seed=0, start=None):
    """TR-ALS of G with TR ranks (r_1..r_N), r_0 = r_N, from tr_als_start
    (or the given cores).  Returns the cores, the number of sweeps taken and
    (history=True) the relative error after every single-core update."""
    G = np.asarray(G, np.float64)
    cores = [np.array(c, np.float64) for c in start] if start is not None else tr_als_start(G.shape, tr_ranks, seed)
    ng = fro(G)
    errs = [fro(G - tr_to_full(cores)) / ng]
    prev = 1.0 - errs[0]
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        for k in range(G.ndim):
            cores[k] = als_update(G, cores, k)
            if history:
                errs.append(fro(G - tr_to_full(cores)) / ng)
        fit = 1.0 - fro(G - tr_to_full(cores)) / ng
        if abs(fit - prev) <= fit_tol:
            break
        prev = fit
    if history:
        return cores, sweeps, errs
    return cores, sweeps


def rbki_htr_als(X, tucker_ranks, p, q, seed, tr_ranks, max_sweeps=20, fit_tol=1e-3):
    """Alg. 3 with the TR-ALS branch: rBKI-TK, TR-ALS of the core (its start
    from the same seed), X_n = G_n x_2 U^(n).  The error is sqrt(||X - [[G; U]]||^2 + ||G - TR(G_n)||^2)
    / ||X|| (orthonormal Tucker factors; both terms explicit)."""
    X = np.asarray(X, np.float64)
    G, factors, e_tk = rbki_tucker(X, tucker_ranks, p, q, seed)
    core_cores, sweeps = tr_als(G, tr_ranks, max_sweeps, fit_tol, seed=seed)
    cores = attach_factors(core_cores, factors)
    nx = fro(X)
    gap2 = fro(G - tr_to_full(core_cores)) ** 2
    err = float(np.sqrt((e_tk * nx) ** 2 + gap2)) / nx
    return cores, err, {"G": G, "factors": factors, "core_cores": core_cores, "sweeps": sweeps,
                        "tucker_error": e_tk, "core_gap2": gap2}
