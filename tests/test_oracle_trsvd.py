"""Pins for the oracle's TR-SVD and Alg. 3: exact recovery of a TT tensor
(the r_0 = 1 special case of a ring), the orthogonality identity of the
truncation error, and the Tucker + ring error split."""
import itertools

import pytest

import numpy as np

import synth
from oracle.trsvd import tr_svd, tr_to_full, attach_factors, rbki_htr
from oracle.rbki import rbki_tucker
from oracle.tensor import fro, tucker_to_full


def test_ring_elementwise_definition():
    rng = np.random.default_rng(1)
    cores = [rng.standard_normal((2, 3, 3)), rng.standard_normal((3, 2, 4)), rng.standard_normal((4, 4, 2))]
    X = tr_to_full(cores)
    for i, j, k in itertools.product(range(3), range(2), range(4)):
        v = np.trace(cores[0][:, i, :] @ cores[1][:, j, :] @ cores[2][:, k, :])
        assert abs(X[i, j, k] - v) < 1e-12


def test_exact_tt_tensor_is_recovered():
    rng = np.random.default_rng(2)
    ranks = (2, 3, 2, 1)       # r_4 = r_0 = 1: a tensor train
    dims = (5, 6, 4, 7)
    r = [1, 2, 3, 2, 1]
    cores = [rng.standard_normal((r[k], dims[k], r[k + 1])) for k in range(4)]
    X = tr_to_full(cores)
    out, discarded = tr_svd(X, ranks)
    assert fro(X - tr_to_full(out)) <= 1e-12 * fro(X)
    assert discarded <= 1e-24 * fro(X) ** 2
    assert [c.shape for c in out] == [(1, 5, 2), (2, 6, 3), (3, 4, 2), (2, 7, 1)]


def test_truncation_error_equals_discarded_energy():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((6, 5, 7, 4))
    for ranks in [(2, 2, 2, 2), (3, 2, 4, 1), (1, 3, 3, 3)]:
        cores, discarded = tr_svd(G, ranks)
        assert abs(fro(G - tr_to_full(cores)) ** 2 - discarded) <= 1e-10 * fro(G) ** 2
        shapes = [c.shape for c in cores]
        r = [ranks[-1]] + list(ranks)
        assert shapes == [(r[k], G.shape[k], r[k + 1]) for k in range(4)]


def test_zero_padding_when_ring_ranks_exceed_the_unfolding():
    # r_0 r_1 = 64 > S_1 = 6: only 6 triplets exist; ranks stay literally 8
    rng = np.random.default_rng(4)
    G = rng.standard_normal((6, 6, 6))
    cores, discarded = tr_svd(G, (8, 8, 8))
    assert [c.shape for c in cores] == [(8, 6, 8)] * 3
    assert fro(G - tr_to_full(cores)) <= 1e-12 * fro(G)


def test_htr_error_split_and_contraction():
    X, _ = synth.tensor_ring_data((14, 12, 13, 11), 3, seed=5, var=1.0 / 3)
    X = synth.add_noise(X, 15.0, np.random.default_rng(6))
    cores, err, info = rbki_htr(X, (6, 6, 6, 6), p=3, q=2, seed=7, tr_ranks=(3, 3, 3, 3))
    nx = fro(X)
    e_tk = info["tucker_error"]
    # ||X - TR||^2 = ||X - [[G;U]]||^2 + ||G - TR(G_n)||^2  (orthonormal U)
    gap = fro(info["G"] - tr_to_full(info["core_cores"])) ** 2
    assert abs((err * nx) ** 2 - ((e_tk * nx) ** 2 + gap)) <= 1e-10 * nx ** 2
    assert abs(gap - info["discarded"]) <= 1e-10 * nx ** 2
    _, err2, _ = rbki_htr(X, (6, 6, 6, 6), p=3, q=2, seed=7, tr_ranks=(3, 3, 3, 3), explicit_error=False)
    assert abs(err2 - err) <= 1e-10
    # X_n = G_n x_2 U^(n): the TR of the contracted cores equals [[TR(G_n); U]]
    lifted = tucker_to_full(tr_to_full(info["core_cores"]), info["factors"])
    assert fro(lifted - tr_to_full(cores)) <= 1e-12 * nx
    for c, U in zip(cores, info["factors"]):
        assert c.shape[1] == U.shape[0]


def test_canonical_signs_fix_singular_vector_signs():
    from oracle.rbki import canonical_signs
    rng = np.random.default_rng(9)
    U = np.linalg.qr(rng.standard_normal((7, 4)))[0]
    D = np.diag([1.0, -1.0, -1.0, 1.0])
    assert np.array_equal(canonical_signs(U @ D), canonical_signs(U))
    C = canonical_signs(U)
    assert np.all(C[np.argmax(np.abs(C), axis=0), np.arange(4)] > 0)


def test_ring_sweep_depends_on_first_step_signs_and_the_rule_fixes_them():
    """With r_0 > 1 negating one first-step singular vector changes the TR-SVD
    truncation (the (a0, a1) split mixes rows and columns of the next
    unfolding), so the sign rule is needed for TR-SVD to be a function of G;
    with it, negating the input gives the negated ring and the same error."""
    rng = np.random.default_rng(10)
    G = rng.standard_normal((6, 5, 7, 4))
    ranks = (2, 3, 2, 3)
    cores, d = tr_svd(G, ranks)
    e0 = fro(G - tr_to_full(cores))
    cores_neg, _ = tr_svd(-G, ranks)
    assert abs(fro(-G - tr_to_full(cores_neg)) - e0) <= 1e-10 * fro(G)
    # flip one first-step left vector by hand and redo the sweep without the rule
    S = G.shape
    r = [ranks[-1]] + list(ranks)
    U, s, Vt = np.linalg.svd(G.reshape(S[0], -1), full_matrices=False)
    errs = []
    for flip in (1.0, -1.0):
        Uf, Vf = U.copy(), Vt.copy()
        Uf[:, 1] *= flip
        Vf[1] *= flip
        k = r[0] * r[1]
        C = (s[:k, None] * Vf[:k]).reshape((r[0], r[1]) + S[1:])
        C = np.moveaxis(C, 0, -1)
        c1 = Uf[:, :k].reshape(S[0], r[0], r[1]).transpose(1, 0, 2)
        out = [c1]
        for kk in range(1, 3):
            M = C.reshape(r[kk] * S[kk], -1)
            U2, s2, V2 = np.linalg.svd(M, full_matrices=False)
            out.append(U2[:, :r[kk + 1]].reshape(r[kk], S[kk], r[kk + 1]))
            C = (s2[:r[kk + 1], None] * V2[:r[kk + 1]]).reshape((r[kk + 1],) + S[kk + 1:] + (r[0],))
        out.append(C.reshape(r[3], S[3], r[0]))
        errs.append(fro(G - tr_to_full(out)))
    assert abs(errs[0] - errs[1]) > 1e-6 * fro(G)


@pytest.mark.parametrize("dims,tk,tr", [((14, 12, 13, 11), (6, 5, 6, 5), (3, 3, 3, 3)),
                                        ((10, 9, 11), (6, 6, 6), (4, 3, 5))])
def test_core_level_error_equals_the_full_ring_error(dims, tk, tr):
    # ||X - TR(X_n)||^2 = ||X - [[G; U]]||^2 + ||G - TR(G_n)||^2 for orthonormal
    # Tucker factors: the large-tensor form of the HTR error, checked against
    # the full ring contracted elementwise (with zero-padded ranks in the
    # second case: r_0 r_1 = 20 > 6)
    X, _ = synth.tensor_ring_data(dims, 3, seed=7, var=1.0 / 3)
    X = synth.add_noise(X, 15.0, np.random.default_rng(8))
    _, e_full, _ = rbki_htr(X, tk, 3, 2, 9, tr, explicit_error=True)
    _, e_core, info = rbki_htr(X, tk, 3, 2, 9, tr, explicit_error="core")
    assert abs(e_full - e_core) <= 1e-12 * e_full
    assert info["core_gap2"] >= 0.0


# ------------------------------------------------------------------ TR-ALS

from oracle.trsvd import tr_als, als_design, als_update, cyclic_unfolding, rbki_htr_als  # noqa: E402


def _ring(dims, r, snr, seed):
    X, _ = synth.tensor_ring_data(dims, r, seed=seed, var=1.0 / r)
    return synth.add_noise(X, snr, np.random.default_rng(seed + 1))


def test_als_design_matrix_is_the_ring_with_an_indicator_core():
    # column (a, b) of the design matrix of core k is the ring whose k-th core
    # is the indicator of (a, b), read along any row of its cyclic unfolding
    X = _ring((5, 4, 6, 3), 2, 10.0, 40)
    cores, _ = tr_svd(X, (2, 3, 2, 2))
    for k in range(4):
        D = als_design(cores, k)
        ra, S, rb = cores[k].shape
        for a in range(ra):
            for b in range(rb):
                E = [c.copy() for c in cores]
                E[k] = np.zeros((ra, S, rb))
                E[k][a, :, b] = 1.0
                col = cyclic_unfolding(tr_to_full(E), k)
                assert np.allclose(col, col[0][None, :], atol=1e-14)
                assert np.allclose(col[0], D[:, a * rb + b], atol=1e-12)


def test_als_update_solves_its_least_squares_problem():
    # normal equations hold after the update, and no perturbation of the
    # updated core lowers the error
    X = _ring((6, 5, 7, 4), 3, 5.0, 41)
    cores, _ = tr_svd(X, (3, 2, 3, 2))
    k = 2
    cores[k] = als_update(X, cores, k)
    D = als_design(cores, k)
    Gk = cyclic_unfolding(X, k)
    ra, S, rb = cores[k].shape
    Zm = cores[k].transpose(1, 0, 2).reshape(S, ra * rb)
    grad = D.T @ (D @ Zm.T - Gk.T)
    assert np.abs(grad).max() <= 1e-10 * np.linalg.norm(D) ** 2 * np.linalg.norm(Gk)
    e0 = fro(X - tr_to_full(cores))
    rng = np.random.default_rng(0)
    for _ in range(5):
        P = [c.copy() for c in cores]
        P[k] = P[k] + 1e-4 * rng.standard_normal(P[k].shape)
        assert fro(X - tr_to_full(P)) >= e0 * (1 - 1e-12)


def test_als_error_never_increases_from_its_start():
    X = _ring((10, 9, 11, 8), 3, 10.0, 42)
    from oracle.trsvd import tr_als_start
    start = tr_als_start(X.shape, (2, 2, 2, 2), 5)
    cores, sweeps, errs = tr_als(X, (2, 2, 2, 2), fit_tol=1e-6, history=True, seed=5)
    assert errs[0] == fro(X - tr_to_full(start)) / fro(X)
    assert np.all(np.diff(errs) <= 1e-12 * errs[1])
    # and from the TR-SVD cores it improves on them
    cores0, _ = tr_svd(X, (2, 2, 2, 2))
    e_svd = fro(X - tr_to_full(cores0)) / fro(X)
    _, _, errs2 = tr_als(X, (2, 2, 2, 2), fit_tol=1e-6, history=True, start=cores0)
    assert errs2[0] == e_svd and errs2[-1] < e_svd and np.all(np.diff(errs2) <= 1e-12 * e_svd)


def test_als_start_is_the_tagged_gaussian_stream():
    from oracle import philox
    from oracle.trsvd import tr_als_start
    cores = tr_als_start((5, 4, 6), (2, 3, 4), 77)
    assert [c.shape for c in cores] == [(4, 5, 2), (2, 4, 3), (3, 6, 4)]
    for k, c in enumerate(cores):
        z = philox.gaussian_at(77, k, np.arange(c.size, dtype=np.uint64), tag=2)
        assert np.array_equal(c.ravel(), z / np.sqrt(c.shape[1] * c.shape[0] * c.shape[2]))
    # a stream of its own: not the sketch's (tag 0)
    assert not np.allclose(cores[0].ravel() * np.sqrt(40), philox.gaussian_at(77, 0, np.arange(40, dtype=np.uint64)))


def test_als_stops_by_the_fit_rule():
    X = _ring((8, 7, 9, 6), 3, 10.0, 43)
    cores, sweeps, errs = tr_als(X, (2, 3, 2, 2), fit_tol=1e-4, history=True)
    N = 4
    fits = [1 - errs[0]] + [1 - errs[s * N] for s in range(1, sweeps + 1)]
    assert abs(fits[sweeps] - fits[sweeps - 1]) <= 1e-4
    assert all(abs(fits[s] - fits[s - 1]) > 1e-4 for s in range(1, sweeps))
    assert tr_als(X, (2, 3, 2, 2), max_sweeps=3, fit_tol=-1.0)[1] == 3


def test_als_keeps_an_exact_train():
    # r_0 = 1 (a tensor train): TR-SVD recovers it, and ALS started there
    # stays exact (its error cannot increase from zero)
    rng = np.random.default_rng(44)
    cores = [rng.standard_normal((1, 5, 3)), rng.standard_normal((3, 6, 2)), rng.standard_normal((2, 4, 1))]
    X = tr_to_full(cores)
    start, _ = tr_svd(X, (3, 2, 1))
    out, sweeps = tr_als(X, (3, 2, 1), start=start)
    assert fro(X - tr_to_full(out)) <= 1e-12 * fro(X)


def test_htr_als_error_splits():
    X = _ring((14, 12, 13, 11), 3, 15.0, 45)
    cores, err, info = rbki_htr_als(X, (6, 5, 6, 5), 3, 2, 9, (3, 3, 3, 3))
    assert abs(err - fro(X - tr_to_full(cores)) / fro(X)) <= 1e-12 * err
