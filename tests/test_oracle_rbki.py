"""Pins for the oracle's Alg. 1 / Alg. 2 against what mathematics fixes:
exact recovery, reduction to a truncated SVD, Eckart-Young, Rayleigh-Ritz
nesting, the HOSVD error bound, the EVD/SVD equivalence of Remark 1 and the
orthogonality identities of the core."""
import numpy as np
import pytest

import synth
from oracle import philox
from oracle.rbki import (rbki_basis, literal_krylov_basis, power_basis, ritz_factor,
                         mode_factor, rbki_tucker, per_mode_error, sketch_size, orth)
from oracle.thosvd import thosvd, leading_left_singular
from oracle.tensor import unfold, project_core, tucker_to_full, fro, view_dims
from oracle.metrics import projector_distance, orthonormality_defect


def noisy_tucker(dims, ranks, snr, seed):
    Xc, rng = synth.orthonormal_tucker(dims, ranks, seed)
    return synth.add_noise(Xc, snr, rng), Xc


def test_sketch_size_rule():
    assert sketch_size(10, 5, 200, 40000) == 15
    assert sketch_size(10, 5, 12, 40000) == 12
    assert sketch_size(10, 5, 200, 8) == 8


def test_exact_rank_tucker_is_recovered():
    Xc, _ = synth.orthonormal_tucker((20, 24, 18), (3, 4, 2), seed=5)
    G, Us, err = rbki_tucker(Xc, (3, 4, 2), p=5, q=2, seed=11)
    assert err <= 1e-12
    for U in Us:
        assert orthonormality_defect(U) < 1e-13


def test_exact_rank_with_rank_deficient_krylov_blocks():
    # S > true rank: W has rank 3 < S = 8, later blocks deflate completely
    Xc, _ = synth.orthonormal_tucker((16, 16, 16), (3, 3, 3), seed=6)
    G, Us, err, infos = rbki_tucker(Xc, (3, 3, 3), p=5, q=2, seed=12, return_info=True)
    assert err <= 1e-12
    for info in infos:
        assert info["widths"][0] == 3 and sum(info["widths"][1:]) == 0


def test_full_krylov_reduces_to_truncated_svd():
    # S (q+1) >= I: the basis spans R^I and U is the LAPACK truncated SVD
    X, _ = noisy_tucker((12, 30, 25), (4, 4, 4), 10.0, seed=7)
    for n in range(3):
        U, info = mode_factor(X, n, 4, p=3, q=2, seed=13, return_info=True)
        I = X.shape[n]
        assert info["Q"].shape[1] == min(I, 7 * 3)
        Xn = unfold(X, n)
        Ut, s = leading_left_singular(Xn, 4)
        if I <= 21:
            assert (s[3] - s[4]) / s[0] > 1e-6
            assert projector_distance(U, Ut) <= 1e-10


def test_strong_gap_converges_to_svd():
    # sigma_{R+1}/sigma_R <= 1e-3 with q >= 2: (1e-3)^(2q+1) is far below 1e-10
    rng = np.random.default_rng(8)
    I, J, R = 60, 500, 5
    Uq = np.linalg.qr(rng.standard_normal((I, I)))[0]
    Vq = np.linalg.qr(rng.standard_normal((J, I)))[0]
    s = np.concatenate([np.linspace(10, 5, R), 5e-3 * np.linspace(1, 0.5, I - R)])
    Xn = (Uq * s) @ Vq.T
    Om = philox.omega(3, 0, J, R + 2)
    Q, _ = rbki_basis(Xn, Om, q=2)
    U, _ = ritz_factor(Xn, Q, R)
    assert projector_distance(U, Uq[:, :R]) <= 1e-10


def test_eckart_young_per_mode_and_orthonormal():
    X, _ = noisy_tucker((30, 26, 34), (5, 5, 5), 0.0, seed=9)
    for n in range(3):
        U = mode_factor(X, n, 5, p=2, q=1, seed=14)
        assert orthonormality_defect(U) < 1e-13
        Ut, _ = leading_left_singular(unfold(X, n), 5)
        assert per_mode_error(X, n, U) >= per_mode_error(X, n, Ut) * (1 - 1e-12)


def test_rayleigh_ritz_nesting_in_q_and_p_and_vs_power_iteration():
    X, _ = noisy_tucker((40, 36, 30), (6, 6, 6), -5.0, seed=10)
    n, R = 0, 6
    Xn = unfold(X, n)
    J = Xn.shape[1]
    errs_q = []
    for q in range(4):
        Q, _ = rbki_basis(Xn, philox.omega(21, n, J, R + 2), q)
        U, _ = ritz_factor(Xn, Q, R)
        errs_q.append(fro(Xn - U @ (U.T @ Xn)))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs_q, errs_q[1:]))
    errs_p = []
    for p in range(0, 6):
        Q, _ = rbki_basis(Xn, philox.omega(21, n, J, R + p), 1)
        U, _ = ritz_factor(Xn, Q, R)
        errs_p.append(fro(Xn - U @ (U.T @ Xn)))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs_p, errs_p[1:]))
    # the power-iteration space (XX^T)^q W lies inside the Krylov space
    for q in (1, 2, 3):
        Om = philox.omega(21, n, J, R + 2)
        Qk, _ = rbki_basis(Xn, Om, q)
        Qp = power_basis(Xn, Om, q)
        Uk, _ = ritz_factor(Xn, Qk, R)
        Up, _ = ritz_factor(Xn, Qp, R)
        assert fro(Xn - Uk @ (Uk.T @ Xn)) <= fro(Xn - Up @ (Up.T @ Xn)) * (1 + 1e-12)


def test_q0_is_single_sketch_range_finder():
    # q = 0: U comes from the range of W = X Omega alone (Sec. 2.2)
    X, _ = noisy_tucker((25, 20, 22), (4, 4, 4), 5.0, seed=15)
    Xn = unfold(X, 1)
    Om = philox.omega(5, 1, Xn.shape[1], 7)
    Q, _ = rbki_basis(Xn, Om, 0)
    Qw, _ = np.linalg.qr(Xn @ Om)
    assert projector_distance(Q, Qw) < 1e-12


def test_hosvd_error_bound():
    # ||X - Xhat||^2 <= sum_n ||X - X x_n U U^T||^2 (eq. (10))
    X, _ = noisy_tucker((28, 30, 26), (5, 4, 6), 0.0, seed=16)
    G, Us, err = rbki_tucker(X, (5, 4, 6), p=5, q=2, seed=17)
    lhs = (err * fro(X)) ** 2
    rhs = sum(per_mode_error(X, n, Us[n]) ** 2 for n in range(3))
    assert lhs <= rhs * (1 + 1e-12)


def test_literal_and_orthonormalised_krylov_span_agree_when_well_conditioned():
    rng = np.random.default_rng(18)
    I, J = 30, 200
    s = np.linspace(1.0, 0.6, I)
    Xn = (np.linalg.qr(rng.standard_normal((I, I)))[0] * s) @ np.linalg.qr(rng.standard_normal((J, I)))[0].T
    Om = philox.omega(4, 0, J, 4)
    Ql, K = literal_krylov_basis(Xn, Om, 2)
    assert np.linalg.cond(K) <= 1e6
    Qo, _ = rbki_basis(Xn, Om, 2)
    assert Qo.shape[1] == Ql.shape[1]
    assert projector_distance(Qo, Ql) <= 1e-9


def test_evd_route_equals_svd_route():
    # Remark 1: eigenvectors of Q^T X X^T Q = left singular vectors of Q^T X
    X, _ = noisy_tucker((26, 24, 28), (5, 5, 5), 5.0, seed=19)
    Xn = unfold(X, 2)
    Q, _ = rbki_basis(Xn, philox.omega(6, 2, Xn.shape[1], 8), 2)
    Ue, _ = ritz_factor(Xn, Q, 5)
    Us, _, _ = np.linalg.svd(Q.T @ Xn, full_matrices=False)
    assert projector_distance(Ue, Q @ Us[:, :5]) <= 1e-10


def test_core_orthogonality_identities():
    X, _ = noisy_tucker((24, 26, 22), (4, 5, 3), 10.0, seed=20)
    G, Us, err = rbki_tucker(X, (4, 5, 3), p=5, q=2, seed=22)
    nx = fro(X)
    # ||X - [[G;U]]||^2 = ||X||^2 - ||G||^2 for orthonormal U and G = X x U^T
    assert abs((err * nx) ** 2 - (nx ** 2 - fro(G) ** 2)) <= 1e-12 * nx ** 2
    # perturbing the core adds exactly its squared norm to the squared error
    dG = np.random.default_rng(0).standard_normal(G.shape) * 1e-3
    e2 = fro(X - tucker_to_full(G + dG, Us)) ** 2
    assert abs(e2 - ((err * nx) ** 2 + fro(dG) ** 2)) <= 1e-10 * nx ** 2


def test_rbki_is_no_better_than_tsvd_on_noise_free_low_rank_plus_tail():
    X, _ = noisy_tucker((30, 30, 30), (5, 5, 5), 15.0, seed=23)
    _, _, e_r = rbki_tucker(X, (5, 5, 5), p=5, q=2, seed=24)
    _, _, e_t = thosvd(X, (5, 5, 5))
    assert e_r >= e_t * (1 - 1e-6)
    assert e_r <= e_t * 1.01


def test_plausible_mistakes_are_caught():
    """Mutations of the method (dropping the Krylov blocks, using X^T X,
    using the wrong eigen-order) each violate one of the pins above."""
    X, _ = noisy_tucker((30, 24, 20), (4, 4, 4), -5.0, seed=25)
    Xn = unfold(X, 0)
    J = Xn.shape[1]
    Om = philox.omega(7, 0, J, 9)
    Q, _ = rbki_basis(Xn, Om, 2)
    U, lam = ritz_factor(Xn, Q, 4)
    Ut, _ = leading_left_singular(Xn, 4)
    good = fro(Xn - U @ (U.T @ Xn))
    # ascending instead of descending eigen-order gives a far worse factor
    Bm = Q.T @ Xn
    w, V = np.linalg.eigh(Bm @ Bm.T)
    Ubad = Q @ V[:, :4]
    assert fro(Xn - Ubad @ (Ubad.T @ Xn)) > 1.1 * good
    # q = 0 (no Krylov blocks) is measurably worse at -5 dB
    Q0, _ = rbki_basis(Xn, Om, 0)
    U0, _ = ritz_factor(Xn, Q0, 4)
    assert fro(Xn - U0 @ (U0.T @ Xn)) > good * (1 + 1e-3)
    assert abs(good - fro(Xn - Ut @ (Ut.T @ Xn))) < 1e-3 * good


def test_power_variant_reduces_to_the_range_finder_at_q0_and_recovers_exact_rank():
    # q = 0: power iteration and the Krylov space are both range(X Omega)
    X, _ = noisy_tucker((22, 18, 20), (4, 3, 5), 5.0, seed=31)
    Gk, Uk, ek = rbki_tucker(X, (4, 3, 5), p=4, q=0, seed=8)
    Gp, Up, ep = rbki_tucker(X, (4, 3, 5), p=4, q=0, seed=8, variant="power")
    assert ep == ek and np.array_equal(Gp, Gk) and all(np.array_equal(a, b) for a, b in zip(Up, Uk))
    # an exactly low-rank Tucker tensor is recovered by the power variant too
    Xc, _ = synth.orthonormal_tucker((20, 24, 18), (3, 4, 2), seed=5)
    _, _, err = rbki_tucker(Xc, (3, 4, 2), p=5, q=2, seed=11, variant="power")
    assert err <= 1e-12


def test_power_basis_spans_the_power_iterate():
    # the basis is an orthonormal basis of (X X^T)^q X Omega (Sec. 3.1), here
    # where that block is well conditioned (q = 1, a few columns)
    X, _ = noisy_tucker((30, 26, 24), (5, 5, 5), 20.0, seed=41)
    Xn = unfold(X, 1)
    Om = philox.omega(3, 1, Xn.shape[1], 6)
    Q = power_basis(Xn, Om, 1)
    Y = Xn @ (Xn.T @ (Xn @ Om))
    Qy, _ = np.linalg.qr(Y)
    assert orthonormality_defect(Q) <= 1e-12
    assert projector_distance(Q, Qy) <= 1e-8


def test_power_variant_error_is_not_below_the_krylov_error_per_mode():
    # the power iterate lies inside the Krylov space of the same Omega, so
    # its per-mode Rayleigh-Ritz error is never smaller
    X, _ = noisy_tucker((36, 30, 28), (5, 5, 5), -3.0, seed=43)
    for q in (1, 2):
        _, Uk, _ = rbki_tucker(X, (5, 5, 5), p=3, q=q, seed=9)
        _, Up, _ = rbki_tucker(X, (5, 5, 5), p=3, q=q, seed=9, variant="power")
        for n in range(3):
            assert per_mode_error(X, n, Uk[n]) <= per_mode_error(X, n, Up[n]) * (1 + 1e-12)


# ------------------------------------------------------- partial columns (Sec. 3.1)

def test_sampled_columns_are_one_per_stratum():
    for J, rate in ((1000, 0.1), (997, 0.37), (64, 0.5), (10, 0.01), (5, 1.0)):
        cols = philox.sampled_columns(3, 2, J, rate)
        m = philox.sample_count(J, rate)
        assert cols.size == m and m >= 1
        assert np.all(np.diff(cols) > 0) and cols[0] >= 0 and cols[-1] < J
        k = np.arange(m)
        assert np.all(cols >= (k * J) // m) and np.all(cols < ((k + 1) * J) // m)
    assert np.array_equal(philox.sampled_columns(3, 2, 77, 1.0), np.arange(77))


def test_sampled_columns_follow_the_scalar_generator():
    # the vectorised draw against the big-integer Philox, one stratum at a time
    J, rate, seed, mode = 1234, 0.05, 2 ** 40 + 9, 1
    m = philox.sample_count(J, rate)
    cols = philox.sampled_columns(seed, mode, J, rate)
    key = philox.seed_key(seed)
    for k in range(m):
        lo, hi = (k * J) // m, ((k + 1) * J) // m
        w0 = philox.philox4x32_scalar((k & 0xFFFFFFFF, k >> 32, mode, philox.TAG_COLUMNS), key)[0]
        assert cols[k] == lo + (w0 * (hi - lo) >> 32)


def test_sampled_columns_are_uniform():
    # each column is drawn with probability m / J over many seeds
    J, rate, trials = 200, 0.1, 3000
    counts = np.zeros(J)
    for s in range(trials):
        counts[philox.sampled_columns(s, 0, J, rate)] += 1
    p = philox.sample_count(J, rate) / J
    z = (counts - trials * p) / np.sqrt(trials * p * (1 - p))
    assert np.abs(z).max() < 5.0
    assert abs(np.mean(z)) < 0.2


def test_full_sampling_rate_is_the_plain_method():
    X, _ = noisy_tucker((30, 25, 20), (4, 3, 5), 10.0, seed=21)
    a = rbki_tucker(X, (4, 3, 5), 5, 2, 9)
    b = rbki_tucker(X, (4, 3, 5), 5, 2, 9, sample_rate=1.0)
    assert a[2] == b[2]
    for u, v in zip(a[1], b[1]):
        assert np.array_equal(u, v)


def test_partial_columns_recover_an_exact_rank_tensor():
    # the sampled columns of an exactly rank-R unfolding span its column space
    Xc, _ = synth.orthonormal_tucker((40, 36, 30), (4, 3, 5), seed=22)
    G, Us, err = rbki_tucker(Xc, (4, 3, 5), 5, 2, 10, sample_rate=0.2)
    assert err <= 1e-12


def test_partial_columns_factor_is_the_rayleigh_ritz_of_the_whole_unfolding():
    # Z uses the whole unfolding (Alg. 2, step 3): of all R-dimensional
    # subspaces of the sampled Krylov space, the factor leaves the least
    # residual of X_(n); the subspace chosen from the sampled columns alone
    # (Z from Y) and random subspaces of the basis do no better
    X, _ = noisy_tucker((60, 50, 40), (6, 5, 4), 0.0, seed=23)
    n, R = 0, 6
    U, info = mode_factor(X, n, R, 3, 1, 11, return_info=True, sample_rate=0.15)
    Q = info["Q"]
    Xn = unfold(X, n)
    e = per_mode_error(X, n, U)
    Y = Xn[:, info["columns"]]
    Uy, _ = ritz_factor(Y, Q, R)
    assert e <= per_mode_error(X, n, Uy) * (1 + 1e-12)
    assert per_mode_error(X, n, Uy) > e * (1 + 1e-6)
    rng = np.random.default_rng(0)
    for _ in range(5):
        V, _ = np.linalg.qr(Q @ rng.standard_normal((Q.shape[1], R)))
        assert e <= per_mode_error(X, n, V) * (1 + 1e-12)
    # and the basis is the Krylov space of the sampled columns with an
    # m-row sketch
    Om = philox.omega(11, n, Y.shape[1], info["S"])
    Qy, _ = rbki_basis(Y, Om, 1)
    assert projector_distance(Q, Qy) <= 1e-12


# ------------------------------------------------- sequential truncation, adaptive q

from oracle.rbki import rbki_tucker_sequential, rbki_tucker_adaptive  # noqa: E402


def test_sequential_recovers_an_exact_rank_tensor():
    Xc, _ = synth.orthonormal_tucker((20, 24, 18), (3, 4, 2), seed=5)
    G, Us, err = rbki_tucker_sequential(Xc, (3, 4, 2), p=5, q=2, seed=11)
    assert err <= 1e-12
    assert G.shape == (3, 4, 2)


def test_sequential_error_is_the_sum_of_its_stage_residuals():
    # sequential truncation with orthonormal factors: the stage residuals
    # are mutually orthogonal, so ||X - Xhat||^2 = sum_n ||Y_{n-1} - Y_{n-1} x_n U U^T||^2
    X, _ = noisy_tucker((30, 26, 22, 12), (5, 4, 6, 3), 5.0, seed=31)
    G, Us, err, infos, st2 = rbki_tucker_sequential(X, (5, 4, 6, 3), 3, 1, 12, return_info=True)
    nx2 = fro(X) ** 2
    assert abs(err ** 2 * nx2 - sum(st2)) <= 1e-10 * nx2
    # and the core is the last partially projected tensor: X x_n U_n^T
    assert fro(G - project_core(X, Us)) <= 1e-12 * fro(G)


def test_sequential_with_a_full_krylov_space_is_st_hosvd():
    # S (q + 1) >= I_n in every mode: each factor is the leading left singular
    # subspace of the successive partially projected unfolding
    X, _ = noisy_tucker((12, 14, 10), (3, 4, 2), 10.0, seed=32)
    G, Us, err = rbki_tucker_sequential(X, (3, 4, 2), p=3, q=3, seed=13)
    Y = X
    from oracle.tensor import mode_product
    for n, R in enumerate((3, 4, 2)):
        Ut, s = leading_left_singular(unfold(Y, n), R)
        assert (s[R - 1] - s[R]) / s[0] > 1e-6
        assert projector_distance(Us[n], Ut) <= 1e-10
        Y = mode_product(Y, Ut.T, n)


def test_sequential_first_mode_is_the_independent_one_and_the_rest_differ():
    X, _ = noisy_tucker((40, 30, 35), (5, 4, 6), 5.0, seed=33)
    Gi, Ui, ei = rbki_tucker(X, (5, 4, 6), 4, 1, 14)
    Gs, Us, es = rbki_tucker_sequential(X, (5, 4, 6), 4, 1, 14)
    assert np.array_equal(Ui[0], Us[0])
    assert projector_distance(Ui[1], Us[1]) > 1e-8


def test_table4_rerr_is_the_independent_form_not_the_sequential_one():
    # Table 4 prints RErr 1.10 for rBKI-TK on the power-functional 200^3 case;
    # the independent-mode form reproduces it (test_oracle_paper), the
    # sequential form does not (it lands below 1, better than T-HOSVD)
    Xc = synth.power_functional((200, 200, 200))
    X = synth.noisy(Xc, 5.0, seed=600)
    G, U, _ = thosvd(X, (10,) * 3)
    Xt = tucker_to_full(G, U)
    Gs, Us, _ = rbki_tucker_sequential(X, (10,) * 3, 5, 2, 601)
    rerr = np.linalg.norm((Xc - tucker_to_full(Gs, Us)).ravel()) / np.linalg.norm((Xc - Xt).ravel())
    assert rerr < 1.0 and abs(rerr - 1.10) > 0.1


def test_adaptive_q_stops_at_the_first_small_fit_change():
    X, _ = noisy_tucker((40, 36, 30), (5, 4, 3), 0.0, seed=34)
    G, Us, err, qu = rbki_tucker_adaptive(X, (5, 4, 3), 3, 15, fit_tol=1e-4, max_q=10)
    fits = [1.0 - rbki_tucker(X, (5, 4, 3), 3, t, 15)[2] for t in range(qu + 1)]
    assert abs(fits[qu] - fits[qu - 1]) <= 1e-4
    assert all(abs(fits[t] - fits[t - 1]) > 1e-4 for t in range(1, qu))
    assert err == rbki_tucker(X, (5, 4, 3), 3, qu, 15)[2]
    # a tolerance no change can meet runs to max_q; a loose one stops at once
    assert rbki_tucker_adaptive(X, (5, 4, 3), 3, 15, fit_tol=-1.0, max_q=3)[3] == 3
    assert rbki_tucker_adaptive(X, (5, 4, 3), 3, 15, fit_tol=1.0, max_q=3)[3] == 1


def test_adaptive_q_on_the_table3_case_is_small():
    # Sec. 3.1: q = 2 is enough in practice; with the stopping rule of
    # Sec. 4 the Gaussian Tucker case of Table 3 stops within 3 steps
    Xc = synth.gaussian_tucker((200, 200, 200), (10, 10, 10), seed=301)
    X = synth.noisy(Xc, -5.0, seed=401)
    _, _, _, qu = rbki_tucker_adaptive(X, (10, 10, 10), 5, 501)
    assert 1 <= qu <= 3
