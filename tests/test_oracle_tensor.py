"""Pins for unfolding and mode products (Table 1, eq. (1)) by brute force on
tiny tensors."""
import itertools

import numpy as np

from oracle.tensor import unfold, fold, mode_product, tucker_to_full, project_core, view_dims


def test_unfold_column_convention_and_fold_inverse():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4, 5, 2))
    for n in range(4):
        A, I, B = view_dims(X.shape, n)
        Xn = unfold(X, n)
        assert Xn.shape == (I, A * B)
        for idx in itertools.product(*[range(s) for s in X.shape]):
            a = int(np.ravel_multi_index(idx[:n], X.shape[:n])) if n else 0
            b = int(np.ravel_multi_index(idx[n + 1:], X.shape[n + 1:])) if n < 3 else 0
            assert Xn[idx[n], a * B + b] == X[idx]
        assert np.array_equal(fold(Xn, n, X.shape), X)


def test_mode_product_brute_force():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, 4, 5))
    M = rng.standard_normal((6, 4))
    Y = mode_product(X, M, 1)
    ref = np.zeros((3, 6, 5))
    for i, k, j, l in itertools.product(range(3), range(6), range(4), range(5)):
        ref[i, k, l] += M[k, j] * X[i, j, l]
    assert np.allclose(Y, ref, rtol=1e-14, atol=1e-14)


def test_tucker_elementwise_definition():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((2, 3, 2))
    Us = [rng.standard_normal((4, 2)), rng.standard_normal((3, 3)), rng.standard_normal((5, 2))]
    X = tucker_to_full(G, Us)
    for i, j, k in itertools.product(range(4), range(3), range(5)):
        v = sum(G[a, b, c] * Us[0][i, a] * Us[1][j, b] * Us[2][k, c]
                for a, b, c in itertools.product(range(2), range(3), range(2)))
        assert abs(X[i, j, k] - v) < 1e-12


def test_project_core_inverts_orthonormal_tucker():
    rng = np.random.default_rng(4)
    G = rng.standard_normal((2, 3, 4))
    Us = [np.linalg.qr(rng.standard_normal((I, R)))[0] for I, R in [(5, 2), (6, 3), (7, 4)]]
    assert np.allclose(project_core(tucker_to_full(G, Us), Us), G, atol=1e-13)
