"""Mode-n matricization, folding and mode-n products (Table 1; eq. (1)-(2)).

Layout convention.  Tensors are row-major NumPy arrays (last index fastest).
For mode n the tensor is viewed as [A_n, I_n, B_n] with A_n = prod_{k<n} I_k
and B_n = prod_{k>n} I_k, and the mode-n unfolding X_(n) in R^{I_n x J_n},
J_n = A_n * B_n, has column index j = a * B_n + b:

    X_(n)[i, a * B_n + b] = X[a, i, b].

The paper does not fix a column order; any fixed order gives the same
X_(n) X_(n)^T and the same left subspace.  The order matters only for which
row of the sketch matrix Omega meets which column, so it is stated here and
followed by the GPU as well.
"""
import numpy as np


def view_dims(shape, n):
    """(A_n, I_n, B_n) of the unfolding-free view of mode n."""
    A = int(np.prod(shape[:n], dtype=np.int64))
    B = int(np.prod(shape[n + 1:], dtype=np.int64))
    return A, int(shape[n]), B


def unfold(X, n):
    """X_(n) in R^{I_n x J_n} with column j = a * B_n + b (a copy)."""
    A, I, B = view_dims(X.shape, n)
    return np.ascontiguousarray(X.reshape(A, I, B).transpose(1, 0, 2).reshape(I, A * B))


def fold(M, n, shape):
    """Inverse of unfold: M in R^{I_n x J_n} back to a tensor of `shape`."""
    A, I, B = view_dims(shape, n)
    return np.ascontiguousarray(M.reshape(I, A, B).transpose(1, 0, 2).reshape(shape))


def mode_product(X, M, n):
    """The mode-n product X x_n M for M in R^{K x I_n} (Table 1): the result
    has mode n of size K and (X x_n M)_(n) = M X_(n)."""
    shape = list(X.shape)
    out_shape = shape[:n] + [M.shape[0]] + shape[n + 1:]
    return fold(M @ unfold(X, n), n, out_shape)


def tucker_to_full(G, factors):
    """[[G; U1, ..., UN]] = G x_1 U1 x_2 U2 ... x_N UN (eq. (1))."""
    X = G
    for n, U in enumerate(factors):
        X = mode_product(X, U, n)
    return X


def project_core(X, factors):
    """G = X x_1 U1^T x_2 U2^T ... x_N UN^T, ascending n (Alg. 2, step 6)."""
    G = X
    for n, U in enumerate(factors):
        G = mode_product(G, U.T, n)
    return G


def fro(X):
    return float(np.sqrt(np.sum(np.square(X, dtype=np.float64))))
