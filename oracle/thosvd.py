"""Truncated HOSVD (T-SVD), the deterministic benchmark of Sec. 4.

U^(n) holds the leading R_n left singular vectors of X_(n) (the optimal
rank-R_n subspace of each unfolding, by the Eckart-Young lemma of Sec. 2.2);
the core is G = X x_1 U^(1)T ... x_N U^(N)T.  RErr in Sec. 4 divides by the
error of this approximation.
"""
import numpy as np

from .tensor import unfold, project_core, tucker_to_full, fro


def leading_left_singular(Xn, R):
    """Leading R left singular vectors of Xn and all its singular values,
    from LAPACK's SVD (wide matrices go through the Gram matrix Xn Xn^T,
    whose eigenvectors are the same vectors)."""
    I, J = Xn.shape
    if J <= 4 * I or I * J <= 4_000_000:
        U, s, _ = np.linalg.svd(Xn, full_matrices=False)
        return U[:, :R], s
    lam, V = np.linalg.eigh(Xn @ Xn.T)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    return V[:, :R], np.sqrt(np.maximum(lam, 0.0))


def thosvd(X, ranks):
    """Truncated HOSVD: returns G, [U^(n)], relative error vs X."""
    X = np.asarray(X, dtype=np.float64)
    factors = [leading_left_singular(unfold(X, n), ranks[n])[0] for n in range(X.ndim)]
    G = project_core(X, factors)
    err = fro(X - tucker_to_full(G, factors)) / fro(X)
    return G, factors, err
