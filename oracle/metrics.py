"""Accuracy metrics of Sec. 4 and subspace comparisons.

Fit(%)  = (1 - ||X - Xhat||_F / ||X||_F) * 100, with X the original (clean)
          tensor when it is known (Sec. 4, first bullet of the metrics list).
RErr    = ||X - Xhat||_F / ||X - X_k||_F, X_k the truncated-HOSVD
          approximation (Sec. 4, second bullet).
"""
import numpy as np

from .tensor import fro


def fit_percent(X_ref, X_hat):
    return (1.0 - fro(np.asarray(X_ref, np.float64) - X_hat) / fro(X_ref)) * 100.0


def rerr(X_ref, X_hat, X_opt):
    X_ref = np.asarray(X_ref, np.float64)
    return fro(X_ref - X_hat) / fro(X_ref - X_opt)


def projector_distance(U1, U2):
    """||U1 U1^T - U2 U2^T||_2 for matrices with orthonormal columns: the sine
    of the largest principal angle between the two column spaces.  Insensitive
    to signs and to rotations inside the space."""
    U1 = np.asarray(U1, np.float64)
    U2 = np.asarray(U2, np.float64)
    P = U1 @ U1.T - U2 @ U2.T
    return float(np.linalg.norm(P, 2))


def orthonormality_defect(U):
    """||U^T U - I||_2."""
    U = np.asarray(U, np.float64)
    return float(np.linalg.norm(U.T @ U - np.eye(U.shape[1]), 2))
