"""Alg. 1 (tensor sketching via rBKI) and Alg. 2 (rBKI-TK), float64.

Readings of the paper taken here (each is listed with its reason in the
design notes of the repository):

* Modes are independent (HOSVD-style): every factor U^(n) is computed from the
  original tensor X, and the core is then accumulated G <- G x_n U^(n)T,
  starting from G = X, in ascending n (Alg. 2, steps 1-6; Sec. 3.2 calls the
  method a randomized HOSVD).
* Omega^(n) has J_n = prod_{p != n} I_p rows and S_n columns (Alg. 1,
  step 1; the dimension printed in Sec. 2.3 is a typo).
* S_n = min(R_n + p, I_n, J_n) with oversampling p (Sec. 4.1 uses
  S_n = R_n + 1/gamma with gamma = 0.2, i.e. p = 5).
* q is an explicit input: Alg. 1 gives q only as Theta(log d / sqrt(eps)),
  which has no constant (Sec. 3.1 says q = 2 is enough in practice).
* The Krylov block K = [W, (XX^T)W, ..., (XX^T)^q W] (eq. (15), Alg. 1,
  step 3) is built with orthonormalisation between steps: each new block is
  X_(n)(X_(n)^T Q_{j-1}), projected off the earlier blocks twice and reduced
  to an orthonormal basis by a rank-revealing QR.  The span equals that of
  the literal K in exact arithmetic; the literal K is numerically singular
  for q >= 2 (its columns all align with the top singular vector).  The
  literal form is kept below (literal_krylov_basis) for the test that
  compares the two where K is well conditioned.  The cost of the
  between-step orthonormalisation is the n s^2 q term of Table 2.
* Directions whose QR diagonal falls below TAU times the largest
  pre-projection column norm of the block are dropped (rank deficiency of K:
  exactly low-rank data, or S_n (q+1) >= I_n); the width of the basis is
  capped at I_n.
* Z = Q^T X_(n) X_(n)^T Q (Alg. 2, step 3), eigendecomposed with eigenvalues
  in descending order (svd of a symmetric PSD matrix; Remark 1); the factor
  is U^(n) = Q Utilde(:, 1:R_n) (Alg. 2, steps 4-5).  If the basis has fewer
  than R_n columns, the missing factor columns are zero.
* Singular vectors have no sign in the paper.  Each factor column is given
  the sign that makes its largest-magnitude entry positive (lowest index on
  ties), so the core, and the TR-SVD of Alg. 3 that depends on its slice
  signs, are fixed by the data.
"""
import numpy as np
import scipy.linalg as sla

from . import philox
from .tensor import unfold, view_dims, project_core, tucker_to_full, fro

TAU = 1e-10


def sketch_size(R, p, I, J):
    """S_n = min(R_n + p, I_n, J_n) (Sec. 2.3: R_n <= S_n <= min(I_n, J_n))."""
    return int(min(R + p, I, J))


def orth(Y, ref, tau=TAU):
    """Orthonormal basis of the numerical range of Y: economy QR with column
    pivoting (the rank-revealing form of Alg. 1's "qr(K, 0)"), keeping the
    columns whose |R_kk| exceeds tau * ref."""
    if Y.shape[1] == 0:
        return np.zeros((Y.shape[0], 0))
    Qf, Rf, _ = sla.qr(Y, mode="economic", pivoting=True)
    d = np.abs(np.diag(Rf))
    r = int(np.sum(d > tau * ref))
    return Qf[:, :r]


def project_off(Y, Qprev):
    """Y - Qprev (Qprev^T Y), applied twice (classical Gram-Schmidt, two passes)."""
    if Qprev.shape[1] == 0:
        return Y
    for _ in range(2):
        Y = Y - Qprev @ (Qprev.T @ Y)
    return Y


def max_col_norm(Y):
    return float(np.max(np.linalg.norm(Y, axis=0))) if Y.size else 0.0


def rbki_basis(Xn, Omega, q, tau=TAU):
    """Alg. 1 on the unfolding Xn (I x J) with sketch matrix Omega (J x S):
    returns Q (I x S'), the orthonormal basis of the block Krylov space
    span[W, (Xn Xn^T) W, ..., (Xn Xn^T)^q W], and the per-block widths."""
    I = Xn.shape[0]
    W = Xn @ Omega                                    # Alg. 1, step 2
    Q = orth(W, max_col_norm(W), tau)[:, :I]
    widths = [Q.shape[1]]
    Qlast = Q
    for _ in range(q):                                # Alg. 1, step 3
        if Q.shape[1] >= I or Qlast.shape[1] == 0:
            widths.append(0)
            continue
        Y = Xn @ (Xn.T @ Qlast)                       # (X X^T) times the last block
        ref = max_col_norm(Y)
        Y = project_off(Y, Q)
        Qj = orth(Y, ref, tau)[:, : I - Q.shape[1]]
        widths.append(Qj.shape[1])
        Q = np.hstack([Q, Qj])
        Qlast = Qj
    return Q, widths


def literal_krylov_basis(Xn, Omega, q):
    """Alg. 1 exactly as printed: K = [W, (XX^T)W, ..., (XX^T)^q W] with no
    orthonormalisation between steps, then an economy QR of K."""
    W = Xn @ Omega
    blocks = [W]
    for _ in range(q):
        blocks.append(Xn @ (Xn.T @ blocks[-1]))
    K = np.hstack(blocks)
    Q, _ = np.linalg.qr(K)
    return Q, K


def power_basis(Xn, Omega, q, tau=TAU):
    """Power-iteration subspace K = (XX^T)^q W (Sec. 3.1), normalised at each
    step: only the last block is kept."""
    W = Xn @ Omega
    Q = orth(W, max_col_norm(W), tau)
    for _ in range(q):
        Y = Xn @ (Xn.T @ Q)
        Q = orth(Y, max_col_norm(Y), tau)
    return Q


def canonical_signs(U):
    """Flip each column so that its largest-magnitude entry (lowest index on
    ties) is positive; zero columns are left alone."""
    U = np.array(U, dtype=np.float64, copy=True)
    if U.size == 0:
        return U
    idx = np.argmax(np.abs(U), axis=0)
    sgn = np.sign(U[idx, np.arange(U.shape[1])])
    sgn[sgn == 0] = 1.0
    return U * sgn


def ritz_factor(Xn, Q, R):
    """Alg. 2, steps 3-5: Z = Q^T Xn Xn^T Q, descending eigendecomposition,
    U = Q Utilde(:, 1:R).  Returns U (I x R) and the eigenvalues of Z."""
    I = Xn.shape[0]
    U = np.zeros((I, R))
    if Q.shape[1] == 0:
        return U, np.zeros(0)
    Bm = Q.T @ Xn
    Z = Bm @ Bm.T                                     # Alg. 2, step 3
    lam, V = np.linalg.eigh(Z)
    order = np.argsort(lam)[::-1]                     # descending (step 4)
    lam, V = lam[order], V[:, order]
    k = min(R, Q.shape[1])
    U[:, :k] = Q @ V[:, :k]                           # step 5
    return canonical_signs(U), lam


def mode_factor(X, n, R, p, q, seed, tau=TAU, return_info=False, variant="krylov", sample_rate=1.0):
    """Factor U^(n) of rBKI-TK for mode n (Alg. 2, steps 2-5).  variant
    "power": the basis is the power iterate of Sec. 3.1 instead of the block
    Krylov space of Alg. 1.

    sample_rate < 1 (Sec. 3.1, partial columns): the basis is built from the
    m = sample_rate * J_n sampled columns Y of the unfolding
    (philox.sampled_columns), with a sketch of m rows and S_n <= m; Z, and so
    the factor, are taken with the whole unfolding, as Alg. 2, step 3 writes
    them (the sampling shortens the construction of the Krylov space only)."""
    A, I, B = view_dims(X.shape, n)
    J = A * B
    Xn = unfold(X, n)
    if sample_rate < 1.0:
        cols = philox.sampled_columns(seed, n, J, sample_rate)
        Y = np.ascontiguousarray(Xn[:, cols])
    else:
        cols, Y = None, Xn
    m = Y.shape[1]
    S = sketch_size(R, p, I, m)
    Om = philox.omega(seed, n, m, S)
    if variant == "power":
        Q = power_basis(Y, Om, q, tau)
        widths = [Q.shape[1]]
    else:
        Q, widths = rbki_basis(Y, Om, q, tau)
    U, lam = ritz_factor(Xn, Q, R)
    if return_info:
        return U, {"S": S, "widths": widths, "Q": Q, "eigenvalues": lam, "columns": cols}
    return U


def rbki_tucker(X, ranks, p, q, seed, tau=TAU, return_info=False, variant="krylov", sample_rate=1.0):
    """Alg. 2 (rBKI-TK).  X is converted to float64 first.  Returns the core
    G (R_1 x ... x R_N), the factors [U^(1), ..., U^(N)] and the relative
    reconstruction error ||X - [[G; U]]||_F / ||X||_F from the explicit
    residual."""
    X = np.asarray(X, dtype=np.float64)
    factors, infos = [], []
    for n in range(X.ndim):
        U, info = mode_factor(X, n, ranks[n], p, q, seed, tau, return_info=True, variant=variant,
                              sample_rate=sample_rate)
        factors.append(U)
        infos.append(info)
    G = project_core(X, factors)                      # Alg. 2, step 6
    err = fro(X - tucker_to_full(G, factors)) / fro(X)
    if return_info:
        return G, factors, err, infos
    return G, factors, err


def per_mode_error(X, n, U):
    """||X_(n) - U U^T X_(n)||_F, the per-mode error of Lemma 4 (eq. (8))."""
    Xn = unfold(np.asarray(X, dtype=np.float64), n)
    return fro(Xn - U @ (U.T @ Xn))


def rbki_tucker_sequential(X, ranks, p, q, seed, tau=TAU, return_info=False, variant="krylov", sample_rate=1.0):
    """Alg. 2 with step 6 taken as sequential truncation (the ST-HOSVD form,
    the other reading of "G <- X x_n U^(n)T" inside the loop): Y_0 = X, the
    factor of mode n is computed from Y_{n-1} (whose modes before n are
    already the ranks R_1 .. R_{n-1}), Y_n = Y_{n-1} x_n U^(n)T, and G = Y_N.
    The sketch of mode n has as many rows as Y_{n-1}'s mode-n unfolding has
    columns (the same stream, with J_n replaced by that number)."""
    X = np.asarray(X, dtype=np.float64)
    from .tensor import mode_product
    Y = X
    factors, infos, stage_err2 = [], [], []
    for n in range(X.ndim):
        U, info = mode_factor(Y, n, ranks[n], p, q, seed, tau, return_info=True, variant=variant,
                              sample_rate=sample_rate)
        stage_err2.append(per_mode_error(Y, n, U) ** 2)
        Y = mode_product(Y, U.T, n)
        factors.append(U)
        infos.append(info)
    G = Y
    err = fro(X - tucker_to_full(G, factors)) / fro(X)
    if return_info:
        return G, factors, err, infos, stage_err2
    return G, factors, err


def fit_fraction(rel_err):
    """Fit of Sec. 4 as a fraction: 1 - ||X - Xhat|| / ||X||."""
    return 1.0 - rel_err


def rbki_tucker_adaptive(X, ranks, p, seed, fit_tol=1e-3, max_q=20, tau=TAU, sample_rate=1.0):
    """rBKI-TK with the number of Krylov steps chosen by the stopping rule of
    Sec. 4: t = 0, 1, ... Krylov steps (the same sketch each time, so the
    Krylov spaces are nested) until |Fit_t - Fit_{t-1}| <= fit_tol, or
    t = max_q; Fit_t is the fit of the rank-k approximation after t steps to
    the input X (the only tensor the method sees), as a fraction.  Returns
    (G, factors, err, q_used)."""
    X = np.asarray(X, dtype=np.float64)
    prev = None
    for t in range(max_q + 1):
        G, factors, err = rbki_tucker(X, ranks, p, t, seed, tau, sample_rate=sample_rate)
        fit = fit_fraction(err)
        if prev is not None and abs(fit - prev) <= fit_tol:
            return G, factors, err, t
        prev = fit
    return G, factors, err, max_q
