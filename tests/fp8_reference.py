"""What the fp8 form of rBKI-TK computes, in float64 on the CPU (test infrastructure).

The fp8 form feeds its Gram and sketch products with block-scaled e4m3
copies of the tensor and of the sketch: every run of 32 consecutive values
along a storage row gets the smallest power-of-two scale 2^s with
max|x| / 2^s <= 448, and x / 2^s is rounded to the nearest OCP e4m3 ("fn")
value, ties to even.  Storage rows are the last dimension for every mode but
the last.  For the last mode (the transposed copy) they run over the
flattened leading index, with the runs of 32 restarting at every run of the
last leading dimension I_{N-1} (the copy pads each such run to a multiple of
64).  The sketch is generated, rounded to bf16, and quantised the same way
in its column layout.  A mode whose Gram product falls back to bf16 (I_n <= 128
or S_n > 64) reads bf16-rounded operands instead.

Everything after that (Krylov basis, Z, eigenvectors, core and error) is the
oracle's float64 arithmetic; the core and the error use the unquantised
tensor.  Written from the OCP 8-bit floating point specification and the
oracle's own functions; shares nothing with the HIP implementation.
"""
import numpy as np

from oracle import philox
from oracle.rbki import rbki_basis, ritz_factor, sketch_size
from oracle.tensor import unfold, view_dims, project_core, tucker_to_full, fro


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), via float32."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_e4m3(y):
    """Nearest e4m3 value (3 mantissa bits, subnormal quantum 2^-9, ties to
    even, magnitudes above 448 saturate); |y| is expected to be <= 448."""
    a = np.abs(y)
    _, e = np.frexp(a)                         # a in [2^(e-1), 2^e)
    quantum = np.where(a >= 2.0 ** -6, np.ldexp(1.0, e - 4), 2.0 ** -9)
    r = np.minimum(np.round(a / quantum) * quantum, 448.0)
    return np.sign(y) * r


def block_quantize(M):
    """Block-scaled e4m3 along the last axis, runs of 32 (zero-padded)."""
    M = np.asarray(M, np.float64)
    n = M.shape[-1]
    npad = -(-n // 32) * 32
    P = np.zeros(M.shape[:-1] + (npad,))
    P[..., :n] = M
    B = P.reshape(M.shape[:-1] + (npad // 32, 32))
    amax = np.abs(B).max(axis=-1, keepdims=True)
    m, e = np.frexp(amax)                      # amax = m 2^e, m in [0.5, 1)
    s = np.where(m <= 0.875, e - 9, e - 8)     # smallest s with amax / 2^s <= 448 (448 = 0.875 2^9)
    s = np.where(amax > 0, np.clip(s, -127, 127), -127)
    Q = round_e4m3(B / np.ldexp(1.0, s)) * np.ldexp(1.0, s)
    return Q.reshape(P.shape)[..., :n]


def uses_fp8(I, S):
    return I > 128 and 1 <= S <= 64


def quantised_mode_operand(X, n, fp8):
    """The mode-n unfolding of the operand the Gram product reads."""
    N = X.ndim
    IN = X.shape[-1]
    rows = X.size // IN
    if n < N - 1:
        V = X.reshape(rows, IN)
        Vq = block_quantize(V) if fp8 else round_bf16(V)
        return unfold(Vq.reshape(X.shape), n)
    L = X.shape[-2]
    T = X.reshape(rows // L, L, IN).transpose(2, 0, 1)   # I_N x H x I_{N-1}
    Tq = block_quantize(T) if fp8 else round_bf16(T)
    return Tq.reshape(IN, rows)                # the last mode's unfolding


def quantised_sketch(X, n, J, S, seed, fp8):
    """Omega^(n) (J x S) as the fp8 form's Gram product reads it."""
    Om = round_bf16(philox.omega(seed, n, J, S))
    if not fp8:
        return Om
    N = X.ndim
    IN = X.shape[-2] if n == N - 1 else X.shape[-1]
    OmT = Om.T.reshape(S, J // IN, IN)         # runs along the copy's storage rows
    return block_quantize(OmT).reshape(S, J).T


def rbki_tucker_fp8_operands(X, ranks, p, q, seed):
    """Factors, core and relative error of rBKI-TK when the Krylov basis and
    Z are built from the fp8 form's operands."""
    X = np.asarray(X, np.float64)
    factors = []
    for n in range(X.ndim):
        A, I, B = view_dims(X.shape, n)
        J = A * B
        S = sketch_size(ranks[n], p, I, J)
        fp8 = uses_fp8(I, S)
        Xn = quantised_mode_operand(X, n, fp8)
        Om = quantised_sketch(X, n, J, S, seed, fp8)
        Q, _ = rbki_basis(Xn, Om, q)
        U, _ = ritz_factor(Xn, Q, ranks[n])
        factors.append(U)
    G = project_core(X, factors)
    err = fro(X - tucker_to_full(G, factors)) / fro(X)
    return G, factors, err
