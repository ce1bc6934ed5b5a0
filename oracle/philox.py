"""Counter-based Gaussian stream for the sketch matrix Omega (Alg. 1, step 1).

The paper only says Omega is a "randomized sketching matrix" with Gaussian
entries (Sec. 2.2 and Alg. 1).  To make the CPU oracle and the GPU draw the
*same* Omega, both sides implement the Philox4x32-10 counter-based generator
from its published definition (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11) and the Box-Muller transform (Box and
Muller, 1958).  This file is the oracle's own implementation; the GPU has
another one, written separately.

Philox4x32-10 (published definition):
  state: four 32-bit counter words (c0, c1, c2, c3) and two key words (k0, k1);
  one round: with (hi0, lo0) = 0xD2511F53 * c0 and (hi1, lo1) = 0xCD9E8D57 * c2
  as 64-bit products split into halves,
      (c0, c1, c2, c3) <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
  the key is advanced by (0x9E3779B9, 0xBB67AE85) between rounds; ten rounds.

Conventions fixed here (shared with the GPU by definition, not by code):
  key        = (seed mod 2^32, seed >> 32)
  Omega^(n)[j, s] has linear index L = s * J_n + j (column-major, so the
  columns do not depend on the sketch width and sketches for different p are
  nested), and is drawn from the Philox block with counter
  (lo32(L >> 1), hi32(L >> 1), n, tag) with tag = 0 for Omega.
  From the four output words w0..w3:
      u1 = (w0 * 2^20 + (w1 >> 12) + 0.5) * 2^-52      (in the open (0, 1);
      u2 = (w2 * 2^20 + (w3 >> 12) + 0.5) * 2^-52       both sums are exact)
      z  = sqrt(-2 ln u1) * (cos(2 pi u2) if L is even else sin(2 pi u2)).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
ROUNDS = 10

TAG_OMEGA = 0
TAG_COLUMNS = 1


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Philox4x32 on arrays of 32-bit words held in uint64 (one block per
    element).  Returns the four output words as uint64 arrays < 2^32."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0          # exact: both factors < 2^32, product < 2^64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox4x32_scalar(ctr, key, rounds=ROUNDS):
    """The same function on Python integers, one block at a time (used only to
    cross-check the vectorised version on small inputs)."""
    c = [int(v) & 0xFFFFFFFF for v in ctr]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
    return tuple(c)


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def words_to_unit(wa, wb):
    """52-bit uniform in the open interval (0, 1) from two 32-bit words
    (k + 1/2) 2^-52 with k < 2^52 is exact in float64, so 1 is never hit."""
    hi = wa.astype(np.float64) * 1048576.0                   # wa * 2^20
    lo = (wb >> np.uint64(12)).astype(np.float64)
    return (hi + lo + 0.5) * (2.0 ** -52)


def gaussian_at(seed, mode, linear_index, tag=TAG_OMEGA):
    """Standard normal values at the given linear indices of the stream
    (seed, mode, tag), by the Box-Muller transform."""
    L = np.asarray(linear_index, dtype=np.uint64)
    pair = L >> np.uint64(1)
    k0, k1 = seed_key(seed)
    n = np.full(L.shape, int(mode) & 0xFFFFFFFF, dtype=np.uint64)
    t = np.full(L.shape, int(tag) & 0xFFFFFFFF, dtype=np.uint64)
    w0, w1, w2, w3 = philox4x32(pair & MASK32, pair >> np.uint64(32), n, t, k0, k1)
    u1 = words_to_unit(w0, w1)
    u2 = words_to_unit(w2, w3)
    radius = np.sqrt(-2.0 * np.log(u1))
    angle = 2.0 * np.pi * u2
    odd = (L & np.uint64(1)).astype(bool)
    return np.where(odd, radius * np.sin(angle), radius * np.cos(angle))


def omega(seed, mode, J, S, chunk=1 << 22):
    """The sketch matrix Omega^(n) in R^{J x S} (Alg. 1, step 1), float64.
    Column s holds stream indices s*J .. s*J + J - 1."""
    out = np.empty((J, S), dtype=np.float64, order="F")
    flat = out.reshape(-1, order="F")
    total = J * S
    for start in range(0, total, chunk):
        stop = min(total, start + chunk)
        flat[start:stop] = gaussian_at(seed, mode, np.arange(start, stop, dtype=np.uint64))
    return out


def sample_count(J, rate):
    """Number of sampled columns m = round(rate * J), at least 1 and at most J
    (rate >= 1: all columns)."""
    if rate >= 1.0:
        return int(J)
    return int(max(1, min(J, int(np.floor(rate * J + 0.5)))))


def sampled_columns(seed, mode, J, rate):
    """Uniform column sample of the mode-n unfolding (Sec. 3.1: the Krylov
    basis may be built from m = rate * J of the J columns).

    Stratified uniform sampling: the columns are split into m consecutive
    strata [floor(k J / m), floor((k+1) J / m)) and stratum k contributes the
    column at offset floor(w * width / 2^32), where w is the first output word
    of the Philox block with counter (lo32(k), hi32(k), mode, tag 1).  Every
    column is drawn with probability about m / J, exactly m distinct columns
    come out, in increasing order, and rate = 1 gives every column.  All
    arithmetic is on integers."""
    m = sample_count(J, rate)
    k = np.arange(m, dtype=np.uint64)
    Jm = np.uint64(J)
    lo = (k * Jm) // np.uint64(m)
    width = ((k + np.uint64(1)) * Jm) // np.uint64(m) - lo
    k0, k1 = seed_key(seed)
    tag = np.full(k.shape, TAG_COLUMNS, dtype=np.uint64)
    w0, _, _, _ = philox4x32(k & MASK32, k >> np.uint64(32), np.full(k.shape, int(mode) & 0xFFFFFFFF, np.uint64),
                             tag, k0, k1)
    return (lo + ((w0 * width) >> np.uint64(32))).astype(np.int64)
