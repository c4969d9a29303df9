"""Sketching operators of the oracle: CountSketch (Clarkson-Woodruff), the
sparse sign embedding, the Gaussian sketch and the subsampled randomized
Hadamard transform, in float64.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Paper: Sec. 1.2 lists the three sketch-and-solve steps (generate S, form SA and
Sb, solve on SA); Sec. 1.2.2 defines the Clarkson-Woodruff sketch as a sparse
matrix combined with a random sign matrix (one nonzero per column of S);
Sec. 1.2.1 defines the Gaussian sketch by i.i.d. Gaussian entries; Sec. 1.3
fixes the shapes S in R^{d x m}, A in R^{m x n}.

Readings fixed here (the paper is silent on them):
  * hash layout: row i uses Philox4x32-10 block j = i >> 1 with counter
    (j mod 2^32, j >> 32, 0, 0) and key (seed mod 2^32, seed >> 32); lane
    i & 1 takes words (2*lane, 2*lane+1) as (w_h, w_s).  The bucket is the
    multiply-shift reduction h = (w_h * d) >> 32 and the sign is +1 when the
    top bit of w_s is clear, else -1.  Entries of S are +-1 with no scale.
  * sparse sign embedding (the sparse sketch family of Sec. 1.2.2 with zeta
    nonzeros per column): nonzero k of column i uses the CountSketch rule
    with counter (j mod 2^32, j >> 32, k, 0), so k = 0 is the CountSketch
    itself; S is the sum of the zeta one-per-column matrices (entries +-1,
    no scale; a collision of two entries in one row adds them).
  * Gaussian sketch: entry G[k, i] is the table value T[q] where q is one
    byte of Philox4x32-10 at counter (j mod 2^32, j >> 32, k, 1), j = i >> 4,
    and key seed: byte (i & 15) of the little-endian 16-byte output, so one
    generator call serves 16 consecutive rows of A for one sketch row.  T[q]
    is the inverse normal CDF at the midpoint (q + 1/2) / 256 rounded to
    bfloat16 (round to nearest even).  SA = d^{-1/2} G bf16(A),
    Sb = d^{-1/2} G bf16(b).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.special import ndtri

from .philox import philox4x32

TAG_COUNT = 0
TAG_GAUSS = 1


# --------------------------------------------------------------------------
# CountSketch hash
# --------------------------------------------------------------------------

def countsketch_hash(seed: int, d: int, i0: int, count: int):
    """Bucket h(i) in [0, d) and sign s(i) in {+1, -1} for rows i0 .. i0+count-1.

    Returns (h uint32[count], s int8[count]).
    """
    return sparse_sign_hash(seed, d, i0, count, 0)


def sparse_sign_hash(seed: int, d: int, i0: int, count: int, k: int):
    """Bucket and sign of nonzero k of columns i0 .. i0+count-1 of the sparse
    sign embedding: the CountSketch rule with counter word 2 set to k (k = 0 is
    the CountSketch hash itself).  Returns (h uint32[count], s int8[count])."""
    if count == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.int8)
    i = np.uint64(i0) + np.arange(count, dtype=np.uint64)
    j = i >> np.uint64(1)
    lane = (i & np.uint64(1)).astype(bool)
    c0 = (j & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    c1 = (j >> np.uint64(32)).astype(np.uint32)
    zero = np.zeros_like(c0)
    w0, w1, w2, w3 = philox4x32(c0, c1, zero + np.uint32(k), zero + TAG_COUNT,
                                seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w_h = np.where(lane, w2, w0)
    w_s = np.where(lane, w3, w1)
    h = ((w_h.astype(np.uint64) * np.uint64(d)) >> np.uint64(32)).astype(np.uint32)
    s = (1 - 2 * (w_s >> np.uint32(31)).astype(np.int16)).astype(np.int8)
    return h, s


def countsketch_matrix(seed: int, d: int, m: int) -> sp.csr_matrix:
    """The sketch S in R^{d x m} as a sparse matrix: S[h(i), i] = s(i)."""
    h, s = countsketch_hash(seed, d, 0, m)
    return sp.csr_matrix((s.astype(np.float64), (h.astype(np.int64), np.arange(m))), shape=(d, m))


def countsketch_apply(A, b, seed: int, d: int):
    """SA = S A and Sb = S b in float64 with S from countsketch_matrix.

    A may be a dense (m, n) array or a scipy sparse matrix; its values are
    widened to float64 first, so the result is the exact product of the
    stored inputs up to float64 rounding.  b may be None.
    """
    m = A.shape[0]
    S = countsketch_matrix(seed, d, m)
    if sp.issparse(A):
        SA = (S @ A.astype(np.float64)).toarray()
    else:
        SA = S @ np.asarray(A, dtype=np.float64)
    Sb = None if b is None else S @ np.asarray(b, dtype=np.float64)
    return np.asarray(SA), Sb


def sparse_sign_matrix(seed: int, d: int, m: int, zeta: int) -> sp.csr_matrix:
    """The sparse sign embedding with zeta nonzeros per column, as the sum of
    zeta independent CountSketch matrices: S[h_k(i), i] += s_k(i) for
    k = 0 .. zeta-1 (two of a column's entries that land in one row add)."""
    rows, cols, vals = [], [], []
    for k in range(zeta):
        h, s = sparse_sign_hash(seed, d, 0, m, k)
        rows.append(h.astype(np.int64))
        cols.append(np.arange(m))
        vals.append(s.astype(np.float64))
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(d, m))
    return S.tocsr()  # duplicates summed


def sparse_sign_apply(A, b, seed: int, d: int, zeta: int):
    """SA = S A and Sb = S b in float64 with S from sparse_sign_matrix."""
    S = sparse_sign_matrix(seed, d, A.shape[0], zeta)
    if sp.issparse(A):
        SA = (S @ A.astype(np.float64)).toarray()
    else:
        SA = S @ np.asarray(A, dtype=np.float64)
    Sb = None if b is None else S @ np.asarray(b, dtype=np.float64)
    return np.asarray(SA), Sb


def countsketch_apply_loop(A, b, seed: int, d: int):
    """The same sketch as an explicit loop over rows in ascending order.

    For each row i: SA[h(i), :] += s(i) A[i, :], Sb[h(i)] += s(i) b[i].
    Slow; for small inputs only.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    h, s = countsketch_hash(seed, d, 0, m)
    SA = np.zeros((d, n))
    Sb = np.zeros(d)
    for i in range(m):
        SA[h[i], :] += s[i] * A[i, :]
        if b is not None:
            Sb[h[i]] += s[i] * float(b[i])
    return SA, (None if b is None else Sb)


# --------------------------------------------------------------------------
# bfloat16 rounding and the Gaussian table
# --------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (8 significant bits),
    ties to even, returned as float64.  Values here stay in the normal range
    of bfloat16; zero maps to zero."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    e = np.floor(np.log2(np.abs(x[nz])))
    ulp = np.exp2(e - 7.0)
    q = x[nz] / ulp
    # guard the log2 boundary: a mantissa in [256, 512) means e was one low
    big = np.abs(q) >= 256.0
    ulp = np.where(big, ulp * 2.0, ulp)
    q = x[nz] / ulp
    out[nz] = np.rint(q) * ulp  # np.rint rounds half to even
    return out


def gaussian_table() -> np.ndarray:
    """T[q] = bf16(Phi^{-1}((q + 1/2) / 256)) for q = 0..255, float64."""
    q = np.arange(256, dtype=np.float64)
    return bf16_round(ndtri((q + 0.5) / 256.0))


def gaussian_codes(seed: int, d: int, i0: int, count: int, rows=None) -> np.ndarray:
    """Byte codes q[k, i] (uint8, shape (d, count)) for columns i0..i0+count-1;
    with `rows` given, only those sketch rows k (shape (len(rows), count))."""
    kk = np.arange(d, dtype=np.uint32) if rows is None else np.asarray(rows, dtype=np.uint32)
    d = kk.size
    if count == 0:
        return np.zeros((d, 0), dtype=np.uint8)
    j0 = i0 >> 4
    j1 = (i0 + count - 1) >> 4
    nb = j1 - j0 + 1
    jj = np.uint64(j0) + np.arange(nb, dtype=np.uint64)
    J = np.repeat(jj, d)                 # block-major: (block, k)
    K = np.tile(kk, nb)
    c0 = (J & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    c1 = (J >> np.uint64(32)).astype(np.uint32)
    c3 = np.full(J.shape, TAG_GAUSS, dtype=np.uint32)
    w = philox4x32(c0, c1, K, c3, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    # bytes of (w0, w1, w2, w3), little-endian: byte b is column 16 j + b
    by = np.stack(w, axis=1).astype(np.uint32)            # (nb * d, 4)
    shifts = np.array([0, 8, 16, 24], dtype=np.uint32)
    q = ((by[:, :, None] >> shifts[None, None, :]) & np.uint32(0xFF)).astype(np.uint8)
    q = q.reshape(nb, d, 16)                              # (block, k, byte)
    full = np.transpose(q, (1, 0, 2)).reshape(d, nb * 16)  # columns 16 j0 .. 16 j1 + 15
    off = i0 - 16 * j0
    return np.ascontiguousarray(full[:, off:off + count])


def gaussian_matrix(seed: int, d: int, m: int, i0: int = 0, rows=None) -> np.ndarray:
    """G[k, i] for i in [i0, i0+m) (unscaled, float64, shape (d, m)); with
    `rows`, only those sketch rows."""
    return gaussian_table()[gaussian_codes(seed, d, i0, m, rows)]


def gaussian_apply(A, b, seed: int, d: int):
    """SA = d^{-1/2} G bf16(A), Sb = d^{-1/2} G bf16(b), in float64."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    G = gaussian_matrix(seed, d, m)
    scale = 1.0 / math.sqrt(d)
    SA = scale * (G @ bf16_round(A))
    Sb = None if b is None else scale * (G @ bf16_round(np.asarray(b, dtype=np.float64)))
    return SA, Sb


# --------------------------------------------------------------------------
# Subsampled randomized Hadamard transform (the Hadamard sketch of Sec. 1.2.1)
# --------------------------------------------------------------------------
#
# Readings fixed here: A is padded with zero rows to m' = 2^L >= m rows;
# S = d^{-1/2} P H D with D = diag(s(i)) random signs, H the unnormalised
# Sylvester-Hadamard matrix (H[r, i] = (-1)^popcount(r & i)) and P the
# selection of d rows r_0 .. r_{d-1} drawn uniformly from [0, m') with
# replacement.  Generator words: s(i) is +1 when the top bit of word (i & 3)
# of Philox4x32-10 at counter (i >> 2 mod 2^32, i >> 34, 0, 2) is clear;
# r_k = (w * m') >> 32 with w word (k & 3) of Philox4x32-10 at counter
# (k >> 2 mod 2^32, k >> 34, 0, 3); key = seed as for the other sketches.

TAG_HAD_SIGN = 2
TAG_HAD_ROWS = 3


def _words_by_index(seed: int, idx: np.ndarray, tag: int) -> np.ndarray:
    idx = idx.astype(np.uint64)
    q = idx >> np.uint64(2)
    c0 = (q & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    c1 = (q >> np.uint64(32)).astype(np.uint32)
    zero = np.zeros_like(c0)
    w = philox4x32(c0, c1, zero, zero + np.uint32(tag), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    lane = (idx & np.uint64(3)).astype(np.int64)
    return np.choose(lane, w)


def hadamard_padded_rows(m: int) -> int:
    """m' = the smallest power of two >= m."""
    return 1 << max(0, (int(m) - 1).bit_length())


def hadamard_signs(seed: int, m: int) -> np.ndarray:
    """s(i) in {+1, -1} for i in [0, m), int8."""
    w = _words_by_index(seed, np.arange(m, dtype=np.uint64), TAG_HAD_SIGN)
    return (1 - 2 * (w >> np.uint32(31)).astype(np.int16)).astype(np.int8)


def hadamard_rows(seed: int, d: int, mp: int) -> np.ndarray:
    """The d sampled rows r_k of H D A, int64."""
    w = _words_by_index(seed, np.arange(d, dtype=np.uint64), TAG_HAD_ROWS)
    return ((w.astype(np.uint64) * np.uint64(mp)) >> np.uint64(32)).astype(np.int64)


def hadamard_sign_matrix(rows: np.ndarray, mp: int) -> np.ndarray:
    """H[rows, :] for the unnormalised Sylvester-Hadamard matrix of order mp:
    entry (k, i) = (-1)^popcount(rows[k] & i)."""
    i = np.arange(mp, dtype=np.int64)
    x = rows[:, None] & i[None, :]
    pc = np.zeros(x.shape, dtype=np.int64)
    while np.any(x):
        pc += x & 1
        x >>= 1
    return 1.0 - 2.0 * (pc & 1)


def hadamard_matrix(seed: int, d: int, m: int) -> np.ndarray:
    """S = d^{-1/2} P H D restricted to the m real rows (dense, float64)."""
    mp = hadamard_padded_rows(m)
    H = hadamard_sign_matrix(hadamard_rows(seed, d, mp), mp)[:, :m]
    return H * hadamard_signs(seed, m).astype(np.float64)[None, :] / math.sqrt(d)


def hadamard_apply(A, b, seed: int, d: int):
    """SA = S A and Sb = S b in float64 with S from hadamard_matrix."""
    A = np.asarray(A, dtype=np.float64)
    S = hadamard_matrix(seed, d, A.shape[0])
    SA = S @ A
    Sb = None if b is None else S @ np.asarray(b, dtype=np.float64)
    return SA, Sb
