"""The Bernoulli dictionary of eq. 13 held as one sign bit per entry, for the
oracle: read the packed bits back into the FP64 dictionary and run the plain
FP64 Matching Pursuit on it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Packed format (the decoder's input): an (M, ldw) array of 32-bit words, row m
holding column m; bit q of word w is b_nm for row n = 32 w + q.  The
dictionary it stands for is psi_nm = (1 - 2 b_nm) / sqrt(N): +1/sqrt(N) for a
0 bit, -1/sqrt(N) for a 1 bit (eq. 13's entries, every column of unit norm).
Bits of rows n >= N are not part of the dictionary.

The decode needs no arithmetic of its own: it is the FP64 Matching Pursuit
of Section 3 (``oracle.solve``, eqs. 8-12 with the tie rule of eq. 16) on the
dictionary read back exactly as defined above, y rounded to FP32 as the
decoder receives it.
"""
from __future__ import annotations

import numpy as np

from . import correlate as _correlate
from . import solve as _solve

_CHUNK = 2048  # columns read back at a time (bounds the temporary bit array)


def _bit_matrix(words: np.ndarray, n: int) -> np.ndarray:
    """(columns, N) array of b_nm in {0, 1}: bit q of word w is row 32 w + q."""
    q = np.arange(32, dtype=np.uint32)
    b = (words[:, :, None] >> q) & np.uint32(1)          # (cols, ldw, 32)
    return b.reshape(words.shape[0], -1)[:, :n]


def _entries(b: np.ndarray, n: int) -> np.ndarray:
    """psi_nm = (1 - 2 b_nm) / sqrt(N) in FP64."""
    return (1.0 - 2.0 * b.astype(np.float64)) / np.sqrt(float(n))


def unpack(bits: np.ndarray, n: int) -> np.ndarray:
    """The FP64 dictionary (N, M), column-major, that ``bits`` stands for."""
    bits = np.asarray(bits)
    if bits.ndim != 2 or bits.dtype != np.uint32:
        raise TypeError("bits must be a 2-D uint32 array (M, ldw)")
    m, ldw = bits.shape
    if n < 1 or ldw * 32 < n:
        raise ValueError("need 1 <= N <= 32 ldw")
    psi = np.empty((n, m), dtype=np.float64, order="F")
    for j0 in range(0, m, _CHUNK):
        j1 = min(m, j0 + _CHUNK)
        psi[:, j0:j1] = _entries(_bit_matrix(bits[j0:j1], n), n).T
    return psi


def solve_signs(bits: np.ndarray, n: int, y: np.ndarray, eps: float, max_iters: int,
                trace: bool = True):
    """FP64 Matching Pursuit (``oracle.solve``) on the sign-bit dictionary."""
    return _solve(unpack(bits, n), y, eps, max_iters, trace=trace)


def correlate_signs(bits: np.ndarray, n: int, r: np.ndarray) -> np.ndarray:
    """c = Psi^T r in FP64 (eq. 9) on the sign-bit dictionary."""
    return _correlate(unpack(bits, n), np.asarray(r, dtype=np.float64))
