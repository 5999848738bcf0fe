"""Seeded synthetic inputs for the Matching Pursuit decoder.

This module only *draws* problems: random dictionaries, sparse signals and the
encoded measurements y = Psi x (Section 2, eqs. 2-4).  It holds none of the
decoder's arithmetic (no correlation, selection or residual update), so the
CPU oracle and the GPU library can both be fed from it without sharing code.

Storage convention used everywhere: a dictionary is returned as a numpy array
``psi`` of shape (N, M) in Fortran (column-major) order, so ``psi[n, m]`` is
the paper's psi_nm and each column psi_m is contiguous in memory (ld = N).

Workloads (all synthetic; the paper measures on no dataset):

* ``c0``  N=256,  M=1024,  K=10,  eps=1e-6, T=2000
* ``c1a`` N=2048, M=8192,  K=128, eps=1e-5, T=20K
* ``c1b`` N=8192, M=32768, K=512, eps=1e-5, T=20K
* ``c2``  N=8192, M=32768, K=256, eps=1e-5, T=20K; values N(0,1) or
          log-uniform magnitudes in [1e-3, 1] with a random sign
* ``c3``  shared N=2048, M=8192 dictionary, B=256 signals, K_b ~ U{16..256}
* ``c4``  512 independent problems, N_i ~ U{128,256,512,1024}, M_i=4N_i,
          K_i=N_i/16
* ``phase`` the Fig. 1 experiment: M=1000, sigma = K/M and rho = N/M on a
          grid, the +-1/sqrt(N) Bernoulli dictionary of eq. 13, nonzeros
          U[-1, 1], eps=1e-7, T=N, 100 trials per cell
* sign-bit problems (:func:`make_sign_problem`): the sizes of ``c0``,
          ``c1a`` or ``c1b`` on the Bernoulli dictionary of eq. 13 held as one
          sign bit per entry (the packed format below)

Dictionaries are Gaussian N(0,1) with every column divided by its FP64 L2 norm
and then rounded to FP32; supports are uniform without replacement; y is
computed in FP64 from the FP32 dictionary and FP32 x, then rounded to FP32.
The FP64 variants of the single-signal workloads (``precision='f64'``) use
the same draws and keep the dictionary, x and y in FP64.
Seeds go through ``numpy.random.SeedSequence([workload_id, seed])``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional

import numpy as np

__all__ = [
    "WORKLOADS", "Problem", "workload", "make_problem", "make_batch",
    "make_ragged", "make_phase_batch", "PhaseBatch", "gaussian_unit_dictionary",
    "bernoulli_dictionary",
    "hadamard_dictionary", "qr_orthonormal_dictionary", "sparse_signal",
    "encode", "rational_unit_dictionary", "rng_streams",
    "bernoulli_signs", "pack_signs", "encode_signs", "make_sign_problem", "SignProblem",
]

# name -> (id used in the seed sequence, N, M, K, eps, iteration cap rule)
WORKLOADS = {
    "c0": dict(wid=0, n=256, m=1024, k=10, eps=1e-6, max_iters=2000),
    "c1a": dict(wid=10, n=2048, m=8192, k=128, eps=1e-5, max_iters=20 * 128),
    "c1b": dict(wid=11, n=8192, m=32768, k=512, eps=1e-5, max_iters=20 * 512),
    "c2": dict(wid=2, n=8192, m=32768, k=256, eps=1e-5, max_iters=20 * 256),
    "c3": dict(wid=3, n=2048, m=8192, b=256, kmin=16, kmax=256, eps=1e-5),
    "c4": dict(wid=4, count=512, n_choices=(128, 256, 512, 1024), eps=1e-5),
    # Fig. 1: M = 1000, sigma = K/M and rho = N/M on a grid, Bernoulli
    # dictionary, nonzeros U[-1, 1], eps = 1e-7, T = N, 100 trials per cell
    "phase": dict(wid=5, m=1000, eps=1e-7, trials=100, draws=4),
}


def workload(name: str) -> dict:
    """The size/stop parameters of a named workload (a copy)."""
    return dict(WORKLOADS[name])


@dataclass
class Problem:
    """One decoding problem: recover x from y = psi @ x."""
    psi: np.ndarray          # (N, M) float32, Fortran order, unit-norm columns
    x: np.ndarray            # (M,) float32 ground truth (K nonzeros)
    y: np.ndarray            # (N,) float32 measurements
    support: np.ndarray      # (K,) int64, sorted
    eps: float
    max_iters: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.psi.shape[0]

    @property
    def m(self) -> int:
        return self.psi.shape[1]


def rng_streams(wid: int, seed: int, count: int) -> List[np.random.Generator]:
    """``count`` independent PCG64 generators spawned from [wid, seed]."""
    ss = np.random.SeedSequence([int(wid), int(seed)])
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(count)]


def gaussian_unit_dictionary(rng: np.random.Generator, n: int, m: int,
                             chunk: int = 2048, dtype=np.float32) -> np.ndarray:
    """N x M Gaussian dictionary, columns normalised in FP64, stored as FP32
    (or kept in FP64 with ``dtype=np.float64``; the same draws, so the FP32
    dictionary is the FP64 one rounded).

    Columns are drawn one after another (column m's N entries are consecutive
    draws), normalised to unit L2 norm (eq. 4) and rounded to ``dtype``.
    """
    cols = np.empty((m, n), dtype=dtype)
    for j0 in range(0, m, chunk):
        j1 = min(m, j0 + chunk)
        g = rng.standard_normal((j1 - j0, n))
        nrm = np.sqrt(np.einsum("ij,ij->i", g, g))
        cols[j0:j1] = (g / nrm[:, None]).astype(dtype)
    return cols.T  # (n, m) view in Fortran order


def bernoulli_dictionary(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    """The paper's +-1/sqrt(N) dictionary (eq. 13), as FP32, column-major."""
    s = rng.integers(0, 2, size=(m, n), dtype=np.int8) * 2 - 1
    cols = (s.astype(np.float64) / np.sqrt(n)).astype(np.float32)
    return cols.T


def bernoulli_signs(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    """The signs of the Bernoulli dictionary (eq. 13): an (M, N) int8 array of
    +-1, row m holding column m's N signs (the same draw as
    :func:`bernoulli_dictionary`)."""
    return rng.integers(0, 2, size=(m, n), dtype=np.int8) * 2 - 1


def pack_signs(s: np.ndarray, ldw: Optional[int] = None) -> np.ndarray:
    """Packed sign-bit format of a +-1 dictionary: an (M, ldw) uint32 array;
    bit q of word w of row m is 1 when entry (32 w + q, m) is negative, 0 when
    positive.  Bits past N in a column's last word, and words past
    ceil(N / 32), are zero."""
    m, n = s.shape
    need = (n + 31) // 32
    ldw = need if ldw is None else int(ldw)
    if ldw < need:
        raise ValueError("ldw must be >= ceil(N / 32)")
    neg = np.zeros((m, ldw * 32), dtype=np.uint8)
    neg[:, :n] = s < 0
    by = np.packbits(neg, axis=1, bitorder="little")          # (M, 4 ldw) bytes
    return np.ascontiguousarray(by).view("<u4").astype(np.uint32, copy=False)


def encode_signs(s: np.ndarray, x: np.ndarray, support: Optional[np.ndarray] = None,
                 dtype=np.float32) -> np.ndarray:
    """y = Psi x (eq. 2) for Psi = S / sqrt(N) with S the (M, N) +-1 array, in
    FP64, rounded to ``dtype``."""
    if support is None:
        support = np.flatnonzero(x)
    n = s.shape[1]
    y = s[support].T.astype(np.float64) @ np.asarray(x[support], dtype=np.float64)
    return (y / np.sqrt(n)).astype(dtype)


@dataclass
class SignProblem:
    """One decoding problem on a Bernoulli dictionary held as sign bits:
    psi_nm = (1 - 2 b_nm) / sqrt(N) with b the bits of :func:`pack_signs`."""
    bits: np.ndarray         # (M, ldw) uint32, packed sign bits
    n: int
    x: np.ndarray            # (M,) float32 ground truth (K nonzeros)
    y: np.ndarray            # (N,) float32 measurements
    support: np.ndarray      # (K,) int64, sorted
    eps: float
    max_iters: int
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.bits.shape[0]


def make_sign_problem(name: str, seed: int, dist: str = "normal") -> SignProblem:
    """The sizes and stopping rule of the single-signal workload ``name``
    (``c0``, ``c1a`` or ``c1b``) on a sign-bit Bernoulli dictionary; x drawn
    as for that workload, y computed in FP64 from the +-1 signs."""
    w = workload(name)
    r_psi, r_sup, r_val = rng_streams(w["wid"] + 200, seed, 3)
    s = bernoulli_signs(r_psi, w["n"], w["m"])
    x, support = sparse_signal(r_sup, r_val, w["m"], w["k"], dist)
    y = encode_signs(s, x, support)
    bits = pack_signs(s)
    return SignProblem(bits, w["n"], x, y, support, w["eps"], w["max_iters"],
                       meta=dict(workload=name, seed=seed, dist=dist, k=w["k"],
                                 dictionary="bernoulli sign bits"))


def hadamard_dictionary(n: int) -> np.ndarray:
    """Sylvester-Hadamard / sqrt(N), N a power of 4 so entries are +-2^-k.

    Orthonormal and exactly representable in FP32 (and BF16/FP8 up to a
    per-column power-of-two scale).
    """
    k = int(round(np.log(n) / np.log(4)))
    if 4 ** k != n:
        raise ValueError("hadamard_dictionary needs N = 4^k")
    h = np.array([[1.0]])
    while h.shape[0] < n:
        h = np.block([[h, h], [h, -h]])
    return np.asfortranarray((h / np.sqrt(n)).astype(np.float32))


def qr_orthonormal_dictionary(rng: np.random.Generator, n: int,
                              dtype=np.float64) -> np.ndarray:
    """Orthonormal N x N dictionary: Q of a Householder QR of a Gaussian."""
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return np.asfortranarray(q.astype(dtype))


def sparse_signal(rng_support: np.random.Generator, rng_values: np.random.Generator,
                  m: int, k: int, dist: str = "normal", dtype=np.float32):
    """K-sparse x (eq. 1): support uniform without replacement.

    ``dist='normal'``: nonzeros i.i.d. N(0,1).  ``dist='loguniform'``:
    magnitudes 10^U(-3,0) with an independent random sign (p = 1/2).
    Returns (x (M,) of ``dtype``, support int64 sorted).
    """
    support = np.sort(rng_support.choice(m, size=k, replace=False)).astype(np.int64)
    if dist == "normal":
        vals = rng_values.standard_normal(k)
    elif dist == "loguniform":
        mag = 10.0 ** rng_values.uniform(-3.0, 0.0, size=k)
        sgn = np.where(rng_values.integers(0, 2, size=k) == 0, -1.0, 1.0)
        vals = mag * sgn
    else:
        raise ValueError(dist)
    x = np.zeros(m, dtype=np.float64)
    x[support] = vals
    return x.astype(dtype), support


def encode(psi: np.ndarray, x: np.ndarray, support: Optional[np.ndarray] = None,
           dtype=np.float32) -> np.ndarray:
    """y = Psi x (eq. 2) in FP64 from the given inputs, rounded to ``dtype``."""
    if support is None:
        support = np.flatnonzero(x)
    cols = np.asarray(psi[:, support], dtype=np.float64)
    y = cols @ np.asarray(x[support], dtype=np.float64)
    return y.astype(dtype)


def make_problem(name: str, seed: int, dist: str = "normal", precision: str = "f32",
                 psi: Optional[np.ndarray] = None) -> Problem:
    """A single-signal workload (``c0``, ``c1a``, ``c1b`` or ``c2``).

    ``precision='f64'`` draws the same problem for the FP64 decoder: the
    dictionary, x and y stay FP64 (no rounding to FP32 anywhere).
    ``psi``: the dictionary this workload and seed draw, already drawn (by an
    earlier call with another ``dist``); it is used as given, which saves
    drawing it again (the dictionary has a stream of its own, so nothing
    else changes)."""
    if precision not in ("f32", "f64"):
        raise ValueError(precision)
    dt = np.float64 if precision == "f64" else np.float32
    w = workload(name)
    r_psi, r_sup, r_val = rng_streams(w["wid"], seed, 3)
    if dist == "loguniform":  # a separate value stream for the second distribution
        r_val = rng_streams(w["wid"] + 100, seed, 1)[0]
    if psi is None:
        psi = gaussian_unit_dictionary(r_psi, w["n"], w["m"], dtype=dt)
    elif psi.shape != (w["n"], w["m"]) or psi.dtype != dt or not psi.flags.f_contiguous:
        raise ValueError("psi must be this workload's (N, M) column-major dictionary")
    x, support = sparse_signal(r_sup, r_val, w["m"], w["k"], dist, dtype=dt)
    y = encode(psi, x, support, dtype=dt)
    return Problem(psi, x, y, support, w["eps"], w["max_iters"],
                   meta=dict(workload=name, seed=seed, dist=dist, k=w["k"],
                             precision=precision))


@dataclass
class Batch:
    """B signals sharing one dictionary (the ``c3`` workload)."""
    psi: np.ndarray          # (N, M) float32 Fortran
    x: np.ndarray            # (M, B) float32 Fortran (column b = signal b)
    y: np.ndarray            # (N, B) float32 Fortran
    k: np.ndarray            # (B,) int64 per-signal sparsity
    eps: float
    max_iters: np.ndarray    # (B,) int64 = 20 K_b


def make_batch(seed: int, b: Optional[int] = None, n: Optional[int] = None,
               m: Optional[int] = None, kmin: Optional[int] = None,
               kmax: Optional[int] = None) -> Batch:
    """The shared-dictionary batch; sizes default to the ``c3`` workload."""
    w = workload("c3")
    n = w["n"] if n is None else n
    m = w["m"] if m is None else m
    b = w["b"] if b is None else b
    kmin = w["kmin"] if kmin is None else kmin
    kmax = w["kmax"] if kmax is None else kmax
    r_psi, r_k, r_sup, r_val = rng_streams(w["wid"], seed, 4)
    psi = gaussian_unit_dictionary(r_psi, n, m)
    ks = r_k.integers(kmin, kmax + 1, size=b).astype(np.int64)
    x = np.zeros((m, b), dtype=np.float32, order="F")
    y = np.zeros((n, b), dtype=np.float32, order="F")
    for j in range(b):
        xj, sup = sparse_signal(r_sup, r_val, m, int(ks[j]))
        x[:, j] = xj
        y[:, j] = encode(psi, xj, sup)
    return Batch(psi, x, y, ks, w["eps"], 20 * ks)


def make_ragged(seed: int, count: Optional[int] = None,
                n_choices=None) -> List[Problem]:
    """Independent problems of uneven size (the ``c4`` workload)."""
    w = workload("c4")
    count = w["count"] if count is None else count
    n_choices = w["n_choices"] if n_choices is None else tuple(n_choices)
    (r_n,) = rng_streams(w["wid"], seed, 1)
    ns = r_n.choice(np.asarray(n_choices), size=count)
    probs = []
    ss = np.random.SeedSequence([w["wid"], int(seed), 1])
    for i, child in enumerate(ss.spawn(count)):
        r_psi, r_sup, r_val = [np.random.Generator(np.random.PCG64(s)) for s in child.spawn(3)]
        n = int(ns[i])
        m, k = 4 * n, n // 16
        psi = gaussian_unit_dictionary(r_psi, n, m)
        x, sup = sparse_signal(r_sup, r_val, m, k)
        probs.append(Problem(psi, x, encode(psi, x, sup), sup, w["eps"], 20 * k,
                             meta=dict(workload="c4", seed=seed, index=i, k=k)))
    return probs


@dataclass
class PhaseBatch:
    """One dictionary draw of the Fig. 1 experiment at one rho: every sigma of
    the grid, ``per_sigma`` signals each, decoded against the same psi."""
    psi: np.ndarray          # (N, M) float32 Fortran, +-fp32(1/sqrt(N))
    x: np.ndarray            # (M, B) float32 Fortran
    y: np.ndarray            # (N, B) float32 Fortran
    sigma_index: np.ndarray  # (B,) index into the sigma grid of each signal
    ks: np.ndarray           # (B,) K of each signal
    eps: float
    max_iters: int           # T = N


def make_phase_batch(seed: int, rho: float, sigmas, draw: int, per_sigma: int,
                     m: Optional[int] = None) -> PhaseBatch:
    """Draw ``draw`` of the Fig. 1 experiment at ``rho``: N = round(rho M)
    rows of the Bernoulli dictionary (eq. 13), and for every sigma in
    ``sigmas`` ``per_sigma`` signals with K = round(sigma M) nonzeros drawn
    from U[-1, 1] on a support uniform without replacement (K is capped at
    M).  y = psi x in FP64, rounded to FP32."""
    w = workload("phase")
    m = w["m"] if m is None else m
    n = max(1, int(round(rho * m)))
    ss = np.random.SeedSequence([w["wid"], int(seed), n, int(draw)])
    r_psi, r_sup, r_val = [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(3)]
    psi = bernoulli_dictionary(r_psi, n, m)
    sig = np.asarray(list(sigmas), dtype=np.float64)
    b = len(sig) * per_sigma
    x = np.zeros((m, b), dtype=np.float32, order="F")
    y = np.zeros((n, b), dtype=np.float32, order="F")
    sidx = np.repeat(np.arange(len(sig)), per_sigma)
    ks = np.minimum(np.maximum(np.rint(sig[sidx] * m).astype(np.int64), 1), m)
    for j in range(b):
        k = int(ks[j])
        sup = np.sort(r_sup.choice(m, size=k, replace=False))
        x[sup, j] = r_val.uniform(-1.0, 1.0, size=k).astype(np.float32)
        y[:, j] = encode(psi, x[:, j], sup)
    return PhaseBatch(psi, x, y, sidx, ks, w["eps"], n)


def rational_unit_dictionary(rng: np.random.Generator, n: int, m: int,
                             den: int = 7) -> List[List[Fraction]]:
    """Columns that are *exactly* unit norm in rational arithmetic.

    Inverse stereographic projection of a random rational t in Q^(N-1):
    psi = (2t, |t|^2 - 1) / (|t|^2 + 1) has |psi|^2 = 1 exactly.  Coordinates
    are then permuted and sign-flipped at random (both keep the norm exact).
    Returned as a list of M columns, each a list of N Fractions.
    """
    cols = []
    for _ in range(m):
        t = [Fraction(int(v), den) for v in rng.integers(-2 * den, 2 * den + 1, size=n - 1)]
        s = sum(v * v for v in t)
        d = s + 1
        col = [2 * v / d for v in t] + [(s - 1) / d]
        perm = rng.permutation(n)
        sg = rng.integers(0, 2, size=n) * 2 - 1
        cols.append([col[int(perm[i])] * int(sg[i]) for i in range(n)])
    return cols
