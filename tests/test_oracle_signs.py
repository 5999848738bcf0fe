"""Pins of the sign-bit dictionary oracle (``oracle.signs``): reading the
packed format back into eq. 13's +-1/sqrt(N) entries, and the FP64 Matching
Pursuit on it, against facts fixed by the format's definition and by
mathematics; planted mistakes must be caught.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

import mpgen
import oracle
from oracle import signs


def _sylvester(n):
    """+-1 Sylvester-Hadamard matrix of order n (a power of two): H^T H = n I."""
    h = np.array([[1]], dtype=np.int64)
    while h.shape[0] < n:
        h = np.kron(np.array([[1, 1], [1, -1]], dtype=np.int64), h)
    return h


def _pack_by_hand(s, ldw=None, tail_garbage=False, rng=None):
    """Pack an (M, N) +-1 array word by word with integer arithmetic (no numpy
    bit routines): bit q of word w is 1 where row 32 w + q is negative.  With
    ``tail_garbage`` the unused bits and words are filled at random: the format
    says they are not part of the dictionary."""
    m, n = s.shape
    need = (n + 31) // 32
    ldw = need if ldw is None else ldw
    out = np.zeros((m, ldw), dtype=np.uint32)
    for j in range(m):
        for w in range(ldw):
            v = 0
            for q in range(32):
                i = 32 * w + q
                if i < n:
                    if s[j, i] < 0:
                        v |= 1 << q
                elif tail_garbage and rng.integers(0, 2):
                    v |= 1 << q
            out[j, w] = v
    return out


# ---- facts ---------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 5, 31, 32, 33, 100])
def test_entries_follow_the_format(n):
    """Every entry is +1/sqrt(N) for a clear bit and -1/sqrt(N) for a set one,
    read at the position the format fixes; tail bits and spare words are
    ignored."""
    rng = np.random.default_rng(n)
    s = rng.integers(0, 2, size=(7, n)) * 2 - 1
    bits = _pack_by_hand(s, ldw=(n + 31) // 32 + 1, tail_garbage=True, rng=rng)
    psi = signs.unpack(bits, n)
    assert psi.shape == (n, 7) and psi.flags.f_contiguous
    want = s.T / np.sqrt(n)
    assert np.array_equal(psi, want)


def test_hadamard_columns_are_orthonormal():
    """The Sylvester matrix read back through the format is orthonormal
    (Psi^T Psi = I): this fixes the scale at exactly 1/sqrt(N), the bit order
    (a permutation applied to the bits but not to y would break recovery
    below) and the sign convention up to a global sign."""
    h = _sylvester(64)
    psi = signs.unpack(_pack_by_hand(h.T), 64)
    np.testing.assert_array_equal(psi * 8.0, h)   # 1/sqrt(64) = 1/8 exactly
    np.testing.assert_allclose(psi.T @ psi, np.eye(64), rtol=0, atol=1e-15)


def test_generator_packing_agrees_with_the_format():
    """mpgen's packed dictionaries (numpy's packbits) read back as the +-1
    draws they were packed from."""
    rng = np.random.default_rng(3)
    s = mpgen.bernoulli_signs(rng, 77, 40)
    np.testing.assert_array_equal(signs.unpack(mpgen.pack_signs(s), 77),
                                  s.T / np.sqrt(77))
    np.testing.assert_array_equal(mpgen.pack_signs(s), _pack_by_hand(s))


def test_hadamard_mp_is_exact_and_breaks_ties_low():
    """Orthonormal +-1/8 columns and dyadic nonzeros: MP is a sort of |Psi^T y|,
    exact in FP64; equal magnitudes go to the smaller index (eq. 16)."""
    h = _sylvester(64)
    x = np.zeros(64)
    x[[40, 5, 17, 3]] = [0.25, 0.5, -0.5, 0.125]
    y = (h @ x) / 8.0
    res = signs.solve_signs(_pack_by_hand(h.T), 64, y, 0.0, 10)
    assert res.idx.tolist() == [5, 17, 40, 3]
    assert res.iters == 4 and res.reason == oracle.CONVERGED and res.rr == 0.0
    np.testing.assert_array_equal(res.x, x)
    np.testing.assert_allclose(res.coef, [0.5, -0.5, 0.25, 0.125], rtol=0, atol=0)


def test_correlation_is_signed_sum_over_sqrt_n():
    """c_m = (sum of r over rows with a clear bit - sum over rows with a set
    bit) / sqrt(N), summed exactly for small integer r."""
    rng = np.random.default_rng(9)
    n, m = 45, 20
    s = rng.integers(0, 2, size=(m, n)) * 2 - 1
    r = rng.integers(-5, 6, size=n).astype(np.float64)
    c = signs.correlate_signs(_pack_by_hand(s), n, r)
    want = np.array([(r[s[j] > 0].sum() - r[s[j] < 0].sum()) for j in range(m)]) / np.sqrt(n)
    np.testing.assert_allclose(c, want, rtol=1e-15, atol=1e-15)


def test_random_bernoulli_recovery():
    """N=128, M=256, K=4 with well separated magnitudes: MP picks the support
    first and drives r to the stop threshold (the paper's claim for small
    sigma, large rho, on its own dictionary)."""
    rng = np.random.default_rng(21)
    s = mpgen.bernoulli_signs(rng, 128, 256)
    x = np.zeros(256)
    sup = [9, 60, 130, 201]
    x[sup] = [1.0, -0.8, 0.6, -0.4]
    y = mpgen.encode_signs(s, x, np.array(sup), dtype=np.float64)
    res = signs.solve_signs(mpgen.pack_signs(s), 128, y, 1e-6, 400)
    assert res.reason == oracle.CONVERGED
    assert sorted(res.idx[:4].tolist()) == sup
    assert np.linalg.norm(res.x - x) <= 1e-5 * np.linalg.norm(x)


# ---- planted mistakes ----------------------------------------------------------

def _battery():
    failed = []
    checks = [
        ("format", lambda: [test_entries_follow_the_format(n) for n in (5, 33)]),
        ("orthonormal", test_hadamard_columns_are_orthonormal),
        ("generator", test_generator_packing_agrees_with_the_format),
        ("hadamard_mp", test_hadamard_mp_is_exact_and_breaks_ties_low),
        ("signed_sum", test_correlation_is_signed_sum_over_sqrt_n),
    ]
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


def test_unmodified_oracle_passes_battery():
    assert _battery() == []


def _bits_msb_first(words, n):
    q = np.arange(31, -1, -1, dtype=np.uint32)
    b = (words[:, :, None] >> q) & np.uint32(1)
    return b.reshape(words.shape[0], -1)[:, :n]


def _bits_last_n(words, n):  # the last N bits of the words instead of the first N
    q = np.arange(32, dtype=np.uint32)
    b = (words[:, :, None] >> q) & np.uint32(1)
    b = b.reshape(words.shape[0], -1)
    return b[:, b.shape[1] - n:]


def _entries_flipped(b, n):
    return (2.0 * b.astype(np.float64) - 1.0) / np.sqrt(float(n))


def _entries_over_n(b, n):
    return (1.0 - 2.0 * b.astype(np.float64)) / float(n)


@pytest.mark.parametrize("name,attr,fn", [
    ("bit_order_reversed", "_bit_matrix", _bits_msb_first),
    ("last_n_bits_taken", "_bit_matrix", _bits_last_n),
    ("sign_convention_flipped", "_entries", _entries_flipped),
    ("scale_one_over_n", "_entries", _entries_over_n),
])
def test_planted_mistakes_are_caught(monkeypatch, name, attr, fn):
    monkeypatch.setattr(signs, attr, fn)
    with np.errstate(all="ignore"):
        assert _battery(), f"mutant {name} passed every pin"
