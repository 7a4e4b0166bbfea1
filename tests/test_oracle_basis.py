"""Pins for the oracle G-sphere (Sec. 2.1, GridInfo): brute-force counts and order."""
import itertools

import numpy as np
import pytest

from oracle import basis
from tests._golden import rows


def brute_count(L, ecut, k, nmax):
    # independent enumeration: cubic cell, |k+G|^2 = (2 pi / L)^2 |n + k|^2
    g = 2.0 * np.pi / L
    cnt = 0
    rng = range(-nmax, nmax + 1)
    for n0 in rng:
        a = (n0 + k[0]) ** 2
        for n1 in rng:
            b = a + (n1 + k[1]) ** 2
            for n2 in rng:
                q2 = g * g * (b + (n2 + k[2]) ** 2)
                if 0.5 * q2 <= ecut:
                    cnt += 1
    return cnt


@pytest.mark.parametrize("row", rows("gsphere_counts.txt"))
def test_counts_match_golden_and_brute_force(row):
    name, L, ecut, k0, k1, k2, count = row
    L, ecut, k = float(L), float(ecut), np.array([float(k0), float(k1), float(k2)])
    S = (96, 96, 96)
    b = basis.gsphere(np.eye(3) * L, S, k, ecut)
    assert b.npw == int(count)
    if b.npw < 5000:
        assert brute_count(L, ecut, k, 20) == int(count)


def test_canonical_order_and_index():
    R = np.array([[7.0, 0.8, 0.0], [0.3, 6.5, 0.4], [0.0, 0.5, 8.0]])
    S = (15, 16, 18)
    b = basis.gsphere(R, S, np.array([0.25, -0.5, 0.1]), 4.0)
    n = b.n
    # lexicographic ascending
    keys = [tuple(r) for r in n]
    assert keys == sorted(keys)
    assert len(set(keys)) == len(keys)
    # index is the wrapped box position
    for r, idx in zip(n[:50], b.index[:50]):
        i = [r[d] % S[d] for d in range(3)]
        assert idx == (i[0] * S[1] + i[1]) * S[2] + i[2]
    assert len(set(b.index.tolist())) == b.npw
    # every point of a brute-force enumeration in a big range is present
    B = 2 * np.pi * np.linalg.inv(R).T
    cnt = 0
    for m in itertools.product(range(-8, 9), repeat=3):
        v = B @ (np.array(m) + b.k)
        if 0.5 * v @ v <= 4.0:
            cnt += 1
    assert cnt == b.npw
    assert np.allclose(b.kG2, np.sum(((n + b.k) @ B.T) ** 2, axis=1))


def test_box_too_small_raises():
    with pytest.raises(ValueError):
        basis.gsphere(np.eye(3) * 10.0, (8, 8, 8), np.zeros(3), 8.0)


def test_box_frequency_map():
    f = basis.box_frequencies((4, 5, 6))
    assert list(f[:, 0, 0, 0]) == [0, 1, -2, -1]
    assert list(f[0, :, 0, 1]) == [0, 1, 2, -2, -1]
    assert list(f[0, 0, :, 2]) == [0, 1, 2, -3, -2, -1]
