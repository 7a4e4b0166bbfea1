"""Pins for I, I^dag, J, J^dag (Sec. 2.1): explicit DFT sums on tiny boxes,
round trip and adjointness."""
import numpy as np
import pytest

from oracle import basis, transforms as T


def _cell():
    return np.array([[5.0, 0.6, 0.2], [0.0, 5.5, -0.4], [0.3, 0.0, 4.8]])


@pytest.mark.parametrize("S", [(5, 6, 4), (7, 5, 6)])
def test_I_and_Idag_equal_explicit_sums(S):
    R = _cell()
    b = basis.gsphere(R, S, np.array([0.5, 0.0, 0.25]), 1.6)
    assert b.npw > 5
    rng = np.random.default_rng(3)
    C = rng.standard_normal(b.npw) + 1j * rng.standard_normal(b.npw)
    B = basis.reciprocal_basis(R)
    G = b.n @ B.T
    # grid points r_j = R (j/S)
    j = np.stack(np.meshgrid(*[np.arange(s) for s in S], indexing="ij"), -1).reshape(-1, 3)
    r = (j / np.array(S)) @ R.T
    phase = np.exp(1j * (r @ G.T))                 # (N, npw)
    IC = phase @ C
    assert np.allclose(T.I(C, b).reshape(-1), IC, atol=1e-12, rtol=0)
    X = rng.standard_normal(S) + 1j * rng.standard_normal(S)
    IdX = phase.conj().T @ X.reshape(-1)
    assert np.allclose(T.Idag(X, b), IdX, atol=1e-12, rtol=0)


def test_round_trip_and_adjoint():
    R = _cell()
    S = (8, 9, 10)
    b = basis.gsphere(R, S, np.zeros(3), 2.5)
    rng = np.random.default_rng(5)
    C = rng.standard_normal((b.npw, 3)) + 1j * rng.standard_normal((b.npw, 3))
    X = rng.standard_normal((3,) + S) + 1j * rng.standard_normal((3,) + S)
    # I^dag I = N on the sphere
    assert np.allclose(T.Idag(T.I(C, b), b), b.N * C, rtol=1e-13, atol=1e-10)
    # <I a, X> = <a, I^dag X>
    lhs = np.vdot(T.I(C, b), X)
    rhs = np.vdot(C, T.Idag(X, b))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # J I = 1 on full-box fields, and J^dag is the adjoint of J
    y = rng.standard_normal(S) + 1j * rng.standard_normal(S)
    assert np.allclose(T.J(T.I_full(y)), y, atol=1e-13)
    x = rng.standard_normal(S) + 1j * rng.standard_normal(S)
    assert abs(np.vdot(T.J(x), y) - np.vdot(x, T.Jdag(y))) < 1e-12 * abs(np.vdot(x, T.Jdag(y)))


def test_full_box_explicit():
    R = _cell()
    S = (4, 5, 3)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(S)
    f = basis.box_frequencies(S).reshape(-1, 3)
    j = np.stack(np.meshgrid(*[np.arange(s) for s in S], indexing="ij"), -1).reshape(-1, 3)
    # J x (G) = (1/N) sum_j x_j exp(-2 pi i m.j/S); the frequency map does not change the phase
    ph = np.exp(-2j * np.pi * (j / np.array(S)) @ f.T)
    assert np.allclose(T.J(x).reshape(-1), ph.T @ x.reshape(-1) / x.size, atol=1e-14)
