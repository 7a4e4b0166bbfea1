"""Pins for H, orthonormalization and protocol B: dense diagonalization at a
tiny cutoff, free-electron eigenvalues, Cholesky properties."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import basis, energy, minimize, operators as ops


def _tiny_system(R=None, fold=(1, 1, 1), Z=(1, 4), ecut=2.0, S=(16, 16, 16), L=7.0):
    cell = W.tiny_cell(nat=2, L=L, ecut=ecut, S=S, nb=4, Z=Z, fold=fold, R=R)
    return cell, energy.build_system(cell)


def test_apply_H_equals_dense_matrix():
    R = np.array([[7.0, 0.5, 0.0], [0.0, 6.6, 0.7], [0.4, 0.0, 7.3]])
    cell, sys = _tiny_system(R=R, fold=(2, 1, 1))
    Veff = sys.Vloc + W.random_potential(11, cell.S, 0.3)
    rng = np.random.default_rng(2)
    for k, b in enumerate(sys.bases):
        H = ops.dense_hamiltonian(b, Veff, sys.P[k], sys.D)
        C = rng.standard_normal((b.npw, 3)) + 1j * rng.standard_normal((b.npw, 3))
        HC = ops.apply_H(C, b, Veff, sys.P[k], sys.D)
        assert np.max(np.abs(HC - H @ C)) < 1e-11 * np.max(np.abs(H))
        assert np.max(np.abs(H - H.conj().T)) < 1e-12 * np.max(np.abs(H))


def test_free_electron_eigenvalues():
    # V_eff = 0, no projectors: eigenvalues are the smallest |k+G|^2/2 exactly
    cell = W.tiny_cell(nat=2, L=6.0, ecut=3.0, S=(12, 12, 12), nb=4, fold=(2, 2, 2))
    sys = energy.build_system(cell, with_local=False, with_projectors=False)
    rng = np.random.default_rng(4)
    for k, b in enumerate(sys.bases[:3]):
        nb = 4
        Y = rng.standard_normal((b.npw, nb)) + 1j * rng.standard_normal((b.npw, nb))
        cg = minimize.protocol_B(Y, b, np.zeros(cell.S), None, 0.0, 60)
        psi, _, _ = ops.cholesky_orthonormalize(cg.Y[0], b)
        Hs = psi.conj().T @ ops.apply_H(psi, b, np.zeros(cell.S), None, 0.0)
        eig = np.linalg.eigvalsh(0.5 * (Hs + Hs.conj().T))
        exact = np.sort(0.5 * b.kG2)[:nb]
        assert np.max(np.abs(eig - exact)) < 1e-10


def test_protocol_B_matches_dense_diagonalization():
    cell, sys = _tiny_system(fold=(1, 1, 2))
    Veff = sys.Vloc + 0.2 * np.cos(np.linspace(0, 6.28, cell.S[0]))[:, None, None] * np.ones(cell.S)
    rng = np.random.default_rng(8)
    for k, b in enumerate(sys.bases):
        H = ops.dense_hamiltonian(b, Veff, sys.P[k], sys.D)
        exact = scipy.linalg.eigh(H, b.omega * np.eye(b.npw), eigvals_only=True)[:4]
        Y = rng.standard_normal((b.npw, 4)) + 1j * rng.standard_normal((b.npw, 4))
        cg = minimize.protocol_B(Y, b, Veff, sys.P[k], sys.D, 200)
        psi, _, _ = ops.cholesky_orthonormalize(cg.Y[0], b)
        Hs = psi.conj().T @ ops.apply_H(psi, b, Veff, sys.P[k], sys.D)
        eig = np.linalg.eigvalsh(0.5 * (Hs + Hs.conj().T))
        assert np.max(np.abs(eig - exact)) < 1e-9
        # band energy is the sum of the lowest eigenvalues
        assert abs(cg.E - exact.sum()) < 1e-9


def test_cholesky_orthonormalization_properties():
    R = np.array([[6.0, 0.3, 0.0], [0.0, 6.2, 0.0], [0.1, 0.0, 5.9]])
    b = basis.gsphere(R, (12, 12, 12), np.array([0.5, 0.5, 0.0]), 3.0)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((b.npw, 5)) + 1j * rng.standard_normal((b.npw, 5))
    psi, Rm, Rinv = ops.cholesky_orthonormalize(Y, b)
    assert np.max(np.abs(psi.conj().T @ (b.omega * psi) - np.eye(5))) < 1e-12
    assert np.allclose(np.tril(Rm, -1), 0)
    assert np.all(np.real(np.diag(Rm)) > 0) and np.allclose(np.imag(np.diag(Rm)), 0)
    U = b.omega * Y.conj().T @ Y
    assert np.max(np.abs(Rm.conj().T @ Rm - U)) < 1e-12 * np.max(np.abs(U))
    # span(psi) = span(Y)
    Q, _ = np.linalg.qr(Y)
    assert np.max(np.abs(psi - Q @ (Q.conj().T @ psi))) < 1e-12
    # a rank-deficient block is rejected
    Yd = Y.copy()
    Yd[:, 2] = Yd[:, 1]
    with pytest.raises(np.linalg.LinAlgError):
        ops.cholesky_orthonormalize(Yd, b)


def test_density_integrates_to_electron_count():
    cell, sys = _tiny_system(fold=(2, 1, 1))
    rng = np.random.default_rng(3)
    psis = []
    for b in sys.bases:
        Y = rng.standard_normal((b.npw, 3)) + 1j * rng.standard_normal((b.npw, 3))
        psis.append(ops.cholesky_orthonormalize(Y, b)[0])
    fills = [np.array([2.0, 2.0, 1.0])] * 2
    n = energy.density(psis, fills, sys)
    assert abs(sys.omega / sys.N * n.sum() - 5.0) < 1e-12
    assert n.min() >= 0
